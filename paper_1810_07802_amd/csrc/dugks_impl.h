// Internal types shared by the kernels and the C-ABI layer of libdugks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dugks {

// Interior columns per strip: a strip is one 64-lane wave whose lanes 0 and
// 63 hold the halo columns on either side.
constexpr int kStripCols = 62;
constexpr int kWave = 64;

// Values held per cell, in this order:
//   f0..f8, [g0..g8], hist_x, hist_y, phi
// where hist = (phi u) of the previous step and phi = sum_q f.
__host__ __device__ constexpr int val_f(int q) { return q; }
__host__ __device__ constexpr int val_g(int q) { return 9 + q; }
__host__ __device__ constexpr int val_hist(bool coupled, int c) { return (coupled ? 18 : 9) + c; }
__host__ __device__ constexpr int val_phi(bool coupled) { return coupled ? 20 : 11; }
__host__ __device__ constexpr int num_values(bool coupled) { return coupled ? 21 : 12; }
// Values stored in groups (all but phi).
__host__ __device__ constexpr int num_grouped(bool coupled) { return num_values(coupled) - 1; }

// Layout of one state buffer, row-blocked: grid row j holds, one after the
// other, the grouped values of its nx cells and then their phi. The grouped
// values are split into groups of four consecutive values, each stored
// cell-interleaved ([nx][4], so that one 16-byte access per cell moves a
// group; a last partial group of w values is [nx][w]): group g starts 4 g nx
// values into the row and phi num_grouped nx values into it. Rows are padded
// to a multiple of 128 bytes. A wave that reads or writes one row of a strip
// touches one contiguous block of the buffer rather than one block per value
// plane, which streams faster from HBM.
__host__ __device__ constexpr long long state_row_values(int nx, bool coupled, int elem_bytes) {
  return ((long long)num_values(coupled) * nx * elem_bytes + 127) / 128 * 128 / elem_bytes;
}
// Index (in values) of value v of cell (i, j); rv = state_row_values().
__host__ __device__ constexpr long long state_index(int v, int i, int j, int nx, long long rv,
                                                    bool coupled) {
  return (long long)j * rv +
         (v == num_grouped(coupled)
              ? (long long)num_grouped(coupled) * nx + i
              : 4LL * (v >> 2) * nx +
                    (long long)i * (num_grouped(coupled) - 4 * (v >> 2) < 4
                                        ? num_grouped(coupled) - 4 * (v >> 2)
                                        : 4) +
                    (v & 3));
}

// Everything a kernel needs about one case. Lives in device memory (an array
// for batches, one entry for a plain handle). Constants are kept in double;
// kernels narrow them to their working precision.
struct CaseDev {
  // geometry and work decomposition
  int nx, ny;
  int nstrips;   // ceil(nx / kStripCols)
  int seg_rows;  // rows per segment
  int nsegs;     // ceil(ny / seg_rows)
  int walls;     // 1: no-slip walls on y = 0 and y = ny
  int coupled;
  int vel_kind, visc_mode, grav_form;
  int cur0;              // state buffer holding local step 0
  long long step0;       // global step index of local step 0
  long long nsteps;      // local steps allowed (active window)
  long long row_vals;    // values per row of a state buffer (state_row_values())
  void* set[2];          // the two state buffers
  // time
  double dt, h, t0;
  // phase field
  double phi_H, phi_L, phibar, inv_dphi, kappa, beta, theta_c;
  double eps_n2;  // regularisation of the unit normal: (eps_n |phi_H - phi_L| / delta_l)^2
  double rho_H, rho_L, drho;
  // density subtracted in the gravity force: the mean density (buoyancy
  // form) or 0 (rho g form), so that both forms are one expression
  double rho_ref;
  double tau_f;
  // viscosity
  double tau_g_uniform;  // used when visc_mode == uniform nu
  double mu_H, mu_L, inv_mu_H, inv_mu_L;
  // forcing
  double gx, gy, Gx, Gy;
  // prescribed velocity
  double U0, L0, T_period;
  // equilibrium weights of the relaxation: cell (Eq. 29) 3h/(2tau+dt), face
  // (Eq. 28) h/(2tau+h); for f, and for g when tau_g is uniform
  double fb, ffb, gb, gfb;
  // stretched mesh (nullptr: unit cells): per axis, x then y, kMeshArrays
  // arrays of the axis length (layout in mesh_axis()); meshf holds the same
  // arrays rounded to float, read by the FP32 kernels
  const double* mesh;
  const float* meshf;
  // the constants the FP32 kernels use, rounded to float on the host (they
  // then load into scalar registers instead of being converted into vector
  // ones); hdt = dt / 2, beta4 = 4 beta
  struct F32 {
    float h, dt, hdt, phi_L, phi_H, phibar, drho, gx, gy, Gx, Gy, theta_c, tau_f, kappa, beta4, ffb,
        fb, eps_n2;
  } f32;
  // non-finite flag of the case (device word): a step that produces a
  // non-finite phi, phi u or p in one of its cells stores 1 there; the host
  // clears it at initialisation and reads it after synchronising
  int* flag;
};

// The float copies of a case's constants (CaseDev::f32), rounded to nearest
// from the double fields: the host fills them once, and kernels that keep
// their constants in vector registers form them the same way at their start.
__host__ __device__ inline CaseDev::F32 narrow_constants(const CaseDev& C) {
  return CaseDev::F32{float(C.h),     float(C.dt),     float(0.5 * C.dt),   float(C.phi_L),
                      float(C.phi_H), float(C.phibar), float(C.drho),       float(C.gx),
                      float(C.gy),    float(C.Gx),     float(C.Gy),         float(C.theta_c),
                      float(C.tau_f), float(C.kappa),  float(4.0 * C.beta), float(C.ffb),
                      float(C.fb),    float(C.eps_n2)};
}

// Metric arrays of one axis of a stretched mesh, each of the axis length,
// in this order: the width w, the distances hm and hp to the previous and
// next centres, the centre c, and what the stencils derive from them (once,
// on the host, in double): 1/w, 1/hm, 1/hp; the weights of the parabola
// derivatives through three centres, d1 = cp (a+ - a) + cm (a - a-) and
// d2 = ep (a+ - a) - em (a - a-), with cp = hm / (hp (hm + hp)),
// cm = hp / (hm (hm + hp)), ep = 2 / (hp (hm + hp)), em = 2 / (hm (hm + hp));
// and the interpolation weights of the next and previous centres at the
// cell centre's mirror point, wp = hm / (hm + hp), wm = hp / (hm + hp).
constexpr int kMeshArrays = 13;
template <typename S>
struct MeshAxisT {
  const S *w, *hm, *hp, *c, *iw, *ihm, *ihp, *cp, *cm, *ep, *em, *wp, *wm;
};
using MeshAxis = MeshAxisT<double>;
template <typename S>
__host__ __device__ inline MeshAxisT<S> mesh_axis(const S* mesh, int nx, int ny, int axis) {
  const S* b = mesh + (axis == 0 ? 0 : kMeshArrays * (long long)nx);
  const long long n = axis == 0 ? nx : ny;
  return MeshAxisT<S>{b,         b + n,     b + 2 * n, b + 3 * n,  b + 4 * n,  b + 5 * n, b + 6 * n,
                      b + 7 * n, b + 8 * n, b + 9 * n, b + 10 * n, b + 11 * n, b + 12 * n};
}

enum VelKind { kVelUniform = 0, kVelRotation = 1, kVelShear = 2, kVelDeform = 3 };
enum ViscMode { kViscUniformNu = 0, kViscReciprocal = 1, kViscLinear = 2 };

// Work item of the step kernel: which case, which column strip, which row
// segment, and the direction the march of a multi-row segment takes (0 up,
// 1 down; see item_dir()).
struct Item {
  int c, strip, seg, dir;
};
// Alternate segments of a periodic case march in opposite directions; wall
// cases march upwards (the step kernel with walls has no downward march).
__host__ __device__ constexpr int item_dir(int seg, bool walls) { return walls ? 0 : (seg & 1); }

// Launch arguments of the step kernel.
struct StepArgs {
  const CaseDev* cases;
  const Item* items;
  int nitems;
  int kofs;                    // offset of this launch inside a step sequence
  const long long* step_base;  // device counter: global step of kofs = 0
  int one_row;                 // every item is one row (seg_rows == 1): row kernel
  int two_row;                 // every item is two rows (seg_rows == 2): the two-row kernel
                               // for periodic FP32 cases, else the march
  int upm_rows;                // rows per segment of the reconstruction march
};

// The reconstruction march (upwind reconstruction, or a stretched mesh):
// strips of kUpmCols columns (a 64-lane wave with two halo lanes on each
// side); segments of StepArgs::upm_rows rows.
constexpr int kUpmCols = 60;

// slot of population q among the six crossing an x-face / a y-face (-1: none)
__host__ __device__ constexpr int up_xslot(int q) {
  return q == 1 ? 0 : q == 2 ? 1 : q == 8 ? 2 : q == 4 ? 3 : q == 5 ? 4 : q == 6 ? 5 : -1;
}
__host__ __device__ constexpr int up_yslot(int q) {
  return q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 2 : q == 6 ? 3 : q == 7 ? 4 : q == 8 ? 5 : -1;
}

// host-side launchers (dugks_kernels.hip)
hipError_t launch_step(bool fp64, bool coupled, bool walls, const StepArgs& a, hipStream_t s);
// the reconstruction march (upwind reconstruction on the unit or a stretched
// mesh, central reconstruction on a stretched mesh; items of kUpmCols-column strips
// and a.upm_rows-row segments) and its resident waves per CU
hipError_t launch_step_upm(bool fp64, bool coupled, bool walls, bool mesh, bool central,
                           const StepArgs& a, hipStream_t s);
int upm_waves_per_cu(bool fp64, bool coupled, bool walls, bool mesh, bool central);
int step_waves_per_cu(bool fp64, bool coupled, bool walls);
hipError_t launch_advance(long long* step_base, long long by, hipStream_t s);
// step_base[0] = value (if not null) and flag[0] = 0 (if not null)
hipError_t launch_reset(long long* step_base, long long value, int* flag, hipStream_t s);
hipError_t launch_init(bool fp64, const CaseDev* dcase, const CaseDev& hcase,
                       const double* phi, const double* u, const double* v,
                       const double* p, hipStream_t s);
hipError_t launch_macros(bool fp64, const CaseDev* dcase, const CaseDev& hcase,
                         long long local_step, double* phi, double* u,
                         double* v, double* p, double* rho, hipStream_t s);
// Diagnostics without device allocation: the device address of the
// library's file-scope partial-sum array on the current device (looked up
// once per device) and its capacity in grid rows; the fused macros and
// reduction kernels writing the seven diagnostics to out (device).
hipError_t noalloc_scratch(double** ptr, int* max_rows);
hipError_t launch_diag_noalloc(bool fp64, const CaseDev* dcase, const CaseDev& hcase,
                               long long local_step, double* part, double* out, hipStream_t s);
hipError_t launch_diag(const CaseDev& hcase, const double* phi, const double* u,
                       const double* v, const double* rho, double* partial,
                       int npartial, double* out, hipStream_t s);

}  // namespace dugks
