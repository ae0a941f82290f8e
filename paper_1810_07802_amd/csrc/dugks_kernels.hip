// HIP kernels of the phase-field DUGKS step for gfx950 (MI355X).
//
// Paper: Yang, Zhong & Zhuo, arXiv:1810.07802. Section and equation numbers
// below refer to it.
//
// Step kernel layout. One 64-lane wave owns a strip of 62 interior columns
// (lanes 1..62; lanes 0 and 63 carry the halo columns) and a segment of rows,
// and marches up the rows. For each new row r it runs the cell stage (macros
// at t_n, equilibria and sources, bar-plus and tilde-plus, Eqs. 15-19, 29-33)
// once; the three most recent rows stay in registers, so every cell stage is
// done once per segment except two halo rows. The x-neighbours' values needed
// by the face reconstruction come through cross-lane permutes, not memory.
// Faces are reconstructed from the bar-plus values of the adjacent cells
// (central scheme: mean, normal difference, mean of the tangential central
// differences, Eq. 27), including the face moments used for the face macros,
// which are linear in the populations and therefore reconstructed from the
// cell moments. The face distributions (Eq. 28) give the microflux (Eq. 22)
// and the cell update (Eq. 24) is written together with phi = sum f and the
// history (phi u) for the next step's time derivative.
//
// Working precision T is float or double. In the float path the density,
// its reciprocal and the relaxation time of g (interpolated across the
// interface) are evaluated in double and narrowed.
//
// The upwind, limited reconstruction and stretched tensor-product meshes run
// as a second march (k_upm; see the section "the reconstruction march"
// below), which shares the cell-stage, face and wall-face arithmetic with
// k_step.

#include <hip/hip_runtime.h>

#include <mutex>

#include "dugks_impl.h"

namespace dugks {
namespace {

__device__ constexpr int EX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};

// D2Q9 weights (Eq. 14). In float the nine stored weights are chosen within
// one ulp of 4/9, 1/9, 1/36 so that they sum to exactly 1 (w1 = 4 w2 and
// w0 = 1 - 4 w1 - 4 w2 are exact); with the rounded weights the zeroth moment
// of every equilibrium would carry a 7e-9 bias per step into sum phi.
// A case constant in the kernel's precision: its float copy (rounded on
// the host) in FP32 kernels, the double field in FP64 ones.
template <typename T>
__device__ __forceinline__ T ck(float f, double d);
template <>
__device__ __forceinline__ float ck<float>(float f, double) { return f; }
template <>
__device__ __forceinline__ double ck<double>(float, double d) { return d; }

// The phase-field terms of a cell: dA = phi - phi_H, dB = phi - phi_L, the
// chemical potential (Eq. 4) and theta (Eq. 6).
template <typename T>
__device__ __forceinline__ void phase_terms(const CaseDev& C, T phi, T lap, T& dA, T& dB, T& mu,
                                            T& theta) {
  const T b4 = ck<T>(C.f32.beta4, 4.0 * C.beta), pbar = ck<T>(C.f32.phibar, C.phibar);
  const T kap = ck<T>(C.f32.kappa, C.kappa), thc = ck<T>(C.f32.theta_c, C.theta_c);
  dA = phi - ck<T>(C.f32.phi_H, C.phi_H);
  dB = phi - ck<T>(C.f32.phi_L, C.phi_L);
  mu = b4 * dA * dB * (phi - pbar) - kap * lap;
  theta = thc * dA * dB;
}
// theta (Eq. 6) of a face or wall value of phi
template <typename T>
__device__ __forceinline__ T theta_of(const CaseDev& C, T phi) {
  const T thc = ck<T>(C.f32.theta_c, C.theta_c);
  return thc * (phi - ck<T>(C.f32.phi_H, C.phi_H)) * (phi - ck<T>(C.f32.phi_L, C.phi_L));
}

// Kernels whose vector registers are not the limit narrow the constants
// themselves (vector conversions at the kernel's start) instead of taking
// the float copies into scalar registers: measured faster where scalar
// registers are the scarcer ones (the periodic unit-mesh kernels). The
// copies pay off where vector registers would otherwise spill: the
// stretched-mesh marches and the marches with walls, whose spill reloads
// inside the loop wait for the prefetched rows.
__device__ __forceinline__ void narrow_in_kernel(CaseDev& C) { C.f32 = narrow_constants(C); }

template <typename T>
__device__ __forceinline__ constexpr T wq(int q);
template <>
__device__ __forceinline__ constexpr float wq<float>(int q) {
  return q == 0 ? 0x1.c71c74p-2f : ((q & 1) ? 0x1.c71c70p-4f : 0x1.c71c70p-6f);
}
template <>
__device__ __forceinline__ constexpr double wq<double>(int q) {
  return q == 0 ? 4.0 / 9.0 : ((q & 1) ? 1.0 / 9.0 : 1.0 / 36.0);
}

__device__ __forceinline__ int wrap(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

// Row index of a (possibly ghost) row: periodic wrap, or mirror about the
// walls (neutral wetting ghost values for the phi stencils).
__device__ __forceinline__ int row_of(int r, int ny, int walls) {
  if (walls) {
    if (r < 0) r = -1 - r;
    if (r >= ny) r = 2 * ny - 1 - r;
    return r;
  }
  return wrap(r, ny);
}

// Cross-lane moves inside the wave: value of lane l-1 / l+1 (wrapping; the
// wrapped values only reach the halo lanes, whose results are discarded).
// Neighbour lanes by DPP wavefront rotates, fused into the consuming ALU
// instruction where the encoding allows: right = lane + 1 (wave_rol:1), left
// = lane - 1 (wave_ror:1), both wrapping around the 64 lanes (every lane
// receives a value, so no lane keeps an old one).
template <int CTRL>
__device__ __forceinline__ float rot(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double rot(double v) {
  int2 w = *reinterpret_cast<int2*>(&v);
  w.x = __builtin_amdgcn_mov_dpp(w.x, CTRL, 0xF, 0xF, true);
  w.y = __builtin_amdgcn_mov_dpp(w.y, CTRL, 0xF, 0xF, true);
  return *reinterpret_cast<double*>(&w);
}
template <typename T>
__device__ __forceinline__ T nbr_r(T v) { return rot<0x134>(v); }  // value of lane + 1
template <typename T>
__device__ __forceinline__ T nbr_l(T v) { return rot<0x13C>(v); }  // value of lane - 1
// The same moves through the LDS unit's crossbar (ds_bpermute) where BP is
// set (FP32): they take no VALU issue slot, at the LDS unit's latency. That
// pays in the central march of the coupled model, whose issue is nearly
// full. The interface-only march has far less arithmetic to hide the
// latency behind, the reconstruction marches keep metrics in LDS and the
// small-grid kernels are latency-bound: there the DPP moves are faster.
template <bool BP, typename T>
__device__ __forceinline__ T xr(T v) {  // value of lane + 1
  if constexpr (BP && sizeof(T) == 4) {
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane + 1) & 63) << 2, __float_as_int(v)));
  } else {
    return nbr_r(v);
  }
}
template <bool BP, typename T>
__device__ __forceinline__ T xl(T v) {  // value of lane - 1
  if constexpr (BP && sizeof(T) == 4) {
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane + 63) & 63) << 2, __float_as_int(v)));
  } else {
    return nbr_l(v);
  }
}

__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// 1/r in double, for a positive r well inside the float range (a density,
// a relaxation denominator). The float path refines a float reciprocal with
// one Newton-Raphson step (relative error ~1e-14, far below what it is
// narrowed to), a third of the instructions of a correctly rounded double
// divide; the double path divides.
template <typename T>
__device__ __forceinline__ double inv_rho(double r);
template <>
__device__ __forceinline__ double inv_rho<float>(double r) {
  double y = (double)__builtin_amdgcn_rcpf((float)r);
  return y * (2.0 - r * y);
}
template <>
__device__ __forceinline__ double inv_rho<double>(double r) {
  return 1.0 / r;
}
// a / r with the reciprocal above
template <typename T>
__device__ __forceinline__ double div_pos(double a, double r) {
  if constexpr (sizeof(T) == 4) return a * inv_rho<float>(r);
  else return a / r;
}

// Density (Eq. 10) with s clamped to [0,1], in double.
__device__ __forceinline__ double rho_of(const CaseDev& C, double phi) {
  double s = (phi - C.phi_L) * C.inv_dphi;
  s = fmin(fmax(s, 0.0), 1.0);
  return C.rho_L + (C.rho_H - C.rho_L) * s;
}

// Relaxation of g for a local tau_g (Eqs. 34-36), in double. Returns the
// equilibrium weight b and tau: cell (Eq. 29) b = 3h/(2tau+dt), face (Eq. 28)
// b = h/(2tau+h); the source weight is tau b in both, and the weight of the
// distribution itself is 1 - b, which the kernels use in the increment form
// psi + b (psi^eq + tau S - psi). The FP32 kernels divide with div_pos.
template <typename T, bool FACE>
__device__ __forceinline__ void g_relax(const CaseDev& C, double phi, double rho,
                                        double& b, double& tau) {
  if (C.visc_mode == kViscUniformNu) {
    tau = C.tau_g_uniform;
    b = FACE ? C.gfb : C.gb;
    return;
  }
  double s = (phi - C.phi_L) * C.inv_dphi;
  s = fmin(fmax(s, 0.0), 1.0);
  double mu = (C.visc_mode == kViscReciprocal)
                  ? inv_rho<T>(s * C.inv_mu_H + (1.0 - s) * C.inv_mu_L)
                  : s * C.mu_H + (1.0 - s) * C.mu_L;
  tau = div_pos<T>(3.0 * mu, rho);
  b = FACE ? div_pos<T>(C.h, 2.0 * tau + C.h) : div_pos<T>(3.0 * C.h, 2.0 * tau + C.dt);
}

// Unit normal n = grad phi / sqrt(|grad phi|^2 + eps^2): zero for a uniform
// field, the plain unit vector wherever |grad phi| >> eps (eps = 0: the plain
// unit vector, and 0 where the gradient is exactly 0).
template <typename T>
__device__ __forceinline__ void normal(const CaseDev& C, T gx, T gy, T& nx, T& ny) {
  const T m2 = gx * gx + gy * gy + ck<T>(C.f32.eps_n2, C.eps_n2);
  const T inv = m2 > T(0) ? rsqrt_t(m2) : T(0);
  nx = gx * inv;
  ny = gy * inv;
}

// Prescribed velocity of the interface-only tests (Eqs. 40-43).
template <typename T>
__device__ __forceinline__ void presc_vel(const CaseDev& C, double x, double y,
                                          double t, T& u, T& v) {
  const double pi = 3.14159265358979323846;
  double U0 = C.U0, L0 = C.L0;
  switch (C.vel_kind) {
    case kVelUniform: u = T(U0); v = T(U0); break;
    case kVelRotation:
      u = T(-U0 * pi / L0 * (y - 0.5 * L0));
      v = T(U0 * pi / L0 * (x - 0.5 * L0));
      break;
    case kVelShear: {
      double sg = (t < 0.5 * C.T_period) ? 1.0 : -1.0;
      u = T(sg * U0 * pi * sin(pi * x / L0) * cos(pi * y / L0));
      v = T(-sg * U0 * pi * cos(pi * x / L0) * sin(pi * y / L0));
      break;
    }
    default: {
      double c = cos(pi * t / C.T_period);
      u = T(-U0 * sin(4.0 * pi * x / L0) * sin(4.0 * pi * y / L0) * c);
      v = T(-U0 * cos(4.0 * pi * x / L0) * cos(4.0 * pi * y / L0) * c);
    }
  }
}

// ------------------------------------------- equilibria + sources, by pairs

// For the g model the relaxation needs g^eq_q + tau S^g_q (Eqs. 17-19). For a
// direction q and its opposite -q, e = xi.u, a = xi.grad rho and b = xi.F
// change sign, so Gamma_q(u)/w_q - 1 = E2 +- 3e with E2 = 4.5 e^2 - 1.5 |u|^2,
// and g^eq + tau S^g = w (Qe +- Qo) with
//   Qe = 3p + rho E2 + tau [3ae - a0 E2 + 3 (3be - b0 (1 + E2))]
//   Qo = 3 rho e + tau [a E2 - 3 a0 e + 3 (b (1 + E2) - 3 b0 e)]
// (a0 = u.grad rho, b0 = u.F): one evaluation serves both directions.
// With G = grad rho + 3F, A = xi.G and A0 = u.G the brackets regroup into
//   Qe = (3p - 3 tau b0) + E2 (rho - tau A0) + 3 tau e A
//   Qo = 3e (rho - tau A0) + tau (E2 A + 3b)
// whose point terms (in parentheses) are shared by all pairs.
template <typename T>
struct GTerms {
  T u, v, m15uu;  // velocity and -1.5 |u|^2
  T Gx, Gy;       // grad rho + 3F
  T F3x, F3y;     // 3F
  T Pp;           // 3p - 3 tau b0
  T Rp, Rp3;      // rho - tau A0 and three times it
  T tau, tau3;
};
template <typename T>
__device__ __forceinline__ GTerms<T> g_terms(T u, T v, T uu, T p, T rho, T tau, T drx, T dry,
                                             T Fx, T Fy) {
  GTerms<T> s;
  s.u = u;
  s.v = v;
  s.m15uu = T(-1.5) * uu;
  s.F3x = T(3) * Fx;
  s.F3y = T(3) * Fy;
  s.Gx = drx + s.F3x;
  s.Gy = dry + s.F3y;
  s.tau = tau;
  s.tau3 = T(3) * tau;
  s.Pp = T(3) * p - s.tau3 * (u * Fx + v * Fy);
  s.Rp = rho - tau * (u * s.Gx + v * s.Gy);
  s.Rp3 = T(3) * s.Rp;
  return s;
}
template <typename T>
__device__ __forceinline__ void g_pair(const GTerms<T>& s, int ex, int ey, T& qe, T& qo) {
  const T e = T(ex) * s.u + T(ey) * s.v;
  const T A = T(ex) * s.Gx + T(ey) * s.Gy;
  const T b3 = T(ex) * s.F3x + T(ey) * s.F3y;
  const T E2 = T(4.5) * e * e + s.m15uu;
  qe = s.Pp + E2 * s.Rp + s.tau3 * e * A;
  qo = e * s.Rp3 + s.tau * (E2 * A + b3);
}
// rest population: e = A = b = 0, and g^eq_0 carries -3p (Eq. 17)
template <typename T>
__device__ __forceinline__ T g_rest(const GTerms<T>& s, T p) {
  return wq<T>(0) * (s.Pp + s.m15uu * s.Rp) - T(3) * p;
}

// ------------------------------------------------------------- cell stage

template <typename T>
struct Cell {
  T fb[9], gb[9];  // bar-plus, Eq. 29
  T gx, gy, mu, Dx, Dy;  // inputs averaged onto faces
  T phi, p;              // for wall faces
  T hx, hy;              // phi u at t_n (history of the next step)
  // moments of bar-plus: f: sum, sum e_x, sum e_y;
  // g: sum over q != 0, sum e_x, sum e_y, sum e_x^2, sum e_x e_y, sum e_y^2
  T M0, Mx, My, N0, Jx, Jy, Pxx, Pxy, Pyy;
};

// Cell macros at t_n (Eqs. 31-33, 4, 6, 10), equilibria and sources
// (Eqs. 15-19), bar-plus (Eq. 29) and tilde-plus (Eq. 30) of a cell with
// order parameter phi, gradient (gx, gy) and Laplacian lap. The tilde-plus
// values go to `tp` (18 values, f then g).
template <typename T, bool CPL>
__device__ __forceinline__ void cell_core(const CaseDev& C, T phi, T gx, T gy, T lap,
                                          const T (&ft)[9], const T (&gt)[9],
                                          T hist_x, T hist_y, double xc, double yc,
                                          double tn, Cell<T>& o, T (&tp)[18]) {
  T dA, dB, mu, theta;  // Eqs. 4, 6
  phase_terms<T>(C, phi, lap, dA, dB, mu, theta);
  T nxv, nyv;
  normal<T>(C, gx, gy, nxv, nyv);
  const T dt = ck<T>(C.f32.dt, C.dt);

  T u, v, p = T(0);
  double rhoD = rho_of(C, (double)phi);
  if (CPL) {
    const T rho = T(rhoD);
    const T irho = T(inv_rho<T>(rhoD));
    const T rg = T(rhoD - C.rho_ref);
    const T Fx = mu * gx + (ck<T>(C.f32.Gx, C.Gx) + rg * ck<T>(C.f32.gx, C.gx));
    const T Fy = mu * gy + (ck<T>(C.f32.Gy, C.Gy) + rg * ck<T>(C.f32.gy, C.gy));
    const T mx = (gt[1] + gt[2] + gt[8]) - (gt[4] + gt[5] + gt[6]);
    const T my = (gt[2] + gt[3] + gt[4]) - (gt[6] + gt[7] + gt[8]);
    const T m0 = ((gt[1] + gt[2]) + (gt[3] + gt[4])) + ((gt[5] + gt[6]) + (gt[7] + gt[8]));
    u = (mx + T(0.5) * dt * Fx) * irho;  // Eq. 32
    v = (my + T(0.5) * dt * Fy) * irho;
    const T drx = ck<T>(C.f32.drho, C.drho) * gx, dry = ck<T>(C.f32.drho, C.drho) * gy;
    const T uu = u * u + v * v;
    p = T(0.6) * m0 + T(0.3) * dt * (u * drx + v * dry) - T(0.4) * rho * uu;  // Eq. 33
    // g: equilibrium (Eq. 17) and source (Eq. 19), bar-plus and tilde-plus
    double gbD, tauD;
    g_relax<T, false>(C, (double)phi, rhoD, gbD, tauD);
    const T gb = T(gbD);
    const GTerms<T> s = g_terms<T>(u, v, uu, p, rho, T(tauD), drx, dry, Fx, Fy);
    // Eq. 29-30 as increments: bar+ = g + b e, tilde+ = g + (4/3) b e with
    // e = g^eq + tau S - g (one multiply-add each)
    const T gb43 = T(4.0 / 3.0) * gb;
    auto relax = [&](int q, T target) {
      const T e = target - gt[q];
      o.gb[q] = gt[q] + gb * e;
      tp[9 + q] = gt[q] + gb43 * e;
    };
    relax(0, g_rest<T>(s, p));
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
      T qe, qo;
      g_pair<T>(s, EX[q], EY[q], qe, qo);
      relax(q, wq<T>(q) * (qe + qo));
      relax(q + 4, wq<T>(q) * (qe - qo));
    }
  } else {
    presc_vel<T>(C, xc, yc, tn, u, v);
  }
  // f: equilibrium (Eq. 15) and source (Eq. 16) with D = d_t(phi u) taken as
  // [(phi u)^n - (phi u)^(n-1)] / dt (zero on the first step)
  const T hx = phi * u, hy = phi * v;
  const T Dx = (hx - hist_x) * T(1.0 / C.dt), Dy = (hy - hist_y) * T(1.0 / C.dt);
  {
    // f^eq + tau_f S^f = w (phi + xi . V) with V = 3 phi u + tau_f (theta n + 3 D)
    const T fbc = ck<T>(C.f32.fb, C.fb), fbc43 = T(4.0 / 3.0 * C.fb), tauf = ck<T>(C.f32.tau_f, C.tau_f);
    const T Vx = T(3) * phi * u + tauf * (theta * nxv + T(3) * Dx);
    const T Vy = T(3) * phi * v + tauf * (theta * nyv + T(3) * Dy);
    auto relax = [&](int q, T target) {
      const T e = target - ft[q];
      o.fb[q] = ft[q] + fbc * e;
      tp[q] = ft[q] + fbc43 * e;
    };
    relax(0, wq<T>(0) * phi);
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
      const T xv = T(EX[q]) * Vx + T(EY[q]) * Vy;
      relax(q, wq<T>(q) * (phi + xv));
      relax(q + 4, wq<T>(q) * (phi - xv));
    }
  }
  o.gx = gx; o.gy = gy; o.mu = mu; o.Dx = Dx; o.Dy = Dy;
  o.phi = phi; o.p = p; o.hx = hx; o.hy = hy;
  // moments of bar-plus
  const T* f = o.fb;
  o.M0 = (f[0] + ((f[1] + f[2]) + (f[3] + f[4]))) + ((f[5] + f[6]) + (f[7] + f[8]));
  o.Mx = (f[1] + f[2] + f[8]) - (f[4] + f[5] + f[6]);
  o.My = (f[2] + f[3] + f[4]) - (f[6] + f[7] + f[8]);
  if (CPL) {
    const T* g = o.gb;
    o.N0 = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    o.Jx = (g[1] + g[2] + g[8]) - (g[4] + g[5] + g[6]);
    o.Jy = (g[2] + g[3] + g[4]) - (g[6] + g[7] + g[8]);
    const T dg = (g[2] + g[4]) + (g[6] + g[8]);
    o.Pxx = (g[1] + g[5]) + dg;
    o.Pyy = (g[3] + g[7]) + dg;
    o.Pxy = (g[2] - g[4]) + (g[6] - g[8]);
  }
}

// The same with the unit-mesh stencils. ph[r][c] is phi on rows (r-1, r,
// r+1) and columns (left, own, right).
template <typename T, bool CPL>
__device__ __forceinline__ void cell_stage(const CaseDev& C, const T (&ph)[3][3],
                                           const T (&ft)[9], const T (&gt)[9],
                                           T hist_x, T hist_y, double xc, double yc,
                                           double tn, Cell<T>& o, T (&tp)[18]) {
  const T c = ph[1][1];
  const T E = ph[1][2], Wv = ph[1][0], N = ph[2][1], S = ph[0][1];
  const T NE = ph[2][2], NW = ph[2][0], SE = ph[0][2], SW = ph[0][0];
  // isotropic D2Q9-weighted gradient (six non-zero points per component) and
  // nine-point Laplacian, the stencils named before Eq. 37
  const T gx = (T(4) * (E - Wv) + (NE - NW) + (SE - SW)) * T(1.0 / 12.0);
  const T gy = (T(4) * (N - S) + (NE - SE) + (NW - SW)) * T(1.0 / 12.0);
  // differences first: near equilibrium mu_phi is a small residual of two
  // O(beta) terms, so the Laplacian must not lose the ulps of phi
  const T lap = T(2.0 / 3.0) * (((E - c) + (Wv - c)) + ((N - c) + (S - c))) +
                T(1.0 / 6.0) * (((NE - c) + (NW - c)) + ((SE - c) + (SW - c)));
  cell_core<T, CPL>(C, c, gx, gy, lap, ft, gt, hist_x, hist_y, xc, yc, tn, o, tp);
}

// ------------------------------------------------------- face distribution

// Face macros (Eqs. 31-33 with dt/2 -> h/2; gradient-type inputs are the mean
// of the two cells, functions of phi are re-evaluated from the face phi) and face original
// distributions (Eq. 28) for the populations crossing a face of normal DIR
// (0: x, 1: y). fbar/gbar hold the reconstructed bar values.
template <typename T, bool CPL, int DIR>
__device__ __forceinline__ void face_df(const CaseDev& C, T phif, T N0f, T Jxf, T Jyf,
                                        T gxf, T gyf, T muf, T Dxf, T Dyf,
                                        const T (&fbar)[9], const T (&gbar)[9],
                                        double xf, double yf, double tf,
                                        T (&fo)[9], T (&go)[9]) {
  const T h = ck<T>(C.f32.h, C.h);
  const T theta = theta_of<T>(C, phif);
  T nxv, nyv;
  normal<T>(C, gxf, gyf, nxv, nyv);
  T u, v;
  if (CPL) {
    const double rhoD = rho_of(C, (double)phif);
    const T rho = T(rhoD), irho = T(inv_rho<T>(rhoD));
    const T rg = T(rhoD - C.rho_ref);
    const T Fx = muf * gxf + (ck<T>(C.f32.Gx, C.Gx) + rg * ck<T>(C.f32.gx, C.gx));
    const T Fy = muf * gyf + (ck<T>(C.f32.Gy, C.Gy) + rg * ck<T>(C.f32.gy, C.gy));
    u = (Jxf + T(0.5) * h * Fx) * irho;
    v = (Jyf + T(0.5) * h * Fy) * irho;
    const T drx = ck<T>(C.f32.drho, C.drho) * gxf, dry = ck<T>(C.f32.drho, C.drho) * gyf;
    const T uu = u * u + v * v;
    const T p = T(0.6) * N0f + T(0.3) * h * (u * drx + v * dry) - T(0.4) * rho * uu;
    double gbD, tauD;
    g_relax<T, true>(C, (double)phif, rhoD, gbD, tauD);
    const T gb = T(gbD);
    const GTerms<T> s = g_terms<T>(u, v, uu, p, rho, T(tauD), drx, dry, Fx, Fy);
    // Eq. 28 in increment form, for the pairs of directions crossing the face
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
      if ((DIR == 0 ? EX[q] : EY[q]) == 0) continue;
      T qe, qo;
      g_pair<T>(s, EX[q], EY[q], qe, qo);
      go[q] = gbar[q] + gb * (wq<T>(q) * (qe + qo) - gbar[q]);
      go[q + 4] = gbar[q + 4] + gb * (wq<T>(q) * (qe - qo) - gbar[q + 4]);
    }
  } else {
    presc_vel<T>(C, xf, yf, tf, u, v);
  }
  const T fbc = ck<T>(C.f32.ffb, C.ffb), tauf = ck<T>(C.f32.tau_f, C.tau_f);
  const T Vx = T(3) * phif * u + tauf * (theta * nxv + T(3) * Dxf);
  const T Vy = T(3) * phif * v + tauf * (theta * nyv + T(3) * Dyf);
#pragma unroll
  for (int q = 1; q <= 4; ++q) {
    if ((DIR == 0 ? EX[q] : EY[q]) == 0) continue;
    const T xv = T(EX[q]) * Vx + T(EY[q]) * Vy;
    fo[q] = fbar[q] + fbc * (wq<T>(q) * (phif + xv) - fbar[q]);
    fo[q + 4] = fbar[q + 4] + fbc * (wq<T>(q) * (phif - xv) - fbar[q + 4]);
  }
}

// No-slip wall on the face below row 0 (BOTTOM) or above row ny-1: face
// bounce-back. Populations leaving the fluid are reconstructed one-sidedly from
// the wall cell, the entering ones take the value of their opposite; u = 0,
// p and phi are the wall cell's, and the normal parts of grad phi and D vanish.
// `c` is the adjacent cell, `cn` the next cell inward, txf/txg the x central
// differences of the adjacent cell's bar-plus values (diagonal populations).
//
// MESH: on a stretched mesh the wall lies dyw_m from the centre, the
// one-sided y difference is divided by the centre distance (times idy), and
// txf/txg hold the x slopes themselves.
template <typename T, bool BOTTOM, bool MESH>
__device__ __forceinline__ void wall_face_g(const CaseDev& C, const Cell<T>& c,
                                            const Cell<T>& cn, const T (&txf)[9],
                                            const T (&txg)[9], T dyw_m, T idy, T (&fo)[9],
                                            T (&go)[9]) {
  const T h = ck<T>(C.f32.h, C.h);
  const T dyw = MESH ? dyw_m : (BOTTOM ? T(-0.5) : T(0.5));
  const T phiw = c.phi;
  const double rhoD = rho_of(C, (double)phiw);
  const T theta = theta_of<T>(C, phiw);
  const T gxw = c.gx;
  T nxv, nyv;
  normal<T>(C, gxw, T(0), nxv, nyv);
  const T rg = T(rhoD - C.rho_ref);
  const T Fx = c.mu * gxw + (ck<T>(C.f32.Gx, C.Gx) + rg * ck<T>(C.f32.gx, C.gx));
  const T Fy = ck<T>(C.f32.Gy, C.Gy) + rg * ck<T>(C.f32.gy, C.gy);
  double gbD, tauD;
  g_relax<T, true>(C, (double)phiw, rhoD, gbD, tauD);
  const T gb = T(gbD), tau = T(tauD);
  const T fbc = ck<T>(C.f32.ffb, C.ffb), tauf = ck<T>(C.f32.tau_f, C.tau_f);
  const T Vx = tauf * (theta * nxv + T(3) * c.Dx);
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    const bool out = BOTTOM ? (EY[q] < 0) : (EY[q] > 0);
    if (!out) continue;
    const T dx = -h * T(EX[q]), dy = dyw - h * T(EY[q]);
    const T sgn = BOTTOM ? T(1) : T(-1);
    T syf = sgn * (cn.fb[q] - c.fb[q]);
    T syg = sgn * (cn.gb[q] - c.gb[q]);
    if (MESH) {
      syf *= idy;
      syg *= idy;
    }
    T fbar = c.fb[q] + dy * syf;
    T gbar = c.gb[q] + dy * syg;
    if (EX[q] != 0) {
      if (MESH) {
        fbar += dx * txf[q];
        gbar += dx * txg[q];
      } else {
        fbar += dx * T(0.5) * txf[q];
        gbar += dx * T(0.5) * txg[q];
      }
    }
    // u = 0: f^eq = w phi, S^f = w e_x (theta n_x + 3 D_x); g^eq = 3 w p,
    // S^g = 3 w (e . F)
    const T fval = fbar + fbc * (wq<T>(q) * (phiw + T(EX[q]) * Vx) - fbar);
    const T bq = T(EX[q]) * Fx + T(EY[q]) * Fy;
    const T gval = gbar + gb * (wq<T>(q) * T(3) * (c.p + tau * bq) - gbar);
    const int qo = ((q + 3) % 8) + 1;  // opposite direction: bounce-back
    fo[q] = fval; go[q] = gval;
    fo[qo] = fval; go[qo] = gval;
  }
}
template <typename T, bool BOTTOM>
__device__ __forceinline__ void wall_face(const CaseDev& C, const Cell<T>& c,
                                          const Cell<T>& cn, const T (&txf)[9],
                                          const T (&txg)[9], T (&fo)[9], T (&go)[9]) {
  wall_face_g<T, BOTTOM, false>(C, c, cn, txf, txg, T(0), T(1), fo, go);
}

// ----------------------------------------------------------- step kernel

// Global-memory access through a uniform base pointer (SGPRs) plus a 32-bit
// byte offset (one VGPR), which maps to the saddr form of global loads and
// stores and keeps 64-bit address arithmetic out of the loop.
typedef __attribute__((address_space(1))) char gchar;
template <typename T>
struct GMem {
  typedef __attribute__((address_space(1))) T type;
};
template <typename T>
__device__ __forceinline__ T gload(const char* base, unsigned off) {
  return *(const typename GMem<T>::type*)((const gchar*)base + off);
}
// A per-lane byte offset re-defined where it is used (an empty asm statement):
// see load_groups() for why loop-invariant offsets need it.
__device__ __forceinline__ unsigned lane_off(unsigned off) {
  asm volatile("" : "+v"(off));
  return off;
}
template <typename T>
__device__ __forceinline__ void gstore(char* base, unsigned off, T v) {
  *(typename GMem<T>::type*)((gchar*)base + off) = v;
}

// The grouped values of one cell (all but phi; layout in state_index()):
// one 4-wide vector access per full group, scalar accesses for a last
// partial group. `base` is the start of the cell's row (uniform over the
// wave), `c` its column and PB the bytes of one value across the row (nx
// values). In a march (OPQ) the per-lane byte offset goes through lane_off():
// the column offset is the same for every row, and hoisted out of the loop as
// a 64-bit value it would no longer match the saddr form (scalar base plus
// 32-bit vector offset); each access would then build a 64-bit address in
// vector registers. Elsewhere the plain offset keeps the scheduler free (the
// asm statement bounds its regions).
template <typename T>
using Vec4 = T __attribute__((ext_vector_type(4)));
template <typename T, int NV, bool OPQ = false>
__device__ __forceinline__ void load_groups(const char* base, long long PB, unsigned c,
                                            T (&v)[NV]) {
  const unsigned co = OPQ ? lane_off(c * (4u * sizeof(T))) : c * (4u * sizeof(T));
#pragma unroll
  for (int g = 0; g < NV / 4; ++g) {
    const Vec4<T> x = gload<Vec4<T>>(base + 4 * g * PB, co);
    v[4 * g] = x.x; v[4 * g + 1] = x.y; v[4 * g + 2] = x.z; v[4 * g + 3] = x.w;
  }
  constexpr int w = NV % 4;
#pragma unroll
  for (int k = 0; k < w; ++k)
    v[NV - w + k] = gload<T>(base + (NV - w) * PB, (c * w + k) * (unsigned)sizeof(T));
}
template <typename T, int NV, bool OPQ = false>
__device__ __forceinline__ void store_groups(char* base, long long PB, unsigned c,
                                             const T (&v)[NV]) {
  const unsigned co = OPQ ? lane_off(c * (4u * sizeof(T))) : c * (4u * sizeof(T));
#pragma unroll
  for (int g = 0; g < NV / 4; ++g) {
    Vec4<T> x;
    x.x = v[4 * g]; x.y = v[4 * g + 1]; x.z = v[4 * g + 2]; x.w = v[4 * g + 3];
    gstore<Vec4<T>>(base + 4 * g * PB, co, x);
  }
  constexpr int w = NV % 4;
#pragma unroll
  for (int k = 0; k < w; ++k)
    gstore<T>(base + (NV - w) * PB, (c * w + k) * (unsigned)sizeof(T), v[NV - w + k]);
}

// Row index of a row in [-2, ny + 2): one period (periodic) or one
// reflection about the wall (walls) brings it into the grid.
__device__ __forceinline__ int row_idx(int r, int ny, int walls) {
  if (r < 0) return walls ? -1 - r : r + ny;
  if (r >= ny) return walls ? 2 * ny - 1 - r : r - ny;
  return r;
}

// Start of grid row `row` of a state buffer (RB bytes per row). The row must
// be the same on every lane of the wave: taking it from the first active lane
// tells the compiler so, which keeps the row address in scalar registers and
// the per-lane column offset in one 32-bit register (the saddr form of the
// global accesses).
template <typename P>
__device__ __forceinline__ P* row_ptr(P* base, int row, long long RB) {
  const unsigned long long a =
      reinterpret_cast<uintptr_t>(base) + (unsigned long long)((long long)row * RB);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return reinterpret_cast<P*>(((unsigned long long)hi << 32) | lo);
}

// Non-finite guard of the update: x sums the new phi with phi u and p of
// the cell stage (a NaN or Inf in f shows in the new phi at once, one in g in
// u and p of the next step). A lane holding a non-finite sum stores 1 in the
// case's flag (a plain vector store; nothing is read back on the device).
template <typename T>
__device__ __forceinline__ void flag_nonfinite(const CaseDev& C, T x) {
  if (!__builtin_isfinite(x) && C.flag) *(volatile int*)C.flag = 1;
}

template <typename T, bool CPL>
struct RowData {
  Cell<T> cell;
  T txf[9], txg[9];  // x central differences (diagonal pops)
  T txMx, txJx, txPxx, txPxy;
  T fnf[9], fng[9];  // face distributions of the face above this row
};

template <typename T, bool CPL, bool BP = false>
__device__ __forceinline__ void x_diffs(RowData<T, CPL>& r) {
  const int diag[4] = {2, 4, 6, 8};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = diag[k];
    r.txf[q] = xr<BP>(r.cell.fb[q]) - xl<BP>(r.cell.fb[q]);
    if (CPL) r.txg[q] = xr<BP>(r.cell.gb[q]) - xl<BP>(r.cell.gb[q]);
  }
  r.txMx = xr<BP>(r.cell.Mx) - xl<BP>(r.cell.Mx);
  if (CPL) {
    r.txJx = xr<BP>(r.cell.Jx) - xl<BP>(r.cell.Jx);
    r.txPxx = xr<BP>(r.cell.Pxx) - xl<BP>(r.cell.Pxx);
    r.txPxy = xr<BP>(r.cell.Pxy) - xl<BP>(r.cell.Pxy);
  }
}

// y-face between row D (below) and row U (above), own column.
template <typename T, bool CPL>
__device__ __forceinline__ void y_face(const CaseDev& C, const RowData<T, CPL>& D,
                                       const RowData<T, CPL>& U, double xf, double yf,
                                       double tf, T (&fo)[9], T (&go)[9]) {
  const T h = ck<T>(C.f32.h, C.h), hq = T(0.25) * ck<T>(C.f32.h, C.h);
  // mean minus h e_y times the normal slope, as weights of the two cells:
  // (1/2 + h e_y) below + (1/2 - h e_y) above
  const T cp = T(0.5) + h, cm = T(0.5) - h;
  T fbar[9], gbar[9];
#pragma unroll
  for (int q = 1; q < 9; ++q) {
    if (EY[q] == 0) continue;
    const T ex = T(EX[q]);
    const T cD = EY[q] > 0 ? cp : cm, cU = EY[q] > 0 ? cm : cp;
    T vf = cD * D.cell.fb[q] + cU * U.cell.fb[q];
    if (EX[q] != 0) vf -= hq * ex * (D.txf[q] + U.txf[q]);
    fbar[q] = vf;
    if (CPL) {
      T vg = cD * D.cell.gb[q] + cU * U.cell.gb[q];
      if (EX[q] != 0) vg -= hq * ex * (D.txg[q] + U.txg[q]);
      gbar[q] = vg;
    }
  }
  const Cell<T>& a = D.cell;
  const Cell<T>& b = U.cell;
  const T phif = T(0.5) * (a.M0 + b.M0) - h * (b.My - a.My) - hq * (D.txMx + U.txMx);
  T N0f = T(0), Jxf = T(0), Jyf = T(0);
  if (CPL) {
    N0f = T(0.5) * (a.N0 + b.N0) - h * (b.Jy - a.Jy) - hq * (D.txJx + U.txJx);
    Jxf = T(0.5) * (a.Jx + b.Jx) - h * (b.Pxy - a.Pxy) - hq * (D.txPxx + U.txPxx);
    Jyf = T(0.5) * (a.Jy + b.Jy) - h * (b.Pyy - a.Pyy) - hq * (D.txPxy + U.txPxy);
  }
  face_df<T, CPL, 1>(C, phif, N0f, Jxf, Jyf, T(0.5) * (a.gx + b.gx), T(0.5) * (a.gy + b.gy),
                     T(0.5) * (a.mu + b.mu), T(0.5) * (a.Dx + b.Dx), T(0.5) * (a.Dy + b.Dy),
                     fbar, gbar, xf, yf, tf, fo, go);
}

// Tangential (y) differences of the diagonal populations and moments at the
// own cell for its x-face: next - prev, or twice the one-sided difference
// next to a wall.
template <typename T, bool CPL>
struct Ty {
  T f[9], g[9], My, Jy, Pxy, Pyy;
};
template <typename T, bool CPL>
__device__ __forceinline__ void y_diffs(const RowData<T, CPL>& up, const RowData<T, CPL>& dn,
                                        T sc, Ty<T, CPL>& t) {
  const int diag[4] = {2, 4, 6, 8};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int q = diag[m];
    t.f[q] = sc * (up.cell.fb[q] - dn.cell.fb[q]);
    if (CPL) t.g[q] = sc * (up.cell.gb[q] - dn.cell.gb[q]);
  }
  t.My = sc * (up.cell.My - dn.cell.My);
  t.Jy = sc * (up.cell.Jy - dn.cell.Jy);
  t.Pxy = sc * (up.cell.Pxy - dn.cell.Pxy);
  t.Pyy = sc * (up.cell.Pyy - dn.cell.Pyy);
}

// x-face east of each cell of output row k and the wall faces of that row
// (face bounce-back, wall_face()), from the records of rows k-1 (prv), k (cur)
// and k+1 (nxt); a bottom
// wall face lands in prv.fnf/fng (the face below row k), a top one in
// cur.fnf/fng (the face above).
template <typename T, bool CPL, bool WALLS, bool BP = false>
__device__ __forceinline__ void row_xface(const CaseDev& C, int k, int ny, int ci, double tn,
                                          RowData<T, CPL>& prv, RowData<T, CPL>& cur_r,
                                          const RowData<T, CPL>& nxt, T (&fx_f)[9], T (&fx_g)[9]) {
  constexpr int walls = WALLS ? 1 : 0;
  const bool top_wall = walls && k == ny - 1;
  const bool bot_wall = walls && k == 0;
  Ty<T, CPL> ty;
  if (WALLS && top_wall) y_diffs<T, CPL>(cur_r, prv, T(2), ty);
  else if (WALLS && bot_wall) y_diffs<T, CPL>(nxt, cur_r, T(2), ty);
  else y_diffs<T, CPL>(nxt, prv, T(1), ty);
  // x-face east of the own cell: L = own lane, R = lane + 1
  {
    const Cell<T>& L = cur_r.cell;
    const T h = ck<T>(C.f32.h, C.h), hq = T(0.25) * ck<T>(C.f32.h, C.h);
    // (1/2 + h e_x) own + (1/2 - h e_x) right neighbour (mean minus h e_x
    // times the normal slope)
    const T cp = T(0.5) + h, cm = T(0.5) - h;
    T fbar[9], gbar[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (EX[q] == 0) continue;
      const T ey = T(EY[q]);
      const T cL = EX[q] > 0 ? cp : cm, cR = EX[q] > 0 ? cm : cp;
      T vf = cL * L.fb[q] + cR * xr<BP>(L.fb[q]);
      if (EY[q] != 0) vf -= hq * ey * (ty.f[q] + xr<BP>(ty.f[q]));
      fbar[q] = vf;
      if (CPL) {
        T vg = cL * L.gb[q] + cR * xr<BP>(L.gb[q]);
        if (EY[q] != 0) vg -= hq * ey * (ty.g[q] + xr<BP>(ty.g[q]));
        gbar[q] = vg;
      }
    }
    const T phif = T(0.5) * (L.M0 + xr<BP>(L.M0)) - h * (xr<BP>(L.Mx) - L.Mx) -
                   hq * (ty.My + xr<BP>(ty.My));
    T N0f = T(0), Jxf = T(0), Jyf = T(0);
    if (CPL) {
      N0f = T(0.5) * (L.N0 + xr<BP>(L.N0)) - h * (xr<BP>(L.Jx) - L.Jx) -
            hq * (ty.Jy + xr<BP>(ty.Jy));
      Jxf = T(0.5) * (L.Jx + xr<BP>(L.Jx)) - h * (xr<BP>(L.Pxx) - L.Pxx) -
            hq * (ty.Pxy + xr<BP>(ty.Pxy));
      Jyf = T(0.5) * (L.Jy + xr<BP>(L.Jy)) - h * (xr<BP>(L.Pxy) - L.Pxy) -
            hq * (ty.Pyy + xr<BP>(ty.Pyy));
    }
    const T gxf = T(0.5) * (L.gx + xr<BP>(L.gx));
    const T gyf = T(0.5) * (L.gy + xr<BP>(L.gy));
    const T muf = T(0.5) * (L.mu + xr<BP>(L.mu));
    const T Dxf = T(0.5) * (L.Dx + xr<BP>(L.Dx));
    const T Dyf = T(0.5) * (L.Dy + xr<BP>(L.Dy));
    const int kr = row_idx(k, ny, walls);
    face_df<T, CPL, 0>(C, phif, N0f, Jxf, Jyf, gxf, gyf, muf, Dxf, Dyf, fbar, gbar,
                       (double)ci + 1.0, (double)kr + 0.5, tn + C.h, fx_f, fx_g);
  }
  if (WALLS) {
    if (top_wall) wall_face<T, false>(C, cur_r.cell, prv.cell, cur_r.txf, cur_r.txg, cur_r.fnf, cur_r.fng);
    if (bot_wall) wall_face<T, true>(C, cur_r.cell, nxt.cell, cur_r.txf, cur_r.txg, prv.fnf, prv.fng);
  }
}

// Update of output row k (Eq. 24) and its stores. cur.fnf/fng hold the face
// above the row, prv.fnf/fng the face below, fx the x-faces east of each
// cell (the west face is the left lane's), tp(q) the tilde-plus values.
template <typename T, bool CPL, bool OPQ, bool BP = false, typename TP>
__device__ __forceinline__ void row_update(const CaseDev& C, int k, int ny, int nx, int walls,
                                           int ci, bool store, char* out, long long RB,
                                           long long PB,
                                           const RowData<T, CPL>& prv, const RowData<T, CPL>& cur_r,
                                           const T (&fx_f)[9], const T (&fx_g)[9], TP tp) {
  constexpr int NV = num_grouped(CPL);
  const unsigned es = sizeof(T);
  const T(&fn_f)[9] = cur_r.fnf;
  const T(&fn_g)[9] = cur_r.fng;
  const T(&fs_f)[9] = prv.fnf;
  const T(&fs_g)[9] = prv.fng;
  char* orow = row_ptr(out, row_idx(k, ny, walls), RB);
  const T dt = ck<T>(C.f32.dt, C.dt);
  T nv[NV];  // new tilde f, tilde g, history
  T phin = T(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    T J = T(0);
    if (EX[q] != 0) J += T(EX[q]) * (fx_f[q] - xl<BP>(fx_f[q]));
    if (EY[q] != 0) J += T(EY[q]) * (fn_f[q] - fs_f[q]);
    nv[val_f(q)] = tp(q) - dt * J;
    phin += nv[val_f(q)];
  }
  if (CPL) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      T J = T(0);
      if (EX[q] != 0) J += T(EX[q]) * (fx_g[q] - xl<BP>(fx_g[q]));
      if (EY[q] != 0) J += T(EY[q]) * (fn_g[q] - fs_g[q]);
      nv[val_g(q)] = tp(9 + q) - dt * J;
    }
  }
  nv[val_hist(CPL, 0)] = cur_r.cell.hx;
  nv[val_hist(CPL, 1)] = cur_r.cell.hy;
  // one masked region for all stores of the row
  if (store) {
    store_groups<T, NV, OPQ>(orow, PB, (unsigned)ci, nv);
    gstore<T>(orow + NV * PB, OPQ ? lane_off((unsigned)ci * es) : (unsigned)ci * es, phin);
    flag_nonfinite(C, phin + cur_r.cell.hx + cur_r.cell.hy + cur_r.cell.p);
  }
}

// The march of one work item: the wave owns a 62-column strip and rows
// [j0, j1) of it, and marches through them upwards (DOWN = false) or
// downwards. Alternate segments march in opposite directions (the item's
// `dir`), so that the two waves on either side of a segment boundary reach it
// at the same time, both at their start or both at their end: the halo rows
// that both read then come from the L2 cache for the second one. Every row,
// face and update goes through the same functions with the same inputs in
// either direction, so the results are the same bit for bit.
template <typename T, bool CPL, bool WALLS, bool DOWN>
__device__ __forceinline__ void march(const CaseDev& C, const Item& it, long long n) {
  constexpr int sgn = DOWN ? -1 : 1;  // marching direction in rows
  const int lane = threadIdx.x;
  constexpr bool BP = sizeof(T) == 4 && CPL;  // neighbour moves through the LDS crossbar (xr, xl)
  const int nx = C.nx, ny = C.ny;
  constexpr int walls = WALLS ? 1 : 0;
  const int i0 = it.strip * kStripCols;
  const int col = i0 - 1 + lane;
  const int ci = wrap(col, nx);
  const int cx = lane == 0 ? wrap(col - 1, nx) : (lane == 63 ? wrap(col + 1, nx) : ci);
  const bool store = lane >= 1 && lane <= kStripCols && col < nx;
  const int cur = (C.cur0 + (int)(n & 1)) & 1;
  const char* in = static_cast<const char*>(cur ? C.set[1] : C.set[0]);
  char* out = static_cast<char*>(cur ? C.set[0] : C.set[1]);
  const long long RB = C.row_vals * (long long)sizeof(T);  // bytes per grid row
  const long long PB = (long long)nx * sizeof(T);            // bytes of one value across a row
  constexpr int NV = num_grouped(CPL);
  const unsigned es = sizeof(T);
  const double tn = C.t0 + (double)n * C.dt;
  const double xc = (double)ci + 0.5;  // wrapped: halo lanes see their true cell
  const int j0 = it.seg * C.seg_rows;
  const int j1 = min(j0 + C.seg_rows, ny);

  __shared__ T stash[2][18][64];

  // Raw inputs of the cell stage of row r (tilde f, g, history) and phi of
  // the row after it in marching order (own column and the halo lanes'
  // extra column). Two sets are in flight: a pass consumes one set in its
  // cell stage and then reloads it for the pass after next, so that more
  // than a pass of arithmetic covers the memory latency.
  struct Raw {
    T f[9], g[9], hx, hy, po, pe;
  };
  auto fetch = [&](int r, Raw& R) {
    T v[NV];
    load_groups<T, NV, true>(row_ptr(in, row_idx(r, ny, walls), RB), PB, (unsigned)ci, v);
#pragma unroll
    for (int q = 0; q < 9; ++q) R.f[q] = v[val_f(q)];
    if (CPL) {
#pragma unroll
      for (int q = 0; q < 9; ++q) R.g[q] = v[val_g(q)];
    }
    R.hx = v[val_hist(CPL, 0)];
    R.hy = v[val_hist(CPL, 1)];
    const char* prow = row_ptr(in, row_idx(r + sgn, ny, walls), RB) + NV * PB;
    R.po = gload<T>(prow, lane_off((unsigned)ci * es));
    R.pe = gload<T>(prow, lane_off((unsigned)cx * es));
  };
  // phi of one row for (left, own, right) columns from own and extra values
  auto phi_lr = [&](T own, T ext, T (&o)[3]) {
    T left = xl<BP>(own), right = xr<BP>(own);
    if (lane == 0) left = ext;
    if (lane == 63) right = ext;
    o[0] = left; o[1] = own; o[2] = right;
  };
  auto phi_row = [&](int r, T (&o)[3]) {
    const char* prow = row_ptr(in, row_idx(r, ny, walls), RB) + NV * PB;
    phi_lr(gload<T>(prow, lane_off((unsigned)ci * es)), gload<T>(prow, lane_off((unsigned)cx * es)), o);
  };
  // pm, p0, pp: phi of the rows below, at and above row r
  auto stage = [&](int r, const Raw& R, const T (&pm)[3], const T (&p0)[3], const T (&pp)[3],
                   RowData<T, CPL>& rd) {
    const int rr = row_idx(r, ny, walls);
    T ph[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { ph[0][k] = pm[k]; ph[1][k] = p0[k]; ph[2][k] = pp[k]; }
    T tp[18];
    cell_stage<T, CPL>(C, ph, R.f, R.g, R.hx, R.hy, xc, (double)rr + 0.5, tn, rd.cell, tp);
    const int slot = r & 1;
#pragma unroll
    for (int q = 0; q < 18; ++q) stash[slot][q][lane] = tp[q];
    x_diffs<T, CPL, BP>(rd);
  };

  // One pass of the march for output row k. With the records of the rows
  // before (prv), at (cur_r) and after (nxt) row k in marching order, and phi
  // of rows k, k + sgn and (from `raw`) k + 2 sgn, it stages row k + sgn into
  // `nxt`, forms the y-face between rows k and k + sgn (a record's fnf/fng
  // hold the face above its row), and (for output rows) the x-face east of
  // row k and the update of row k. The passes start two rows before the
  // segment so that every row, halo rows included, goes through the same
  // code: results do not depend on the segmentation, bit for bit.
  auto pass = [&](int k, Raw& raw, RowData<T, CPL>& prv, RowData<T, CPL>& cur_r,
                  RowData<T, CPL>& nxt, const T (&pa)[3], const T (&pb)[3], T (&pc)[3]) {
    const int rs = k + sgn;
    // the phi ring advances every pass (ghost rows mirror into the grid), the
    // cell stage runs only for rows that exist
    phi_lr(raw.po, raw.pe, pc);
    if (!(walls && (rs < 0 || rs >= ny))) {
      if (DOWN) stage(rs, raw, pc, pb, pa, nxt);
      else stage(rs, raw, pa, pb, pc, nxt);
    }
    // inputs of pass k + 2 sgn (row k + 3 sgn); rows past the segment's halo
    // are never staged, so the fetch stays on the rows the segment reads
    fetch(DOWN ? max(k - 3, j0 - 1) : min(k + 3, j1 + 1), raw);
    // the y-face between rows k and k + sgn, above the lower one
    RowData<T, CPL>& lo = DOWN ? nxt : cur_r;
    RowData<T, CPL>& hi = DOWN ? cur_r : nxt;
    const int kl = DOWN ? k - 1 : k;  // the lower row
    const bool face = DOWN ? k <= j1 : k >= j0 - 1;
    if (face && !(walls && (kl < 0 || kl >= ny - 1))) {
      const int kr = row_idx(kl, ny, walls);
      y_face<T, CPL>(C, lo, hi, xc, (double)kr + 1.0, tn + C.h, lo.fnf, lo.fng);
    }
    if (DOWN ? k >= j1 : k < j0) return;
    // the rows below and above row k
    RowData<T, CPL>& below = DOWN ? nxt : prv;
    RowData<T, CPL>& above = DOWN ? prv : nxt;
    T fx_f[9], fx_g[9];
    row_xface<T, CPL, WALLS, BP>(C, k, ny, ci, tn, below, cur_r, above, fx_f, fx_g);
    const int slot = k & 1;
    row_update<T, CPL, true, BP>(C, k, ny, nx, walls, ci, store, out, RB, PB, below, cur_r, fx_f,
                             fx_g, [&](int q) { return stash[slot][q][lane]; });
  };

  // The three row records and the three phi rows rotate after each pass. (A
  // loop unrolled by three, rotating by renaming instead of copies, needs
  // ~285 registers and ran 40% slower on gfx950: spills, or one wave per SIMD.)
  RowData<T, CPL> R0, R1, R2;
  T P0[3], P1[3], P2[3];
  auto rotate = [&]() {
    R0 = R1;
    R1 = R2;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      P0[m] = P1[m];
      P1[m] = P2[m];
    }
  };
  Raw ra, rb;  // inputs of the even and odd passes (counted from the first)
  // passes k = kb, kb + sgn, ..., two halo passes and one per segment row
  const int kb = DOWN ? j1 + 1 : j0 - 2;
  const int npass = j1 - j0 + 2;
  phi_row(kb, P0);
  phi_row(kb + sgn, P1);
  fetch(kb + sgn, ra);
  fetch(kb + 2 * sgn, rb);
  for (int m = 0; m < npass; m += 2) {
    const int k = kb + m * sgn;
    pass(k, ra, R0, R1, R2, P0, P1, P2);
    rotate();
    if (m + 1 < npass) {
      pass(k + sgn, rb, R0, R1, R2, P0, P1, P2);
      rotate();
    }
  }
}

template <typename T, bool CPL, bool WALLS>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? 2 : 1) void k_step(StepArgs A) {
  const int nb = gridDim.x;
  const int per = nb >> 3;  // grid is a multiple of 8 (one share per XCD)
  const int idx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (idx >= A.nitems) return;
  const Item it = A.items[idx];
  // The case constants are copied into registers once: read through the
  // descriptor pointer, they would be re-read after every store of the march
  // (the stores could alias them as far as the compiler knows).
  const CaseDev* Cg = A.cases + it.c;
  CaseDev C = *Cg;
  if (!WALLS) narrow_in_kernel(C);
  const long long n = *A.step_base + A.kofs - C.step0;
  if (n < 0 || n >= C.nsteps) return;
  // wall cases march upwards only (see item_dir): one copy of the march
  // keeps their register budget
  if (!WALLS && it.dir) march<T, CPL, WALLS, !WALLS>(C, it, n);
  else march<T, CPL, WALLS, false>(C, it, n);
}

// --------------------------------------------------- one-row step kernel

// The fields of a row record that the faces and slopes of the neighbouring
// rows read (y_face, y_diffs, wall_face) and that the x-faces of the row
// read (row_xface): the populations that cross a face, the x differences of
// the diagonal ones, the moments and the face inputs. kRec values per lane.
constexpr int kRec = 42;
template <typename T, bool CPL, bool PUT>
__device__ __forceinline__ void move_record(T (*X)[64], int lane, RowData<T, CPL>& r) {
  int m = 0;
  auto mv = [&](T& v) {
    if (PUT) X[m][lane] = v;
    else v = X[m][lane];
    ++m;
  };
  const int cross[8] = {1, 2, 3, 4, 5, 6, 7, 8};
  const int diag[4] = {2, 4, 6, 8};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    mv(r.cell.fb[cross[k]]);
    if (CPL) mv(r.cell.gb[cross[k]]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    mv(r.txf[diag[k]]);
    if (CPL) mv(r.txg[diag[k]]);
  }
  mv(r.cell.M0); mv(r.cell.Mx); mv(r.cell.My); mv(r.txMx);
  if (CPL) {
    mv(r.cell.N0); mv(r.cell.Jx); mv(r.cell.Jy); mv(r.cell.Pxx); mv(r.cell.Pxy); mv(r.cell.Pyy);
    mv(r.txJx); mv(r.txPxx); mv(r.txPxy);
  }
  mv(r.cell.gx); mv(r.cell.gy); mv(r.cell.mu); mv(r.cell.Dx); mv(r.cell.Dy);
}

// One output row j of one 62-column strip per work group of three waves,
// for tiles of one row (seg_rows == 1), where a single wave marching three
// rows would be latency-bound. Wave w stages row j - 1 + w; the row records
// meet in LDS; at the same time wave 0 forms the face between rows j - 1 and
// j, wave 1 the face above row j and wave 2 the x-faces of row j (wave 1 when
// a wall bounds the row); wave 1 then updates row j. Every quantity goes
// through the same functions, with the same inputs, as in the march of
// k_step, so the results are the same bit for bit.
template <typename T, bool CPL, bool WALLS>
__global__ __launch_bounds__(192, sizeof(T) == 4 ? 2 : 1) void k_step_row(StepArgs A) {
  const int nb = gridDim.x;
  const int per = nb >> 3;  // grid is a multiple of 8 (one share per XCD)
  const int idx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (idx >= A.nitems) return;  // uniform over the work group
  const Item it = A.items[idx];
  CaseDev C = A.cases[it.c];
  narrow_in_kernel(C);
  const long long n = *A.step_base + A.kofs - C.step0;
  if (n < 0 || n >= C.nsteps) return;  // uniform over the work group

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const int nx = C.nx, ny = C.ny;
  constexpr int walls = WALLS ? 1 : 0;
  const int i0 = it.strip * kStripCols;
  const int col = i0 - 1 + lane;
  const int ci = wrap(col, nx);
  const int cx = lane == 0 ? wrap(col - 1, nx) : (lane == 63 ? wrap(col + 1, nx) : ci);
  const bool store = lane >= 1 && lane <= kStripCols && col < nx;
  const int cur = (C.cur0 + (int)(n & 1)) & 1;
  const char* in = static_cast<const char*>(cur ? C.set[1] : C.set[0]);
  char* out = static_cast<char*>(cur ? C.set[0] : C.set[1]);
  const long long RB = C.row_vals * (long long)sizeof(T);  // bytes per grid row
  const long long PB = (long long)nx * sizeof(T);            // bytes of one value across a row
  constexpr int NV = num_grouped(CPL);
  const unsigned es = sizeof(T);
  const double tn = C.t0 + (double)n * C.dt;
  const double xc = (double)ci + 0.5;
  const int j = it.seg;  // tiles of one row: segment index = row
  const int r = j - 1 + w;
  const bool exists = !(walls && (r < 0 || r >= ny));

  __shared__ T rec[3][kRec][64];
  __shared__ T below[18][64];  // face between rows j - 1 and j (f, g)
  __shared__ T east[18][64];   // x-faces east of the cells of row j (f, g)
  __shared__ T tplus[18][64];  // tilde-plus of row j

  RowData<T, CPL> rd;
  if (exists) {
    T v[NV];
    load_groups<T, NV>(row_ptr(in, row_idx(r, ny, walls), RB), PB, (unsigned)ci, v);
    T f[9], g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      f[q] = v[val_f(q)];
      g[q] = CPL ? v[val_g(q)] : T(0);
    }
    T ph[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const char* prow = row_ptr(in, row_idx(r - 1 + a, ny, walls), RB) + NV * PB;
      const T own = gload<T>(prow, (unsigned)ci * es), ext = gload<T>(prow, (unsigned)cx * es);
      T left = nbr_l(own), right = nbr_r(own);
      if (lane == 0) left = ext;
      if (lane == 63) right = ext;
      ph[a][0] = left; ph[a][1] = own; ph[a][2] = right;
    }
    T tp[18];
    cell_stage<T, CPL>(C, ph, f, g, v[val_hist(CPL, 0)], v[val_hist(CPL, 1)], xc,
                       (double)row_idx(r, ny, walls) + 0.5, tn, rd.cell, tp);
    if (w == 1) {
#pragma unroll
      for (int q = 0; q < 18; ++q) tplus[q][lane] = tp[q];
    }
    x_diffs<T, CPL>(rd);
    move_record<T, CPL, true>(rec[w], lane, rd);
  }
  __syncthreads();
  const bool bot_wall = walls && j == 0;
  const bool top_wall = walls && j == ny - 1;
  const bool wall_row = bot_wall || top_wall;  // wave 1 forms the x-faces itself
  T fx_f[9], fx_g[9];
  RowData<T, CPL> prv;
  if (w == 2 && !wall_row) {
    // x-faces of row j: rows j - 1 and j from LDS, row j + 1 is this wave's
    RowData<T, CPL> pj, cj;
    move_record<T, CPL, false>(rec[0], lane, pj);
    move_record<T, CPL, false>(rec[1], lane, cj);
    row_xface<T, CPL, WALLS>(C, j, ny, ci, tn, pj, cj, rd, fx_f, fx_g);
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (EX[q] == 0) continue;
      east[q][lane] = fx_f[q];
      if (CPL) east[9 + q][lane] = fx_g[q];
    }
  }
  if (w == 0) {
    // the face above row j - 1 (below row j)
    if (exists && !(walls && r >= ny - 1)) {
      RowData<T, CPL> up;
      move_record<T, CPL, false>(rec[1], lane, up);
      y_face<T, CPL>(C, rd, up, xc, (double)row_idx(r, ny, walls) + 1.0, tn + C.h, rd.fnf, rd.fng);
#pragma unroll
      for (int q = 1; q < 9; ++q) {
        if (EY[q] == 0) continue;
        below[q][lane] = rd.fnf[q];
        if (CPL) below[9 + q][lane] = rd.fng[q];
      }
    }
  } else if (w == 1) {
    RowData<T, CPL> nxt;
    if (!(walls && j - 1 < 0)) move_record<T, CPL, false>(rec[0], lane, prv);
    if (!(walls && j + 1 >= ny)) move_record<T, CPL, false>(rec[2], lane, nxt);
    if (!(walls && j >= ny - 1))
      y_face<T, CPL>(C, rd, nxt, xc, (double)row_idx(j, ny, walls) + 1.0, tn + C.h, rd.fnf, rd.fng);
    if (wall_row) row_xface<T, CPL, WALLS>(C, j, ny, ci, tn, prv, rd, nxt, fx_f, fx_g);
  }
  __syncthreads();
  if (w == 1) {
    if (!wall_row) {
#pragma unroll
      for (int q = 1; q < 9; ++q) {
        if (EX[q] == 0) continue;
        fx_f[q] = east[q][lane];
        if (CPL) fx_g[q] = east[9 + q][lane];
      }
    }
    if (!bot_wall) {
#pragma unroll
      for (int q = 1; q < 9; ++q) {
        if (EY[q] == 0) continue;
        prv.fnf[q] = below[q][lane];
        if (CPL) prv.fng[q] = below[9 + q][lane];
      }
    }
    row_update<T, CPL, false>(C, j, ny, nx, walls, ci, store, out, RB, PB, prv, rd, fx_f, fx_g,
                       [&](int q) { return tplus[q][lane]; });
  }
}

// --------------------------------------------------- two-row step kernel

// Two output rows j and j + 1 of one 62-column strip per work group of four
// waves, for 2-row tiles of periodic cases in FP32. Wave w stages row
// j - 1 + w; after the records meet in LDS, wave 0 forms the face below row j
// and the face above row j + 1, wave 1 the face between the two rows, wave 2
// the x-faces of row j + 1 and wave 3 those of row j; waves 1 and 2 then
// update the two rows. A 128^2 grid takes 192 such groups where one-row tiles
// take 384: one group per CU, so no two waves share a SIMD, which costs less
// than the second face on wave 0. Every quantity goes through the same
// functions, with the same inputs, as in the march: the same bits.
template <typename T, bool CPL>
__global__ __launch_bounds__(256) void k_step_row2(StepArgs A) {
  static_assert(sizeof(T) == 4, "the LDS records of four rows fit 64 KB in FP32 only");
  const int nb = gridDim.x;
  const int per = nb >> 3;  // grid is a multiple of 8 (one share per XCD)
  const int idx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (idx >= A.nitems) return;  // uniform over the work group
  const Item it = A.items[idx];
  CaseDev C = A.cases[it.c];
  narrow_in_kernel(C);
  const long long n = *A.step_base + A.kofs - C.step0;
  if (n < 0 || n >= C.nsteps) return;  // uniform over the work group

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const int nx = C.nx, ny = C.ny;
  constexpr int walls = 0;
  const int i0 = it.strip * kStripCols;
  const int col = i0 - 1 + lane;
  const int ci = wrap(col, nx);
  const int cx = lane == 0 ? wrap(col - 1, nx) : (lane == 63 ? wrap(col + 1, nx) : ci);
  const bool store = lane >= 1 && lane <= kStripCols && col < nx;
  const int cur = (C.cur0 + (int)(n & 1)) & 1;
  const char* in = static_cast<const char*>(cur ? C.set[1] : C.set[0]);
  char* out = static_cast<char*>(cur ? C.set[0] : C.set[1]);
  const long long RB = C.row_vals * (long long)sizeof(T);  // bytes per grid row
  const long long PB = (long long)nx * sizeof(T);            // bytes of one value across a row
  constexpr int NV = num_grouped(CPL);
  const unsigned es = sizeof(T);
  const double tn = C.t0 + (double)n * C.dt;
  const double xc = (double)ci + 0.5;
  const int j = it.seg * 2;     // tiles of two rows: segment index = row pair
  const bool two = j + 1 < ny;  // the last tile of an odd ny has one row
  const int r = j - 1 + w;      // staged row (periodic)

  __shared__ T rec[4][kRec][64];
  __shared__ T tplus[2][18][64];  // tilde-plus of rows j and j + 1
  // crossing populations of four faces (f in slots 0-5, g in 6-11): below
  // row j, between the rows, above row j + 1, and the x-faces of row j
  __shared__ T fyb[12][64], fym[12][64], fya[12][64], fx0[12][64];

  RowData<T, CPL> rd;
  {
    T v[NV];
    load_groups<T, NV>(row_ptr(in, row_idx(r, ny, walls), RB), PB, (unsigned)ci, v);
    T f[9], g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      f[q] = v[val_f(q)];
      g[q] = CPL ? v[val_g(q)] : T(0);
    }
    T ph[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const char* prow = row_ptr(in, row_idx(r - 1 + a, ny, walls), RB) + NV * PB;
      const T own = gload<T>(prow, (unsigned)ci * es), ext = gload<T>(prow, (unsigned)cx * es);
      T left = nbr_l(own), right = nbr_r(own);
      if (lane == 0) left = ext;
      if (lane == 63) right = ext;
      ph[a][0] = left; ph[a][1] = own; ph[a][2] = right;
    }
    T tp[18];
    cell_stage<T, CPL>(C, ph, f, g, v[val_hist(CPL, 0)], v[val_hist(CPL, 1)], xc,
                       (double)row_idx(r, ny, walls) + 0.5, tn, rd.cell, tp);
    if (w == 1 || w == 2) {
#pragma unroll
      for (int q = 0; q < 18; ++q) tplus[w - 1][q][lane] = tp[q];
    }
    x_diffs<T, CPL>(rd);
    move_record<T, CPL, true>(rec[w], lane, rd);
  }
  __syncthreads();
  // face distributions of the populations crossing a y-face / an x-face
  auto put = [&](T(*F)[64], bool yface, const T(&fo)[9], const T(&go)[9]) {
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      const int sl = yface ? up_yslot(q) : up_xslot(q);
      if (sl < 0) continue;
      F[sl][lane] = fo[q];
      if (CPL) F[6 + sl][lane] = go[q];
    }
  };
  auto get = [&](const T(*F)[64], bool yface, T(&fo)[9], T(&go)[9]) {
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      const int sl = yface ? up_yslot(q) : up_xslot(q);
      if (sl < 0) continue;
      fo[q] = F[sl][lane];
      if (CPL) go[q] = F[6 + sl][lane];
    }
  };
  T fx_f[9], fx_g[9];
  if (w == 0) {
    // the face below row j (above row j - 1): this wave's row and row j
    RowData<T, CPL> up;
    move_record<T, CPL, false>(rec[1], lane, up);
    y_face<T, CPL>(C, rd, up, xc, (double)row_idx(j - 1, ny, walls) + 1.0, tn + C.h, rd.fnf, rd.fng);
    put(fyb, true, rd.fnf, rd.fng);
    if (two) {
      // the face above row j + 1: rows j + 1 and j + 2
      RowData<T, CPL> a, b;
      move_record<T, CPL, false>(rec[2], lane, a);
      move_record<T, CPL, false>(rec[3], lane, b);
      y_face<T, CPL>(C, a, b, xc, (double)row_idx(j + 1, ny, walls) + 1.0, tn + C.h, a.fnf, a.fng);
      put(fya, true, a.fnf, a.fng);
    }
  } else if (w == 1) {
    // the face above row j (below row j + 1); this wave updates row j
    RowData<T, CPL> up;
    move_record<T, CPL, false>(rec[2], lane, up);
    y_face<T, CPL>(C, rd, up, xc, (double)row_idx(j, ny, walls) + 1.0, tn + C.h, rd.fnf, rd.fng);
    if (two) put(fym, true, rd.fnf, rd.fng);
  } else if (w == 2) {
    // x-faces of row j + 1 (this wave's row, which it updates)
    if (two) {
      RowData<T, CPL> pj, nj;
      move_record<T, CPL, false>(rec[1], lane, pj);
      move_record<T, CPL, false>(rec[3], lane, nj);
      row_xface<T, CPL, false>(C, j + 1, ny, ci, tn, pj, rd, nj, fx_f, fx_g);
    }
  } else {
    // x-faces of row j: rows j - 1, j, j + 1
    RowData<T, CPL> pj, cj, nj;
    move_record<T, CPL, false>(rec[0], lane, pj);
    move_record<T, CPL, false>(rec[1], lane, cj);
    move_record<T, CPL, false>(rec[2], lane, nj);
    row_xface<T, CPL, false>(C, j, ny, ci, tn, pj, cj, nj, fx_f, fx_g);
    put(fx0, false, fx_f, fx_g);
  }
  __syncthreads();
  if (w == 1) {
    RowData<T, CPL> prv;
    get(fyb, true, prv.fnf, prv.fng);
    get(fx0, false, fx_f, fx_g);
    row_update<T, CPL, false>(C, j, ny, nx, walls, ci, store, out, RB, PB, prv, rd, fx_f, fx_g,
                              [&](int q) { return tplus[0][q][lane]; });
  } else if (w == 2 && two) {
    RowData<T, CPL> prv;
    get(fym, true, prv.fnf, prv.fng);
    get(fya, true, rd.fnf, rd.fng);
    row_update<T, CPL, false>(C, j + 1, ny, nx, walls, ci, store, out, RB, PB, prv, rd, fx_f,
                              fx_g, [&](int q) { return tplus[1][q][lane]; });
  }
}

__global__ void k_advance(long long* step_base, long long by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step_base[0] += by;
}

// Set a step counter and clear a non-finite flag (a kernel rather than
// memsets, so that a caller may capture it in a graph).
__global__ void k_reset(long long* step_base, long long value, int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (step_base) step_base[0] = value;
    if (flag) flag[0] = 0;
  }
}

// ------------------------------------------------------------ init / macros

// phi on the 3x3 neighbourhood of cell (i, j) from a row-major field.
// ------------------------------------------------------- stretched meshes

// On a stretched tensor-product mesh the gradient and Laplacian stencils are
// weighted sums of the first and second derivatives of the parabola through
// three neighbouring centres, on the rows j-1, j, j+1 (columns i-1, i, i+1),
// the neighbouring rows weighted by the opposite distance so that the sum is
// centred on the cell: exact on quadratics, and the unit-mesh stencils on
// unit widths.
// Metric arrays in the kernel's precision: FP32 kernels read the float copy
// (one load and no conversion per value; a row's metrics stay uniform).
template <typename T>
__device__ __forceinline__ const T* mesh_of(const CaseDev& C);
template <>
__device__ __forceinline__ const float* mesh_of<float>(const CaseDev& C) { return C.meshf; }
template <>
__device__ __forceinline__ const double* mesh_of<double>(const CaseDev& C) { return C.mesh; }

// The metric arrays are read through the constant address space: they do
// not change during a launch, so a row's metrics (uniform over the wave)
// load into scalar registers, and a column's load with global rather than
// flat instructions.
template <typename S>
struct KMem {
  typedef __attribute__((address_space(4))) S type;
};
template <typename S>
using KAxis = MeshAxisT<typename KMem<S>::type>;
template <typename S>
__device__ __forceinline__ KAxis<S> kaxis(const S* mesh, int nx, int ny, int axis) {
  return mesh_axis((const typename KMem<S>::type*)mesh, nx, ny, axis);
}

// The stencil weights of one cell along one axis: the parabola weights and
// the weights of the neighbouring rows (columns) in the centred sum.
template <typename T>
struct StW {
  T cp, cm, ep, em, wp, wm;
  template <typename A>
  __device__ static StW load(const A& ax, int k) {
    return StW{ax.cp[k], ax.cm[k], ax.ep[k], ax.em[k], ax.wp[k], ax.wm[k]};
  }
};

template <typename T>
__device__ __forceinline__ void mesh_stencils(const StW<T>& x, const StW<T>& y, const T (&ph)[3][3],
                                              T& gx, T& gy, T& lap) {
  const T cpx = x.cp, cmx = x.cm, epx = x.ep, emx = x.em, wpx = x.wp, wmx = x.wm;
  const T cpy = y.cp, cmy = y.cm, epy = y.ep, emy = y.em, wpy = y.wp, wmy = y.wm;
  T dxr[3], dxxr[3], dyc[3], dyyc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T fx = ph[k][2] - ph[k][1], bx = ph[k][1] - ph[k][0];
    const T fy = ph[2][k] - ph[1][k], by = ph[1][k] - ph[0][k];
    dxr[k] = cpx * fx + cmx * bx;
    dxxr[k] = epx * fx - emx * bx;
    dyc[k] = cpy * fy + cmy * by;
    dyyc[k] = epy * fy - emy * by;
  }
  gx = T(2.0 / 3.0) * dxr[1] + T(1.0 / 3.0) * (wpy * dxr[2] + wmy * dxr[0]);
  gy = T(2.0 / 3.0) * dyc[1] + T(1.0 / 3.0) * (wpx * dyc[2] + wmx * dyc[0]);
  lap = T(5.0 / 6.0) * (dxxr[1] + dyyc[1]) + T(1.0 / 6.0) * (wpy * dxxr[2] + wmy * dxxr[0]) +
        T(1.0 / 6.0) * (wpx * dyyc[2] + wmx * dyyc[0]);
}
// ... of cell (i, j), the weights read from the metric arrays
template <typename T>
__device__ __forceinline__ void mesh_stencils(const CaseDev& C, const T (&ph)[3][3], int i, int j,
                                              T& gx, T& gy, T& lap) {
  mesh_stencils<T>(StW<T>::load(kaxis(mesh_of<T>(C), C.nx, C.ny, 0), i),
                   StW<T>::load(kaxis(mesh_of<T>(C), C.nx, C.ny, 1), j), ph, gx, gy, lap);
}

// Gradient and Laplacian of the init and readout kernels: the unit-mesh
// stencils (as in cell_stage), or the stretched-mesh ones.
template <typename T>
__device__ __forceinline__ void cell_stencils(const CaseDev& C, const T (&ph)[3][3], int i, int j,
                                              T& gx, T& gy, T& lap) {
  if (C.mesh) {
    mesh_stencils<T>(C, ph, i, j, gx, gy, lap);
    return;
  }
  gx = (T(4) * (ph[1][2] - ph[1][0]) + (ph[2][2] - ph[2][0]) + (ph[0][2] - ph[0][0])) * T(1.0 / 12.0);
  gy = (T(4) * (ph[2][1] - ph[0][1]) + (ph[2][2] - ph[0][2]) + (ph[2][0] - ph[0][0])) * T(1.0 / 12.0);
  const T cc = ph[1][1];
  lap = T(2.0 / 3.0) * (((ph[1][2] - cc) + (ph[1][0] - cc)) + ((ph[2][1] - cc) + (ph[0][1] - cc))) +
        T(1.0 / 6.0) * (((ph[2][2] - cc) + (ph[2][0] - cc)) + ((ph[0][2] - cc) + (ph[0][0] - cc)));
}

// Cell centre (for a prescribed velocity).
__device__ __forceinline__ void cell_centre(const CaseDev& C, int i, int j, double& x, double& y) {
  if (C.mesh) {
    x = mesh_axis(C.mesh, C.nx, C.ny, 0).c[i];
    y = mesh_axis(C.mesh, C.nx, C.ny, 1).c[j];
  } else {
    x = i + 0.5;
    y = j + 0.5;
  }
}

template <typename S, typename T>
__device__ __forceinline__ void gather3x3(const S* __restrict__ f, long long rs, int i, int j,
                                          int nx, int ny, int walls, T (&ph)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int r = row_of(j + a - 1, ny, walls);
#pragma unroll
    for (int b = 0; b < 3; ++b) ph[a][b] = T(f[(long long)r * rs + wrap(i + b - 1, nx)]);
  }
}

// Initial state: tilde = psi^eq - (dt/2) S with d_t(phi u) = 0, from
// the macros phi, u, v, p (double, [ny][nx]); hist = phi u; phi.
template <typename T, bool CPL>
__global__ void k_init(const CaseDev* __restrict__ Cd, int buf, const double* __restrict__ phi0,
                       const double* __restrict__ u0, const double* __restrict__ v0,
                       const double* __restrict__ p0) {
  const CaseDev& C = *Cd;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= C.nx || j >= C.ny) return;
  const long long c = (long long)j * C.nx + i, rv = C.row_vals;
  T* __restrict__ st = static_cast<T*>(C.set[buf]);
  auto at = [&](int v) -> T& { return st[state_index(v, i, j, C.nx, rv, CPL)]; };
  T ph[3][3];
  gather3x3<double, T>(phi0, C.nx, i, j, C.nx, C.ny, C.walls, ph);
  T gx, gy, lap;
  cell_stencils<T>(C, ph, i, j, gx, gy, lap);
  const T phi = ph[1][1];
  T dA, dB, mu, theta;
  phase_terms<T>(C, phi, lap, dA, dB, mu, theta);
  T nxv, nyv;
  normal<T>(C, gx, gy, nxv, nyv);
  const T hdt = ck<T>(C.f32.hdt, 0.5 * C.dt);
  T u, v;
  if (CPL) {
    u = u0 ? T(u0[c]) : T(0);
    v = v0 ? T(v0[c]) : T(0);
    const T p = p0 ? T(p0[c]) : T(0);
    const double rhoD = rho_of(C, (double)phi);
    const T rho = T(rhoD);
    const T rg = T(rhoD - C.rho_ref);
    const T Fx = mu * gx + (ck<T>(C.f32.Gx, C.Gx) + rg * ck<T>(C.f32.gx, C.gx));
    const T Fy = mu * gy + (ck<T>(C.f32.Gy, C.Gy) + rg * ck<T>(C.f32.gy, C.gy));
    const T drx = ck<T>(C.f32.drho, C.drho) * gx, dry = ck<T>(C.f32.drho, C.drho) * gy;
    const T uu = u * u + v * v;
    const T a0 = u * drx + v * dry, b0 = u * Fx + v * Fy;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const T e = T(EX[q]) * u + T(EY[q]) * v;
      const T Gh = e * (T(3) + T(4.5) * e) - T(1.5) * uu;
      const T aq = T(EX[q]) * drx + T(EY[q]) * dry;
      const T bq = T(EX[q]) * Fx + T(EY[q]) * Fy;
      const T Sg = wq<T>(q) * ((aq - a0) * Gh + T(3) * (bq - b0) * (T(1) + Gh));
      T geq = wq<T>(q) * (T(3) * p + rho * Gh);
      if (q == 0) geq -= T(3) * p;
      at(val_g(q)) = geq - hdt * Sg;
    }
  } else {
    double xc, yc;
    cell_centre(C, i, j, xc, yc);
    presc_vel<T>(C, xc, yc, 0.0, u, v);
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const T en = T(EX[q]) * nxv + T(EY[q]) * nyv;
    const T feq = wq<T>(q) * phi * (T(1) + T(3) * (T(EX[q]) * u + T(EY[q]) * v));
    const T Sf = wq<T>(q) * theta * en;
    at(val_f(q)) = feq - hdt * Sf;
  }
  at(val_hist(CPL, 0)) = phi * u;
  at(val_hist(CPL, 1)) = phi * v;
  // phi = sum of the stored f (the same sum the step kernel forms)
  T s = T(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) s += at(val_f(q));
  at(val_phi(CPL)) = s;
}

// Cell macros of cell (i, j) of a state (Eqs. 31-33, 10): phi, u, v, p in
// the working precision, rho in double.
template <typename T, bool CPL>
__device__ __forceinline__ void cell_macros(const CaseDev& C, const T* __restrict__ st, int i,
                                            int j, double t, T& phi, T& u, T& v, T& p,
                                            double& rhoD) {
  const long long rv = C.row_vals;
  T ph[3][3];
  gather3x3<T, T>(st + state_index(val_phi(CPL), 0, 0, C.nx, rv, CPL), rv, i, j, C.nx, C.ny,
                  C.walls, ph);
  phi = ph[1][1];
  rhoD = rho_of(C, (double)phi);
  p = T(0);
  if (CPL) {
    T gx, gy, lap;
    cell_stencils<T>(C, ph, i, j, gx, gy, lap);
    T dA, dB, mu, theta;
    phase_terms<T>(C, phi, lap, dA, dB, mu, theta);
    const T rho = T(rhoD), irho = T(inv_rho<T>(rhoD));
    const T rg = T(rhoD - C.rho_ref);
    const T Fx = mu * gx + (ck<T>(C.f32.Gx, C.Gx) + rg * ck<T>(C.f32.gx, C.gx));
    const T Fy = mu * gy + (ck<T>(C.f32.Gy, C.Gy) + rg * ck<T>(C.f32.gy, C.gy));
    T g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = st[state_index(val_g(q), i, j, C.nx, rv, CPL)];
    const T mx = (g[1] + g[2] + g[8]) - (g[4] + g[5] + g[6]);
    const T my = (g[2] + g[3] + g[4]) - (g[6] + g[7] + g[8]);
    const T m0 = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    const T dt = ck<T>(C.f32.dt, C.dt);
    u = (mx + T(0.5) * dt * Fx) * irho;
    v = (my + T(0.5) * dt * Fy) * irho;
    const T drx = ck<T>(C.f32.drho, C.drho) * gx, dry = ck<T>(C.f32.drho, C.drho) * gy;
    p = T(0.6) * m0 + T(0.3) * dt * (u * drx + v * dry) - T(0.4) * rho * (u * u + v * v);
  } else {
    double xc, yc;
    cell_centre(C, i, j, xc, yc);
    presc_vel<T>(C, xc, yc, t, u, v);
  }
}

// Cell macros of a state into double arrays.
template <typename T, bool CPL>
__global__ void k_macros(const CaseDev* __restrict__ Cd, int buf, double t,
                         double* __restrict__ ophi, double* __restrict__ ou,
                         double* __restrict__ ov, double* __restrict__ op,
                         double* __restrict__ orho) {
  const CaseDev& C = *Cd;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= C.nx || j >= C.ny) return;
  const long long c = (long long)j * C.nx + i;
  T phi, u, v, p;
  double rhoD;
  cell_macros<T, CPL>(C, static_cast<const T*>(C.set[buf]), i, j, t, phi, u, v, p, rhoD);
  if (ophi) ophi[c] = (double)phi;
  if (ou) ou[c] = (double)u;
  if (ov) ov[c] = (double)v;
  if (op) op[c] = (double)p;
  if (orho) orho[c] = rhoD;
}

// Diagnostics in double, in a fixed order: per-block partial sums (wavefront
// butterflies, then the block's waves), then one block folds the partials.
// out: sum phi, sum rho u, sum rho v, sum rho |u|^2 / 2, max |u|, sum rho,
// #non-finite.
constexpr int kDiagThreads = 256;
constexpr int kDiagQ = 7;

// Sum and maximum over the 64 lanes of a wave by a fixed butterfly of lane
// exchanges (every lane ends with the result; the order, and so the rounding,
// is the same on every run).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) x += __shfl_xor(x, m, kWave);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) x = fmax(x, __shfl_xor(x, m, kWave));
  return x;
}

__global__ void k_diag_partial(int nx, int ny, const double* __restrict__ phi,
                               const double* __restrict__ u, const double* __restrict__ v,
                               const double* __restrict__ rho, double* __restrict__ part) {
  constexpr int kWaves = kDiagThreads / kWave;
  __shared__ double sh[kDiagQ][kWaves];
  double a[kDiagQ] = {0, 0, 0, 0, 0, 0, 0};
  const long long n = (long long)nx * ny;
  for (long long c = (long long)blockIdx.x * kDiagThreads + threadIdx.x; c < n;
       c += (long long)gridDim.x * kDiagThreads) {
    const double r = rho[c], uu = u[c], vv = v[c], ph = phi[c];
    a[0] += ph;
    a[1] += r * uu;
    a[2] += r * vv;
    a[3] += 0.5 * r * (uu * uu + vv * vv);
    a[4] = fmax(a[4], sqrt(uu * uu + vv * vv));
    a[5] += r;
    const bool bad = !isfinite(ph) || !isfinite(uu) || !isfinite(vv) || !isfinite(r);
    a[6] += bad ? 1.0 : 0.0;
  }
  // wavefront reductions, then the waves' results through LDS
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kDiagQ; ++k) {
    const double r = k == 4 ? wave_max(a[k]) : wave_sum(a[k]);
    if (lane == 0) sh[k][w] = r;
  }
  __syncthreads();
  if (threadIdx.x < kDiagQ) {
    const int k = threadIdx.x;
    double r = sh[k][0];
    for (int x = 1; x < kWaves; ++x) r = k == 4 ? fmax(r, sh[k][x]) : r + sh[k][x];
    part[(long long)blockIdx.x * kDiagQ + k] = r;
  }
}

__global__ void k_diag_final(int nblocks, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a[kDiagQ] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < nblocks; ++b)
    for (int k = 0; k < kDiagQ; ++k) {
      const double x = part[(long long)b * kDiagQ + k];
      if (k == 4) a[k] = fmax(a[k], x);
      else a[k] += x;
    }
  for (int k = 0; k < kDiagQ; ++k) out[k] = a[k];
}

// ------------------------------------------ diagnostics without allocation

// The diagnostics of k_diag_partial / k_diag_final for callers that cannot
// allocate device memory: the cell macros are formed inside the reduction
// (no macro arrays), one work group per grid row folds its row into seven
// partial sums, and one work group folds the rows in row order. The per-row
// partials live in this file-scope device array: one copy per GPU, held for
// the life of the process and shared by every call on that GPU, so calls
// that overlap on one GPU race on it. Host code never passes the array's
// name to a kernel: noalloc_scratch() looks up its device address.
constexpr int kNoAllocRows = 65536;
static __device__ __align__(256) double scratch[kNoAllocRows * kDiagQ];

template <typename T, bool CPL>
__global__ __launch_bounds__(kDiagThreads) void k_diag_rows(const CaseDev* __restrict__ Cd, int buf,
                                                            double t, double* __restrict__ part) {
  constexpr int kWaves = kDiagThreads / kWave;
  __shared__ double sh[kDiagQ][kWaves];
  const CaseDev& C = *Cd;
  const int j = blockIdx.x;
  const T* st = static_cast<const T*>(C.set[buf]);
  double a[kDiagQ] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < C.nx; i += kDiagThreads) {
    T phi, u, v, p;
    double r;
    cell_macros<T, CPL>(C, st, i, j, t, phi, u, v, p, r);
    const double ph = (double)phi, uu = (double)u, vv = (double)v;
    a[0] += ph;
    a[1] += r * uu;
    a[2] += r * vv;
    a[3] += 0.5 * r * (uu * uu + vv * vv);
    a[4] = fmax(a[4], sqrt(uu * uu + vv * vv));
    a[5] += r;
    const bool bad = !isfinite(ph) || !isfinite(uu) || !isfinite(vv) || !isfinite(r);
    a[6] += bad ? 1.0 : 0.0;
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kDiagQ; ++k) {
    const double r = k == 4 ? wave_max(a[k]) : wave_sum(a[k]);
    if (lane == 0) sh[k][w] = r;
  }
  __syncthreads();
  if (threadIdx.x < kDiagQ) {
    const int k = threadIdx.x;
    double r = sh[k][0];
    for (int x = 1; x < kWaves; ++x) r = k == 4 ? fmax(r, sh[k][x]) : r + sh[k][x];
    part[(long long)j * kDiagQ + k] = r;
  }
}

// ----------------- upwind reconstruction and stretched meshes: pieces

// van Leer's limited slope of two one-sided differences (or slopes).
template <typename T>
__device__ __forceinline__ T van_leer(T a, T b) {
  // branch-free: the quotient is formed on every lane and discarded by the
  // select where a b <= 0 (a + b may then be 0). In float the hardware
  // reciprocal (1 ulp) replaces the correctly rounded division, which takes
  // ten instructions and, as the arm of a branch, a divergent jump.
  const T ab = a * b;  // 2 a b below is exactly ab + ab
  const T q = sizeof(T) == 4 ? (ab + ab) * T(__builtin_amdgcn_rcpf(float(a + b))) : (ab + ab) / (a + b);
  return ab > T(0) ? q : T(0);
}

// Metrics of one cell along one axis of a stretched mesh: width, the
// reciprocal centre distances to the previous and next cells, the weights of
// the parabola derivative d1 = cp (a+ - a) + cm (a - a-), and twice the
// reciprocal width (read from the metric arrays, which the host derives once).
template <typename T>
struct Met {
  T w, ihm, ihp, cp, cm, iw2;  // iw2 = 2 / w
  template <typename A>
  __device__ static Met load(const A& ax, int k) {
    return Met{ax.w[k], ax.ihm[k], ax.ihp[k], ax.cp[k], ax.cm[k], T(2) * ax.iw[k]};
  }
};

// s clamped to [-cap, cap] (cap >= 0): one median-of-three in float
__device__ __forceinline__ float clamp_sym(float s, float cap) {
  return __builtin_amdgcn_fmed3f(s, -cap, cap);
}
__device__ __forceinline__ double clamp_sym(double s, double cap) { return fmin(fmax(s, -cap), cap); }

// Limited slope on a stretched mesh: van Leer of the one-sided slopes,
// capped at twice the smaller one-sided difference over the cell's width, so
// that the one-dimensional reconstruction anywhere in the cell stays between
// the neighbours (the cap never binds on linear data, nor on unit widths);
// the divisions use the cell's precomputed reciprocals.
template <typename T>
__device__ __forceinline__ T lim_mesh(T b, T f, const Met<T>& m) {
  const T s = van_leer(b * m.ihm, f * m.ihp);
  return clamp_sym(s, fmin(fabs(b), fabs(f)) * m.iw2);
}

// ------------------------------ the reconstruction march

// The upwind, limited reconstruction (on the unit and on a stretched mesh)
// and the central one on a stretched mesh do not fit k_step's march: the
// upwind face value of each population is a non-linear function of the
// cells, so the face macros must be summed from the nine reconstructed
// values instead of reconstructed cell moments, a face reads the limited
// slopes of both its cells (a radius-two stencil), and on a stretched mesh
// every stencil carries the local widths. k_upm marches like k_step: one
// 64-lane wave owns a strip of kUpmCols = 60 columns (lanes 2..61; two halo
// lanes on each side, since an x-face reads the limited x slopes of both its
// cells and a slope reads the cell's neighbours) and marches up a segment
// of rows. Each row's limited slopes are formed once and kept in its
// record: the x slopes from the neighbouring lanes (DPP), the y slopes from
// the rows below and above when the row above is staged. Output row k needs
// rows k-2..k+2 staged, so the pass that stages row s also forms the y
// slopes of row s-1, the y-face between rows s-2 and s-1, the x-faces of row
// s-1 and the update of row s-2. The cell stage, face distributions and wall
// faces are k_step's (cell_stage / cell_core, face_df, wall_face_g).
//
// Stretched mesh: the reconstruction interpolates linearly to the face (the
// value, the tangential slope and the face inputs), slopes are derivatives
// over the centre distances, the upwind trace starts from the actual half
// width, and the update divides the fluxes by the cell's widths. On unit
// widths every formula reduces to the unit-mesh one. The central
// reconstruction's parabola slopes are cheap and are formed where used.
template <typename T, bool CPL>
struct URow {
  Cell<T> cell;
  T lxf[9], lxg[9];  // limited x slopes of the planes with e_x != 0
  T lyf[9], lyg[9];  // limited y slopes of the planes with e_y != 0
  T fsf[9], fsg[9];  // the face below the row (populations with e_y != 0)
  // the row's part of the y-face above it: the upwind traces of the
  // populations with e_y > 0, formed as soon as the row's y slopes exist
  T tdf[9], tdg[9];
};

template <typename T, bool CPL, bool WALLS, bool MESH, bool CEN>
__device__ __forceinline__ void upm_march(const CaseDev& C, const Item& it, long long n,
                                          int seg_rows) {
  static_assert(MESH || !CEN, "the central reconstruction on the unit mesh is k_step's");
  const int lane = threadIdx.x;
  const int nx = C.nx, ny = C.ny;
  constexpr int walls = WALLS ? 1 : 0;
  const int i0 = it.strip * kUpmCols;
  const int col = i0 - 2 + lane;
  const int ci = wrap(col, nx);
  const int cx = lane == 0 ? wrap(col - 1, nx) : (lane == 63 ? wrap(col + 1, nx) : ci);
  const bool store = lane >= 2 && lane <= kUpmCols + 1 && col < nx;
  const int cur = (C.cur0 + (int)(n & 1)) & 1;
  const char* in = static_cast<const char*>(cur ? C.set[1] : C.set[0]);
  char* out = static_cast<char*>(cur ? C.set[0] : C.set[1]);
  const long long RB = C.row_vals * (long long)sizeof(T);
  const long long PB = (long long)nx * sizeof(T);
  constexpr int NV = num_grouped(CPL);
  const unsigned es = sizeof(T);
  const double tn = C.t0 + (double)n * C.dt;
  const double xc = (double)ci + 0.5;
  const int j0 = it.seg * seg_rows;
  const int j1 = min(j0 + seg_rows, ny);
  const T h = ck<T>(C.f32.h, C.h), hal = T(0.5) - h;
  // stretched mesh: the metrics of the lane's column (1/hm, 1/hp, 2/w, w/2
  // and the stencil weights cp, cm, ep, em, wp, wm) through xmv(). The
  // upwind march keeps them in LDS (xm, one row per value, written once and
  // read where used through an offset the compiler cannot hoist, so that
  // they hold no registers across the march; the LDS comes from a second
  // x-face slot), the central one in registers, as does the FP64 march with
  // walls, whose LDS would then hold one wave less per CU (both measured
  // slower with the LDS copy). Those of a row (uniform over the wave) come
  // through ymet(). Y: the row metrics in the kernel's precision; Yd: the
  // double arrays, for positions (a prescribed velocity).
  constexpr bool XLDS = MESH && !CEN && !(WALLS && sizeof(T) == 8);
  // Values that a lane takes from its neighbour are mostly formed on the
  // neighbour and moved once (x differences, east traces); the FP64
  // periodic mesh march moves the inputs instead: the same bits, and
  // measured, it then does not spill.
  constexpr bool MOVE_IN = MESH && sizeof(T) == 8 && !WALLS;
  double xcen = xc, xeast = (double)ci + 1.0;
  KAxis<T> Y{};
  KAxis<double> Yd{};
  __shared__ T xm[XLDS ? 10 : 1][64];
  T xr[10] = {};
  T dBr = T(0.5);  // the east neighbour's half width (metrics in registers)
  if constexpr (MESH) {
    const KAxis<T> X = kaxis(mesh_of<T>(C), nx, ny, 0);
    const KAxis<double> Xd = kaxis(C.mesh, nx, ny, 0);
    Y = kaxis(mesh_of<T>(C), nx, ny, 1);
    Yd = kaxis(C.mesh, nx, ny, 1);
    xr[0] = X.ihm[ci];
    xr[1] = X.ihp[ci];
    xr[2] = T(2) * X.iw[ci];
    xr[3] = T(0.5) * X.w[ci];
    xr[4] = X.cp[ci];
    xr[5] = X.cm[ci];
    xr[6] = X.ep[ci];
    xr[7] = X.em[ci];
    xr[8] = X.wp[ci];
    xr[9] = X.wm[ci];
    if constexpr (XLDS) {
#pragma unroll
      for (int k = 0; k < 10; ++k) xm[k][lane] = xr[k];
    } else {
      dBr = nbr_r(xr[3]);
    }
    xcen = Xd.c[ci];
    xeast = Xd.c[ci] + 0.5 * Xd.w[ci];
  }
  auto xmv = [&](int k) {
    if constexpr (XLDS) {
      unsigned off = (unsigned)lane * (unsigned)sizeof(T);
      asm volatile("" : "+v"(off));
      return *(const T*)((const char*)&xm[k][0] + off);
    } else {
      return xr[k];
    }
  };
  // the limiter metrics of the lane's column (1/hm, 1/hp, 2/w)
  auto xmet = [&]() { return Met<T>{T(0), xmv(0), xmv(1), T(0), T(0), xmv(2)}; };
  auto ymet = [&](int r) { return Met<T>::load(Y, row_idx(r, ny, walls)); };
  // the east face of the lane's cell: the half widths of the two cells and
  // 1 / their sum (the distance to the next centre)
  struct XFace {
    T dA, dB, iH;
  };
  auto xfm = [&]() {
    if (!MESH) return XFace{T(0.5), T(0.5), T(1)};
    const T dA = xmv(3);
    return XFace{dA, XLDS ? nbr_r(dA) : dBr, xmv(1)};
  };

  __shared__ T stash[3][18][64];  // tilde-plus of the rows staged by the last three passes
  // x-faces of the last rows formed (crossing populations): two slots by
  // pass parity, or one slot with walls or the column metrics in LDS (the
  // update of a row then reads its x-faces before the next row's replace
  // them; it saves the LDS of an eighth wave per CU)
  constexpr int XS = (WALLS || XLDS) ? 1 : 2;
  __shared__ T fxs[XS][12][64];
  __shared__ T topn[6][64];       // row ny - 2, populations 2..4 (f, g): the top wall face

  struct Raw {
    T f[9], g[9], hx, hy, po, pe;
  };
  auto fetch = [&](int r, Raw& R) {
    T v[NV];
    load_groups<T, NV, true>(row_ptr(in, row_idx(r, ny, walls), RB), PB, (unsigned)ci, v);
#pragma unroll
    for (int q = 0; q < 9; ++q) R.f[q] = v[val_f(q)];
    if (CPL) {
#pragma unroll
      for (int q = 0; q < 9; ++q) R.g[q] = v[val_g(q)];
    }
    R.hx = v[val_hist(CPL, 0)];
    R.hy = v[val_hist(CPL, 1)];
    const char* prow = row_ptr(in, row_idx(r + 1, ny, walls), RB) + NV * PB;
    R.po = gload<T>(prow, lane_off((unsigned)ci * es));
    R.pe = gload<T>(prow, lane_off((unsigned)cx * es));
  };
  auto phi_lr = [&](T own, T ext, T (&o)[3]) {
    T left = nbr_l(own), right = nbr_r(own);
    if (lane == 0) left = ext;
    if (lane == 63) right = ext;
    o[0] = left; o[1] = own; o[2] = right;
  };
  auto phi_row = [&](int r, T (&o)[3]) {
    const char* prow = row_ptr(in, row_idx(r, ny, walls), RB) + NV * PB;
    phi_lr(gload<T>(prow, lane_off((unsigned)ci * es)), gload<T>(prow, lane_off((unsigned)cx * es)), o);
  };
  // x slope of the parabola through the lane's cell and its neighbours
  // (central reconstruction on a stretched mesh)
  auto xslope_c = [&](T v) { return xmv(4) * (nbr_r(v) - v) + xmv(5) * (v - nbr_l(v)); };
  // stage row r into rd (cell stage, tilde-plus to the stash slot, limited x
  // slopes, or with the central reconstruction the parabola ones)
  auto stage = [&](int r, int slot, const Raw& R, const T (&pm)[3], const T (&p0)[3],
                   const T (&pp)[3], URow<T, CPL>& rd) {
    const int rr = row_idx(r, ny, walls);
    T ph[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { ph[0][k] = pm[k]; ph[1][k] = p0[k]; ph[2][k] = pp[k]; }
    T tp[18];
    if constexpr (MESH) {
      T gx, gy, lap;
      const StW<T> wx{xmv(4), xmv(5), xmv(6), xmv(7), xmv(8), xmv(9)};
      mesh_stencils<T>(wx, StW<T>::load(Y, rr), ph, gx, gy, lap);
      cell_core<T, CPL>(C, ph[1][1], gx, gy, lap, R.f, R.g, R.hx, R.hy, xcen, Yd.c[rr], tn, rd.cell, tp);
    } else {
      cell_stage<T, CPL>(C, ph, R.f, R.g, R.hx, R.hy, xc, (double)rr + 0.5, tn, rd.cell, tp);
    }
#pragma unroll
    for (int q = 0; q < 18; ++q) stash[slot][q][lane] = tp[q];
    if (WALLS && r == ny - 2) {  // every segment that outputs row ny - 1 stages row ny - 2
#pragma unroll
      for (int q = 2; q <= 4; ++q) {
        topn[q - 2][lane] = rd.cell.fb[q];
        topn[1 + q][lane] = rd.cell.gb[q];
      }
    }
    Met<T> mx{};
    if (MESH && !CEN) mx = xmet();
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (EX[q] == 0) continue;
      if constexpr (CEN) {
        rd.lxf[q] = xslope_c(rd.cell.fb[q]);
        if (CPL) rd.lxg[q] = xslope_c(rd.cell.gb[q]);
        continue;
      }
      // the backward difference of a lane is the forward one of the lane
      // before it (the same subtraction, taken from that lane; see MOVE_IN)
      auto lim = [&](T c) {
        const T fwd = nbr_r(c) - c;
        const T bwd = MOVE_IN ? c - nbr_l(c) : nbr_l(fwd);
        return MESH ? lim_mesh<T>(bwd, fwd, mx) : van_leer(bwd, fwd);
      };
      rd.lxf[q] = lim(rd.cell.fb[q]);
      if (CPL) rd.lxg[q] = lim(rd.cell.gb[q]);
    }
  };
  // x central differences (stretched mesh: x slopes of the parabola) of the
  // diagonal planes of a wall row (wall faces)
  auto xdiffs = [&](const Cell<T>& c, T (&txf)[9], T (&txg)[9]) {
    const T cpx = MESH ? xmv(4) : T(0), cmx = MESH ? xmv(5) : T(0);
    auto d = [&](T v) {
      if (MESH) return cpx * (nbr_r(v) - v) + cmx * (v - nbr_l(v));
      return nbr_r(v) - nbr_l(v);
    };
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      txf[q] = T(0);
      txg[q] = T(0);
      if (EX[q] == 0 || EY[q] == 0) continue;
      txf[q] = d(c.fb[q]);
      if (CPL) txg[q] = d(c.gb[q]);
    }
  };
  // limited y slopes of row r (record m) from the rows below (d) and above
  // (u); one-sided and unlimited at a wall row
  auto yslopes = [&](int r, const URow<T, CPL>& d, URow<T, CPL>& m, const URow<T, CPL>& u) {
    Met<T> my{};
    if (MESH) my = ymet(r);
    // from the row's centre to its upper face, less h (the trace of a
    // population leaving upwards)
    const T up = MESH ? T(0.5) * my.w - h : hal;
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (EY[q] == 0) continue;
      const T c = m.cell.fb[q];
      const T cg = CPL ? m.cell.gb[q] : T(0);
      if (WALLS && r == 0) {
        m.lyf[q] = u.cell.fb[q] - c;
        if (CPL) m.lyg[q] = u.cell.gb[q] - cg;
        if (MESH) {
          m.lyf[q] = m.lyf[q] * my.ihp;
          if (CPL) m.lyg[q] = m.lyg[q] * my.ihp;
        }
      } else if (WALLS && r == ny - 1) {
        m.lyf[q] = c - d.cell.fb[q];
        if (CPL) m.lyg[q] = cg - d.cell.gb[q];
        if (MESH) {
          m.lyf[q] = m.lyf[q] * my.ihm;
          if (CPL) m.lyg[q] = m.lyg[q] * my.ihm;
        }
      } else if (MESH) {
        m.lyf[q] = lim_mesh<T>(c - d.cell.fb[q], u.cell.fb[q] - c, my);
        if (CPL) m.lyg[q] = lim_mesh<T>(cg - d.cell.gb[q], u.cell.gb[q] - cg, my);
      } else {
        m.lyf[q] = van_leer(c - d.cell.fb[q], u.cell.fb[q] - c);
        if (CPL) m.lyg[q] = van_leer(cg - d.cell.gb[q], u.cell.gb[q] - cg);
      }
      if (EY[q] > 0) {  // the lower cell's traces of the y-face above the row
        T v = c + up * m.lyf[q];
        if (EX[q] != 0) v -= h * T(EX[q]) * m.lxf[q];
        m.tdf[q] = v;
        if (CPL) {
          T w = cg + up * m.lyg[q];
          if (EX[q] != 0) w -= h * T(EX[q]) * m.lxg[q];
          m.tdg[q] = w;
        }
      }
    }
  };
  // the x-face east of each cell of row r (record m; the east cell is lane + 1)
  // into LDS
  auto xface = [&](int r, int xs, const URow<T, CPL>& m) {
    const XFace xf = xfm();
    const T dAx = xf.dA, dBx = xf.dB, iHx = xf.iH;
    T fbar[9], gbar[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int en = EX[q], et = EY[q];
      // a trace that starts in the east cell is formed on the east lane
      // and moved over once (the same arithmetic as on this lane; see
      // MOVE_IN)
      auto rec = [&](const T& a, const T& lx, const T& ly) {
        if constexpr (MESH && !MOVE_IN) {
          if (en > 0) {
            T v = a + (dAx - h) * lx;
            if (et != 0) v -= h * T(et) * ly;
            return v;
          }
          if (en < 0) {
            T v = a + (h - dAx) * lx;
            if (et != 0) v -= h * T(et) * ly;
            return nbr_r(v);
          }
          T vA = a;
          if (et != 0) vA -= h * T(et) * ly;
          return (dBx * vA + dAx * nbr_r(vA)) * iHx;
        } else if constexpr (MESH) {
          if (en > 0) {
            T v = a + (dAx - h) * lx;
            if (et != 0) v -= h * T(et) * ly;
            return v;
          }
          if (en < 0) {
            T v = nbr_r(a) + (h - dBx) * nbr_r(lx);
            if (et != 0) v -= h * T(et) * nbr_r(ly);
            return v;
          }
          T vA = a, vB = nbr_r(a);
          if (et != 0) {
            vA -= h * T(et) * ly;
            vB -= h * T(et) * nbr_r(ly);
          }
          return (dBx * vA + dAx * vB) * iHx;
        } else {
          if (en > 0) {
            T v = a + hal * lx;
            if (et != 0) v -= h * T(et) * ly;
            return v;
          }
          if (en < 0) {
            T v = a - hal * lx;
            if (et != 0) v -= h * T(et) * ly;
            return nbr_r(v);
          }
          T v = T(0.5) * (a + nbr_r(a));
          if (et != 0) v -= h * T(et) * (T(0.5) * (ly + nbr_r(ly)));
          return v;
        }
      };
      fbar[q] = rec(m.cell.fb[q], m.lxf[q], m.lyf[q]);
      gbar[q] = (CPL && q > 0) ? rec(m.cell.gb[q], m.lxg[q], m.lyg[q]) : T(0);
    }
    const T phif = (fbar[0] + ((fbar[1] + fbar[2]) + (fbar[3] + fbar[4]))) +
                   ((fbar[5] + fbar[6]) + (fbar[7] + fbar[8]));
    T N0f = T(0), Jxf = T(0), Jyf = T(0);
    if (CPL) {
      N0f = ((gbar[1] + gbar[2]) + (gbar[3] + gbar[4])) + ((gbar[5] + gbar[6]) + (gbar[7] + gbar[8]));
      Jxf = (gbar[1] + gbar[2] + gbar[8]) - (gbar[4] + gbar[5] + gbar[6]);
      Jyf = (gbar[2] + gbar[3] + gbar[4]) - (gbar[6] + gbar[7] + gbar[8]);
    }
    const Cell<T>& a = m.cell;
    // face inputs: the mean of the two cells (linear interpolation to the
    // face on a stretched mesh)
    auto mean = [&](T v) {
      if (MESH) return (dBx * v + dAx * nbr_r(v)) * iHx;
      return T(0.5) * (v + nbr_r(v));
    };
    const int rr = row_idx(r, ny, walls);
    T fo[9], go[9];
    face_df<T, CPL, 0>(C, phif, N0f, Jxf, Jyf, mean(a.gx), mean(a.gy), mean(a.mu), mean(a.Dx),
                       mean(a.Dy), fbar, gbar, xeast, MESH ? Yd.c[rr] : (double)rr + 0.5,
                       tn + C.h, fo, go);
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (EX[q] == 0) continue;
      fxs[xs][up_xslot(q)][lane] = fo[q];
      if (CPL) fxs[xs][6 + up_xslot(q)][lane] = go[q];
    }
  };
  // the y-face between rows r (record d, below) and r + 1 (record u), into
  // u's face below
  auto yface = [&](int r, const URow<T, CPL>& d, URow<T, CPL>& u) {
    // half heights of the two rows and 1 / their sum (stretched mesh)
    T dA = T(0.5), dB = T(0.5), iH = T(1);
    if (MESH) {
      const Met<T> ma = ymet(r);
      dA = T(0.5) * ma.w;
      dB = T(0.5) * ymet(r + 1).w;
      iH = ma.ihp;  // 1 / (dA + dB)
    }
    T fbar[9], gbar[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int en = EY[q], et = EX[q];
      auto rec = [&](const T& tD, const T& aD, const T& lxD, const T& aU, const T& lyU,
                     const T& lxU) {
        if (en > 0) return tD;  // formed with the lower row's y slopes
        if constexpr (MESH) {
          if (en < 0) {
            T v = aU + (h - dB) * lyU;
            if (et != 0) v -= h * T(et) * lxU;
            return v;
          }
          T vA = aD, vB = aU;
          if (et != 0) {
            vA -= h * T(et) * lxD;
            vB -= h * T(et) * lxU;
          }
          return (dB * vA + dA * vB) * iH;
        } else {
          if (en < 0) {
            T v = aU - hal * lyU;
            if (et != 0) v -= h * T(et) * lxU;
            return v;
          }
          T v = T(0.5) * (aD + aU);
          if (et != 0) v -= h * T(et) * (T(0.5) * (lxD + lxU));
          return v;
        }
      };
      fbar[q] = rec(d.tdf[q], d.cell.fb[q], d.lxf[q], u.cell.fb[q], u.lyf[q], u.lxf[q]);
      gbar[q] = (CPL && q > 0)
                    ? rec(d.tdg[q], d.cell.gb[q], d.lxg[q], u.cell.gb[q], u.lyg[q], u.lxg[q])
                    : T(0);
    }
    const T phif = (fbar[0] + ((fbar[1] + fbar[2]) + (fbar[3] + fbar[4]))) +
                   ((fbar[5] + fbar[6]) + (fbar[7] + fbar[8]));
    T N0f = T(0), Jxf = T(0), Jyf = T(0);
    if (CPL) {
      N0f = ((gbar[1] + gbar[2]) + (gbar[3] + gbar[4])) + ((gbar[5] + gbar[6]) + (gbar[7] + gbar[8]));
      Jxf = (gbar[1] + gbar[2] + gbar[8]) - (gbar[4] + gbar[5] + gbar[6]);
      Jyf = (gbar[2] + gbar[3] + gbar[4]) - (gbar[6] + gbar[7] + gbar[8]);
    }
    const Cell<T>& a = d.cell;
    const Cell<T>& b = u.cell;
    auto mean = [&](T va, T vb) {
      if (MESH) return (dB * va + dA * vb) * iH;
      return T(0.5) * (va + vb);
    };
    const int rr = row_idx(r, ny, walls);
    face_df<T, CPL, 1>(C, phif, N0f, Jxf, Jyf, mean(a.gx, b.gx), mean(a.gy, b.gy),
                       mean(a.mu, b.mu), mean(a.Dx, b.Dx), mean(a.Dy, b.Dy), fbar, gbar, xcen,
                       MESH ? Yd.c[rr] + 0.5 * Yd.w[rr] : (double)rr + 1.0, tn + C.h, u.fsf, u.fsg);
  };
  // Central reconstruction on a stretched mesh: the face value is the
  // interpolation of the two cells less h xi times the normal difference and
  // the interpolated tangential slope (terms whose velocity component is
  // zero are left out). The parabola slopes: the x slopes of a row are
  // formed once when it is staged (in its record, for the y-faces below and
  // above it), the y slopes of row r from the rows below (d) and above (u)
  // where its x-face uses them.
  auto yslope_c = [&](int r, T dv, T cv, T uv, const Met<T>& my) {
    if (WALLS && r == 0) return (uv - cv) * my.ihp;
    if (WALLS && r == ny - 1) return (cv - dv) * my.ihm;
    return my.cp * (uv - cv) + my.cm * (cv - dv);
  };
  auto xface_c = [&](int r, int xs, const URow<T, CPL>& d, const URow<T, CPL>& m,
                     const URow<T, CPL>& u) {
    const Met<T> my = ymet(r);
    const XFace xf = xfm();
    const T dA = xf.dA, dB = xf.dB, iH = xf.iH;
    auto rec = [&](int q, T dv, T a, T uv) {
      const T aB = nbr_r(a);
      const T af = (dB * a + dA * aB) * iH;
      if (EX[q] == 0 && EY[q] == 0) return af;
      const T dn = (aB - a) * iH;
      if (EY[q] == 0) return af - h * (T(EX[q]) * dn);
      const T st = yslope_c(r, dv, a, uv, my);
      const T dtg = (dB * st + dA * nbr_r(st)) * iH;
      if (EX[q] == 0) return af - h * (T(EY[q]) * dtg);
      return af - h * (T(EX[q]) * dn + T(EY[q]) * dtg);
    };
    T fbar[9], gbar[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      fbar[q] = rec(q, d.cell.fb[q], m.cell.fb[q], u.cell.fb[q]);
      gbar[q] = (CPL && q > 0) ? rec(q, d.cell.gb[q], m.cell.gb[q], u.cell.gb[q]) : T(0);
    }
    const T phif = (fbar[0] + ((fbar[1] + fbar[2]) + (fbar[3] + fbar[4]))) +
                   ((fbar[5] + fbar[6]) + (fbar[7] + fbar[8]));
    T N0f = T(0), Jxf = T(0), Jyf = T(0);
    if (CPL) {
      N0f = ((gbar[1] + gbar[2]) + (gbar[3] + gbar[4])) + ((gbar[5] + gbar[6]) + (gbar[7] + gbar[8]));
      Jxf = (gbar[1] + gbar[2] + gbar[8]) - (gbar[4] + gbar[5] + gbar[6]);
      Jyf = (gbar[2] + gbar[3] + gbar[4]) - (gbar[6] + gbar[7] + gbar[8]);
    }
    const Cell<T>& a = m.cell;
    auto mean = [&](T v) { return (dB * v + dA * nbr_r(v)) * iH; };
    const int rr = row_idx(r, ny, walls);
    T fo[9], go[9];
    face_df<T, CPL, 0>(C, phif, N0f, Jxf, Jyf, mean(a.gx), mean(a.gy), mean(a.mu), mean(a.Dx),
                       mean(a.Dy), fbar, gbar, xeast, Yd.c[rr], tn + C.h, fo, go);
#pragma unroll
    for (int q = 1; q < 9; ++q) {
      if (EX[q] == 0) continue;
      fxs[xs][up_xslot(q)][lane] = fo[q];
      if (CPL) fxs[xs][6 + up_xslot(q)][lane] = go[q];
    }
  };
  auto yface_c = [&](int r, const URow<T, CPL>& d, URow<T, CPL>& u) {
    const Met<T> ma = ymet(r);
    const T dA = T(0.5) * ma.w, dB = T(0.5) * ymet(r + 1).w;
    const T iH = ma.ihp;  // 1 / (dA + dB)
    auto rec = [&](int q, T aA, T aB, T sA, T sB) {
      const T af = (dB * aA + dA * aB) * iH;
      if (EX[q] == 0 && EY[q] == 0) return af;
      const T dn = (aB - aA) * iH;
      if (EX[q] == 0) return af - h * (T(EY[q]) * dn);
      const T dtg = (dB * sA + dA * sB) * iH;
      if (EY[q] == 0) return af - h * (T(EX[q]) * dtg);
      return af - h * (T(EY[q]) * dn + T(EX[q]) * dtg);
    };
    T fbar[9], gbar[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      fbar[q] = rec(q, d.cell.fb[q], u.cell.fb[q], d.lxf[q], u.lxf[q]);
      gbar[q] = (CPL && q > 0) ? rec(q, d.cell.gb[q], u.cell.gb[q], d.lxg[q], u.lxg[q]) : T(0);
    }
    const T phif = (fbar[0] + ((fbar[1] + fbar[2]) + (fbar[3] + fbar[4]))) +
                   ((fbar[5] + fbar[6]) + (fbar[7] + fbar[8]));
    T N0f = T(0), Jxf = T(0), Jyf = T(0);
    if (CPL) {
      N0f = ((gbar[1] + gbar[2]) + (gbar[3] + gbar[4])) + ((gbar[5] + gbar[6]) + (gbar[7] + gbar[8]));
      Jxf = (gbar[1] + gbar[2] + gbar[8]) - (gbar[4] + gbar[5] + gbar[6]);
      Jyf = (gbar[2] + gbar[3] + gbar[4]) - (gbar[6] + gbar[7] + gbar[8]);
    }
    const Cell<T>& a = d.cell;
    const Cell<T>& b = u.cell;
    auto mean = [&](T va, T vb) { return (dB * va + dA * vb) * iH; };
    const int rr = row_idx(r, ny, walls);
    face_df<T, CPL, 1>(C, phif, N0f, Jxf, Jyf, mean(a.gx, b.gx), mean(a.gy, b.gy),
                       mean(a.mu, b.mu), mean(a.Dx, b.Dx), mean(a.Dy, b.Dy), fbar, gbar, xcen,
                       Yd.c[rr] + 0.5 * Yd.w[rr], tn + C.h, u.fsf, u.fsg);
  };

  // update of output row r (record m) from its faces: east m.fx, west the
  // left lane's, below m.fs, above (fnf, fng)
  auto update = [&](int r, int slot, int xs, const URow<T, CPL>& m, const T (&fnf)[9],
                    const T (&fng)[9]) {
    const int rr = row_idx(r, ny, walls);
    char* orow = row_ptr(out, rr, RB);
    const T dt = ck<T>(C.f32.dt, C.dt);
    // face length over cell area: 1/dx and 1/dy (1 on unit cells)
    const T ay = MESH ? Y.iw[rr] : T(1);
    const T axw = MESH ? T(0.5) * xmv(2) : T(1);  // 1 / w of the lane's column
    // the flux difference of population q (plane off: 0 f, 6 g) from its
    // east/west and upper/lower faces
    auto flux = [&](int q, int off, T fn, T fs) {
      if constexpr (MESH) {
        T Jx = T(0), Jy = T(0);
        if (EX[q] != 0) {
          const T e = fxs[xs][off + up_xslot(q)][lane];
          Jx = T(EX[q]) * (e - nbr_l(e));
        }
        if (EY[q] != 0) Jy = T(EY[q]) * (fn - fs);
        return axw * Jx + ay * Jy;
      } else {
        T J = T(0);
        if (EX[q] != 0) {
          // the west face through the LDS crossbar (xl) in the coupled
          // model: 1.2% faster here, slower on the stretched mesh
          const T e = fxs[xs][off + up_xslot(q)][lane];
          J += T(EX[q]) * (e - xl<CPL>(e));
        }
        if (EY[q] != 0) J += T(EY[q]) * (fn - fs);
        return J;
      }
    };
    T nv[NV];
    T phin = T(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      nv[val_f(q)] = stash[slot][q][lane] - dt * flux(q, 0, fnf[q], m.fsf[q]);
      phin += nv[val_f(q)];
    }
    if (CPL) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        nv[val_g(q)] = stash[slot][9 + q][lane] - dt * flux(q, 6, fng[q], m.fsg[q]);
    }
    nv[val_hist(CPL, 0)] = m.cell.hx;
    nv[val_hist(CPL, 1)] = m.cell.hy;
    if (store) {
      store_groups<T, NV, true>(orow, PB, (unsigned)ci, nv);
      gstore<T>(orow + NV * PB, lane_off((unsigned)ci * es), phin);
      flag_nonfinite(C, phin + m.cell.hx + m.cell.hy);
    }
  };

  // One pass: stage row s into R1; y slopes of row s - 1 (R0); the y-face
  // between rows s - 2 (Rm) and s - 1; the x-faces of row s - 1; the update
  // of row s - 2. p is the pass index (stash slots rotate by three).
  auto pass = [&](int s, int p, Raw& raw, URow<T, CPL>& Rm, URow<T, CPL>& R0, URow<T, CPL>& R1,
                  const T (&pa)[3], const T (&pb)[3], T (&pc)[3]) {
    const int slot = p % 3;
    phi_lr(raw.po, raw.pe, pc);
    const bool ex1 = !(walls && (s < 0 || s >= ny));
    const int r0 = s - 1, rm = s - 2;
    const bool ex0 = !(walls && (r0 < 0 || r0 >= ny));
    const bool exm = !(walls && (rm < 0 || rm >= ny));
    // central: the y-face between rows s - 2 and s - 1 needs neither row s
    // nor its slopes, so it comes first and the lower row's x slopes die
    // before row s's are formed
    const bool yf = rm >= j0 - 1 && rm < j1 && ex0 && exm;
    if (CEN && yf) yface_c(rm, Rm, R0);
    if (ex1) stage(s, slot, raw, pa, pb, pc, R1);
    fetch(min(s + 2, j1 + 1), raw);
    if (!CEN && ex0 && r0 >= j0 - 1) yslopes(r0, Rm, R0, R1);
    if (XS == 2 && r0 >= j0 && r0 < j1) {
      if constexpr (CEN) xface_c(r0, p & 1, Rm, R0, R1);
      else xface(r0, p & 1, R0);
    }
    // the face below row s - 1: between rows s - 2 and s - 1, or the bottom wall
    if (rm >= j0 - 1 && rm < j1) {
      if (ex0 && exm) {
        if constexpr (!CEN) yface(rm, Rm, R0);
      } else if (WALLS && rm == -1) {
        T txf[9], txg[9];
        xdiffs(R0.cell, txf, txg);
        T dyw = T(0), idy = T(1);
        if (MESH) {
          const Met<T> m0 = ymet(0);
          dyw = T(-0.5) * m0.w;
          idy = m0.ihp;
        }
        wall_face_g<T, true, MESH>(C, R0.cell, R1.cell, txf, txg, dyw, idy, R0.fsf, R0.fsg);
      }
    }
    // the update of row s - 2 (with one x-face slot it reads its x-faces
    // from LDS before the x-faces of row s - 1 replace them)
    if (rm >= j0 && rm < j1) {
      const int ms = (p + 1) % 3;  // slot of row s - 2
      const int xs = XS == 1 ? 0 : (p + 1) & 1;
      if (WALLS && rm == ny - 1) {
        // top wall: the next row inward (row ny - 2) from LDS
        Cell<T> cn;
#pragma unroll
        for (int q = 2; q <= 4; ++q) {
          cn.fb[q] = topn[q - 2][lane];
          cn.gb[q] = topn[1 + q][lane];
        }
        T txf[9], txg[9], fnf[9], fng[9];
        xdiffs(Rm.cell, txf, txg);
        T dyw = T(0), idy = T(1);
        if (MESH) {
          const Met<T> mt = ymet(ny - 1);
          dyw = T(0.5) * mt.w;
          idy = mt.ihm;
        }
        wall_face_g<T, false, MESH>(C, Rm.cell, cn, txf, txg, dyw, idy, fnf, fng);
        update(rm, ms, xs, Rm, fnf, fng);
      } else {
        update(rm, ms, xs, Rm, R0.fsf, R0.fsg);
      }
    }
    if (XS == 1 && ex0 && r0 >= j0 && r0 < j1) {
      if constexpr (CEN) xface_c(r0, 0, Rm, R0, R1);
      else xface(r0, 0, R0);
    }
  };

  URow<T, CPL> R0, R1, R2;
  T P0[3], P1[3], P2[3];
  auto rotate = [&]() {
    R0 = R1;
    R1 = R2;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      P0[m] = P1[m];
      P1[m] = P2[m];
    }
  };
  Raw ra, rb;
  const int kb = j0 - 2;
  const int npass = j1 - j0 + 4;
  phi_row(kb - 1, P0);
  phi_row(kb, P1);
  fetch(kb, ra);
  fetch(kb + 1, rb);
  for (int m = 0; m < npass; m += 2) {
    pass(kb + m, m, ra, R0, R1, R2, P0, P1, P2);
    rotate();
    if (m + 1 < npass) {
      pass(kb + m + 1, m + 1, rb, R0, R1, R2, P0, P1, P2);
      rotate();
    }
  }
}

template <typename T, bool CPL, bool WALLS, bool MESH, bool CEN>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? 2 : 1) void k_upm(StepArgs A) {
  const int nb = gridDim.x;
  const int per = nb >> 3;  // grid is a multiple of 8 (one share per XCD)
  const int idx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (idx >= A.nitems) return;
  const Item it = A.items[idx];
  CaseDev C = A.cases[it.c];
  if (!MESH && !WALLS) narrow_in_kernel(C);
  const long long n = *A.step_base + A.kofs - C.step0;
  if (n < 0 || n >= C.nsteps) return;
  upm_march<T, CPL, WALLS, MESH, CEN>(C, it, n, A.upm_rows);
}

}  // namespace

// ----------------------------------------------------------------- launchers

hipError_t launch_step(bool fp64, bool coupled, bool walls, const StepArgs& a, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  const int per = (a.nitems + 7) / 8;
  if (walls && !coupled) return hipErrorInvalidValue;
  if (a.two_row && !fp64 && !walls) {  // four waves per two-row tile
    dim3 grid(per * 8), block(4 * kWave);
    if (!coupled) hipLaunchKernelGGL((k_step_row2<float, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step_row2<float, true>), grid, block, 0, s, a);
    return hipGetLastError();
  }
  if (a.one_row) {  // three waves per one-row tile
    dim3 grid(per * 8), block(3 * kWave);
    if (fp64) {
      if (!coupled) hipLaunchKernelGGL((k_step_row<double, false, false>), grid, block, 0, s, a);
      else if (walls) hipLaunchKernelGGL((k_step_row<double, true, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_step_row<double, true, false>), grid, block, 0, s, a);
    } else {
      if (!coupled) hipLaunchKernelGGL((k_step_row<float, false, false>), grid, block, 0, s, a);
      else if (walls) hipLaunchKernelGGL((k_step_row<float, true, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_step_row<float, true, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
  }
  dim3 grid(per * 8), block(kWave);
  if (fp64) {
    if (!coupled) hipLaunchKernelGGL((k_step<double, false, false>), grid, block, 0, s, a);
    else if (walls) hipLaunchKernelGGL((k_step<double, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step<double, true, false>), grid, block, 0, s, a);
  } else {
    if (!coupled) hipLaunchKernelGGL((k_step<float, false, false>), grid, block, 0, s, a);
    else if (walls) hipLaunchKernelGGL((k_step<float, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_step<float, true, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, bool M, bool CEN>
static void launch_upm(bool coupled, bool walls, const StepArgs& a, hipStream_t s) {
  const dim3 grid((a.nitems + 7) / 8 * 8), block(kWave);
  if (!coupled) hipLaunchKernelGGL((k_upm<T, false, false, M, CEN>), grid, block, 0, s, a);
  else if (walls) hipLaunchKernelGGL((k_upm<T, true, true, M, CEN>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_upm<T, true, false, M, CEN>), grid, block, 0, s, a);
}
template <typename T>
static void launch_upm_modes(bool coupled, bool walls, bool mesh, bool central, const StepArgs& a,
                             hipStream_t s) {
  if (!mesh) launch_upm<T, false, false>(coupled, walls, a, s);
  else if (central) launch_upm<T, true, true>(coupled, walls, a, s);
  else launch_upm<T, true, false>(coupled, walls, a, s);
}

hipError_t launch_step_upm(bool fp64, bool coupled, bool walls, bool mesh, bool central,
                           const StepArgs& a, hipStream_t s) {
  if (a.nitems <= 0) return hipSuccess;
  if (walls && !coupled) return hipErrorInvalidValue;
  if (central && !mesh) return hipErrorInvalidValue;  // k_step covers that case
  if (fp64) launch_upm_modes<double>(coupled, walls, mesh, central, a, s);
  else launch_upm_modes<float>(coupled, walls, mesh, central, a, s);
  return hipGetLastError();
}

template <typename T, bool M, bool CEN>
static int upm_occupancy(bool coupled, bool walls) {
  int nb = 0;
  hipError_t e;
  auto occ = [&](const void* k) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kWave, 0);
  };
  if (!coupled) e = occ((const void*)k_upm<T, false, false, M, CEN>);
  else if (walls) e = occ((const void*)k_upm<T, true, true, M, CEN>);
  else e = occ((const void*)k_upm<T, true, false, M, CEN>);
  return e == hipSuccess && nb > 0 ? nb : 1;
}
template <typename T>
static int upm_occupancy_modes(bool coupled, bool walls, bool mesh, bool central) {
  if (!mesh) return upm_occupancy<T, false, false>(coupled, walls);
  return central ? upm_occupancy<T, true, true>(coupled, walls)
                 : upm_occupancy<T, true, false>(coupled, walls);
}
int upm_waves_per_cu(bool fp64, bool coupled, bool walls, bool mesh, bool central) {
  return fp64 ? upm_occupancy_modes<double>(coupled, walls, mesh, central)
              : upm_occupancy_modes<float>(coupled, walls, mesh, central);
}

// Resident waves per CU of the step kernel (one wave per work group).
int step_waves_per_cu(bool fp64, bool coupled, bool walls) {
  int nb = 0;
  hipError_t e;
  auto occ = [&](const void* k) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kWave, 0); };
  if (fp64) {
    if (!coupled) e = occ((const void*)k_step<double, false, false>);
    else if (walls) e = occ((const void*)k_step<double, true, true>);
    else e = occ((const void*)k_step<double, true, false>);
  } else {
    if (!coupled) e = occ((const void*)k_step<float, false, false>);
    else if (walls) e = occ((const void*)k_step<float, true, true>);
    else e = occ((const void*)k_step<float, true, false>);
  }
  return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_advance(long long* step_base, long long by, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, step_base, by);
  return hipGetLastError();
}

hipError_t launch_reset(long long* step_base, long long value, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, step_base, value, flag);
  return hipGetLastError();
}

hipError_t launch_init(bool fp64, const CaseDev* dcase, const CaseDev& hc, const double* phi,
                       const double* u, const double* v, const double* p, hipStream_t s) {
  dim3 block(128), grid((hc.nx + 127) / 128, hc.ny);
  const int buf = hc.cur0;
  if (fp64) {
    if (hc.coupled) hipLaunchKernelGGL((k_init<double, true>), grid, block, 0, s, dcase, buf, phi, u, v, p);
    else hipLaunchKernelGGL((k_init<double, false>), grid, block, 0, s, dcase, buf, phi, u, v, p);
  } else {
    if (hc.coupled) hipLaunchKernelGGL((k_init<float, true>), grid, block, 0, s, dcase, buf, phi, u, v, p);
    else hipLaunchKernelGGL((k_init<float, false>), grid, block, 0, s, dcase, buf, phi, u, v, p);
  }
  return hipGetLastError();
}

hipError_t launch_macros(bool fp64, const CaseDev* dcase, const CaseDev& hc, long long local_step,
                         double* phi, double* u, double* v, double* p, double* rho, hipStream_t s) {
  dim3 block(128), grid((hc.nx + 127) / 128, hc.ny);
  const int buf = (hc.cur0 + (int)(local_step & 1)) & 1;
  const double t = hc.t0 + (double)local_step * hc.dt;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, dcase, buf, t, phi, u, v, p, rho);
  };
  if (fp64) {
    if (hc.coupled) go(k_macros<double, true>);
    else go(k_macros<double, false>);
  } else {
    if (hc.coupled) go(k_macros<float, true>);
    else go(k_macros<float, false>);
  }
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address).
hipError_t noalloc_scratch(double** ptr, int* max_rows) {
  static std::mutex lock;
  static double* addr[256] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  *max_rows = kNoAllocRows;
  return hipSuccess;
}

hipError_t launch_diag_noalloc(bool fp64, const CaseDev* dcase, const CaseDev& hc,
                               long long local_step, double* part, double* out, hipStream_t s) {
  if (hc.ny > kNoAllocRows) return hipErrorInvalidValue;
  const int buf = (hc.cur0 + (int)(local_step & 1)) & 1;
  const double t = hc.t0 + (double)local_step * hc.dt;
  dim3 grid(hc.ny), block(kDiagThreads);
  if (fp64) {
    if (hc.coupled) hipLaunchKernelGGL((k_diag_rows<double, true>), grid, block, 0, s, dcase, buf, t, part);
    else hipLaunchKernelGGL((k_diag_rows<double, false>), grid, block, 0, s, dcase, buf, t, part);
  } else {
    if (hc.coupled) hipLaunchKernelGGL((k_diag_rows<float, true>), grid, block, 0, s, dcase, buf, t, part);
    else hipLaunchKernelGGL((k_diag_rows<float, false>), grid, block, 0, s, dcase, buf, t, part);
  }
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, hc.ny, part, out);
  return hipGetLastError();
}

hipError_t launch_diag(const CaseDev& hc, const double* phi, const double* u, const double* v,
                       const double* rho, double* partial, int npartial, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_diag_partial, dim3(npartial), dim3(kDiagThreads), 0, s, hc.nx, hc.ny, phi,
                     u, v, rho, partial);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, npartial, partial, out);
  return hipGetLastError();
}

}  // namespace dugks
