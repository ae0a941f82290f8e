// C ABI of libdugks (declared in include/dugks.h): handle life cycle,
// parameter validation and derived constants, initialisation, stepping,
// readout, diagnostics, checkpoints and batches (with HIP graphs).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>


#include "dugks_host.h"

using dugks::CaseDev;
using dugks::Item;
using dugks::StepArgs;

namespace dugks {
namespace host {

thread_local std::string g_create_error = "no error";

int fail(dugks_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

int hip_fail(dugks_handle* h, hipError_t e, const char* what) {
  return fail(h, DUGKS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Resident step waves on the current device (CUs x waves per CU).
int wave_capacity(bool fp64, bool coupled, bool walls) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 2048;
  }
  return prop.multiProcessorCount * dugks::step_waves_per_cu(fp64, coupled, walls);
}

// Compute units of the current device (256 if it cannot be queried).
long long cu_count() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 256;
  }
  return prop.multiProcessorCount;
}

// Waves (tiles) of a list of cases cut into segments of `seg` rows.
long long tile_count(const std::vector<StripShape>& cs, int seg) {
  long long w = 0;
  for (const auto& c : cs) w += (long long)c.nstrips * ((c.ny + seg - 1) / seg);
  return w;
}

// The shortest segment (at most 4096 rows) whose tiles number at most
// `budget`: with budget = the device's resident-wave capacity, every tile
// starts at once and none is left to run alone in a second round, at the
// least repeated work (each segment stages two halo rows twice).
int fit_seg_rows(const std::vector<StripShape>& cs, long long budget) {
  int hi = 1;
  for (const auto& c : cs) hi = std::max(hi, std::min(c.ny, 4096));
  if (tile_count(cs, hi) > budget) return hi;
  int lo = 1;
  while (lo < hi) {  // smallest seg with tile_count(seg) <= budget (count is non-increasing)
    const int mid = lo + (hi - lo) / 2;
    if (tile_count(cs, mid) <= budget) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Automatic segment length: one round of resident waves (fit_seg_rows) for
// most grids; when that needs segments longer than 64 rows (grids far larger
// than the device caches) eight rounds of shorter tiles, which keeps the
// rows in flight closer together and measured faster on MI355X (4096^2
// FP32 coupled: 23.4k MLUPS with 137-row segments, 26.8k with 17).
// The reconstruction march takes one round of resident waves with its own strips
// (60 columns) and capacity; where that needs segments longer than 64 rows,
// the shortest segments that number at most 32 waves per CU. Measured on
// MI355X (microseconds per step, upwind bubble): 4096^2 FP32 18 rows 655,
// 24 638, 32 634, 48 641, 64 699; FP64 16 rows 1613, 35 1484, 48 1494,
// 64 1635; the one-round choice is the fastest at 1024^2 (10 rows), 128^2
// (1 row) and 256 x 1024 with walls (3 rows).
int auto_upm_rows(const dugks_handle* h) {
  int dev = 0;
  hipDeviceProp_t prop;
  long long cus = 256, cap = 2048;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    cus = prop.multiProcessorCount;
    cap = cus * dugks::upm_waves_per_cu(h->fp64(), h->coupled(), h->params.bc_y == DUGKS_BC_WALLS,
                                        h->mesh, !h->upwind());
  } else {
    (void)hipGetLastError();
  }
  const std::vector<StripShape> cs = {
      StripShape{(h->nx + dugks::kUpmCols - 1) / dugks::kUpmCols, h->ny}};
  const int a = fit_seg_rows(cs, cap);
  return a > 64 ? fit_seg_rows(cs, 32 * cus) : a;
}

int auto_seg_rows(const std::vector<StripShape>& cs, long long capacity, bool fp64, bool walls) {
  const int a = fit_seg_rows(cs, capacity);
  if (a > 64) return fit_seg_rows(cs, 8 * capacity);
  if (a == 1 && !fp64 && !walls) {
    // one-row tiles that outnumber the CUs put two work groups (six waves)
    // on some CUs, whose waves then share SIMDs; two-row tiles that fit one
    // per CU run the four-wave two-row kernel instead (128^2: 5.0 against
    // 5.2 us per step)
    const long long cus = cu_count();
    if (tile_count(cs, 1) > cus && tile_count(cs, 2) <= cus) return 2;
  }
  return a;
}

// Derived constants (Sec. II.B, Eqs. 3, 28-29, 34, 37) into the descriptor.
void fill_case(dugks_handle* h) {
  CaseDev& C = h->hc;
  const dugks_params& P = h->params;
  C.nx = h->nx;
  C.ny = h->ny;
  C.coupled = h->coupled() ? 1 : 0;
  C.nstrips = (h->nx + dugks::kStripCols - 1) / dugks::kStripCols;
  C.walls = P.bc_y == DUGKS_BC_WALLS ? 1 : 0;
  C.seg_rows = h->seg_rows > 0
                   ? h->seg_rows
                   : auto_seg_rows({StripShape{C.nstrips, h->ny}},
                                   wave_capacity(h->fp64(), h->coupled(), C.walls != 0),
                                   h->fp64(), C.walls != 0);
  C.nsegs = (h->ny + C.seg_rows - 1) / C.seg_rows;
  C.walls = P.bc_y == DUGKS_BC_WALLS ? 1 : 0;
  C.vel_kind = P.vel_kind;
  C.visc_mode = P.visc_mode;
  C.grav_form = P.gravity_form == DUGKS_GRAV_BUOYANCY ? 1 : 0;
  C.row_vals = dugks::state_row_values(h->nx, h->coupled(), (int)h->elem());
  C.set[0] = h->buf[0];
  C.set[1] = h->buf[1];
  // Eq. 37 with sqrt(3RT) = 1 and delta_l the smallest cell width (1 on
  // the unit mesh)
  double dl = 1.0;
  if (h->mesh) {
    dl = HUGE_VAL;
    for (double w : h->mdx) dl = std::min(dl, w);
    for (double w : h->mdy) dl = std::min(dl, w);
  }
  C.dt = P.cfl * dl;
  C.h = 0.5 * C.dt;
  C.mesh = h->mesh ? h->dmesh : nullptr;
  C.meshf = h->mesh ? reinterpret_cast<const float*>(h->dmesh + dugks::kMeshArrays * (size_t)(h->nx + h->ny))
                    : nullptr;
  C.flag = h->dflag;
  C.t0 = 0.0;
  const double D = P.phi_H - P.phi_L;
  C.phi_H = P.phi_H;
  C.phi_L = P.phi_L;
  C.phibar = 0.5 * (P.phi_H + P.phi_L);
  C.inv_dphi = 1.0 / D;
  C.kappa = 1.5 * P.sigma * P.W / (D * D);
  C.beta = 12.0 * P.sigma / (P.W * D * D * D * D);
  C.theta_c = -4.0 / (P.W * D);
  C.rho_H = P.rho_H;
  C.rho_L = P.rho_L;
  C.drho = (P.rho_H - P.rho_L) / D;
  C.rho_ref = C.grav_form ? 0.5 * (P.rho_H + P.rho_L) : 0.0;
  C.tau_f = P.M_phi / kRT;
  C.tau_g_uniform = P.nu / kRT;
  C.mu_H = P.mu_H;
  C.mu_L = P.mu_L;
  C.inv_mu_H = P.mu_H > 0 ? 1.0 / P.mu_H : 0.0;
  C.inv_mu_L = P.mu_L > 0 ? 1.0 / P.mu_L : 0.0;
  C.gx = P.gx;
  C.gy = P.gy;
  C.Gx = P.Gx;
  C.Gy = P.Gy;
  C.U0 = P.U0;
  C.L0 = P.L0;
  C.T_period = P.T_period;
  // regularisation of the unit normal, in gradient units (over the smallest
  // width on a stretched mesh)
  C.eps_n2 = (P.eps_n * D / dl) * (P.eps_n * D / dl);
  C.fb = 3.0 * C.h / (2.0 * C.tau_f + C.dt);
  C.ffb = C.h / (2.0 * C.tau_f + C.h);
  C.gb = 3.0 * C.h / (2.0 * C.tau_g_uniform + C.dt);
  C.gfb = C.h / (2.0 * C.tau_g_uniform + C.h);
  C.f32 = dugks::narrow_constants(C);
  C.step0 = 0;
  C.nsteps = LLONG_MAX;
}

// Metric arrays of a stretched mesh (layout of CaseDev::mesh, see
// MeshAxis): per axis the widths, the distances to the previous and next
// centres (x periodic; y periodic, or with walls mirrored so that the ghost
// row has the width of its row), the centres, and the reciprocals and
// stencil weights derived from them.
static std::vector<double> mesh_metrics(const dugks_handle* h, bool walls) {
  std::vector<double> m;
  auto axis = [&](const std::vector<double>& w, bool mirror) {
    const int n = (int)w.size();
    auto at = [&](int k) {
      if (k < 0) return mirror ? w[0] : w[n - 1];
      if (k >= n) return mirror ? w[n - 1] : w[0];
      return w[k];
    };
    std::vector<std::vector<double>> a(dugks::kMeshArrays, std::vector<double>(n));
    double x = 0.0;
    for (int k = 0; k < n; ++k) {
      const double hm = 0.5 * (at(k - 1) + w[k]), hp = 0.5 * (w[k] + at(k + 1)), s = hm + hp;
      a[0][k] = w[k];
      a[1][k] = hm;
      a[2][k] = hp;
      a[3][k] = x + 0.5 * w[k];
      a[4][k] = 1.0 / w[k];
      a[5][k] = 1.0 / hm;
      a[6][k] = 1.0 / hp;
      a[7][k] = hm / (hp * s);
      a[8][k] = hp / (hm * s);
      a[9][k] = 2.0 / (hp * s);
      a[10][k] = 2.0 / (hm * s);
      a[11][k] = hm / s;
      a[12][k] = hp / s;
      x += w[k];
    }
    for (const auto& v : a) m.insert(m.end(), v.begin(), v.end());
  };
  axis(h->mdx, false);
  axis(h->mdy, walls);
  return m;
}

int upload_case(dugks_handle* h) {
  if (!h->dirty_case) return DUGKS_OK;
  fill_case(h);
  if (h->mesh) {  // the metrics depend on the y boundary
    const std::vector<double> m = mesh_metrics(h, h->hc.walls != 0);
    const std::vector<float> mf(m.begin(), m.end());  // rounded to nearest
    HIPCHK(h, hipMemcpyAsync(h->dmesh, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, hipMemcpyAsync(h->dmesh + m.size(), mf.data(), mf.size() * sizeof(float),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));  // m and mf are locals
  }
  HIPCHK(h, hipMemcpyAsync(h->dc, &h->hc, sizeof(CaseDev), hipMemcpyHostToDevice, h->stream));
  if (h->borrowed) {  // a pool case: the pool launches it with its own items, and
    h->dirty_case = false;  // h->hc, the source of the copy, lives as long as the case
    return DUGKS_OK;
  }
  std::vector<Item> it;
  it.reserve((size_t)h->hc.nstrips * h->hc.nsegs);
  for (int s = 0; s < h->hc.nsegs; ++s)
    for (int x = 0; x < h->hc.nstrips; ++x) it.push_back(Item{0, x, s, dugks::item_dir(s, h->hc.walls != 0)});
  if ((int)it.size() != h->nitems) {
    if (h->items) (void)hipFree(h->items);
    h->items = nullptr;
    HIPCHK(h, hipMalloc(&h->items, it.size() * sizeof(Item)));
    h->nitems = (int)it.size();
  }
  HIPCHK(h, hipMemcpyAsync(h->items, it.data(), it.size() * sizeof(Item), hipMemcpyHostToDevice,
                           h->stream));
  std::vector<Item> ut;
  if (h->general()) {
    h->upm_rows = h->seg_rows ? std::min(h->seg_rows, h->ny) : auto_upm_rows(h);
    const int ns = (h->nx + dugks::kUpmCols - 1) / dugks::kUpmCols;
    const int nseg = (h->ny + h->upm_rows - 1) / h->upm_rows;
    ut.reserve((size_t)ns * nseg);
    for (int s = 0; s < nseg; ++s)
      for (int x = 0; x < ns; ++x) ut.push_back(Item{0, x, s, 0});
    if ((int)ut.size() != h->nuitems) {
      if (h->uitems) (void)hipFree(h->uitems);
      h->uitems = nullptr;
      h->nuitems = 0;
      HIPCHK(h, hipMalloc(&h->uitems, ut.size() * sizeof(Item)));
      h->nuitems = (int)ut.size();
    }
    HIPCHK(h, hipMemcpyAsync(h->uitems, ut.data(), ut.size() * sizeof(Item), hipMemcpyHostToDevice,
                             h->stream));
  }
  // the pinned-host source of the copies above is a local: wait here
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->dirty_case = false;
  return DUGKS_OK;
}

int validate(const dugks_handle* h, const dugks_params* p, std::string& why) {
  auto bad = [&](const char* m) { why = m; return DUGKS_EINVAL; };
  if (!(p->phi_H != p->phi_L)) return bad("phi_H must differ from phi_L");
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return bad("cfl must lie in (0, 1]");
  if (!(p->W > 0.0)) return bad("W must be > 0");
  if (!(p->eps_n >= 0.0 && std::isfinite(p->eps_n))) return bad("eps_n must be finite and >= 0");
  if (!(p->sigma >= 0.0)) return bad("sigma must be >= 0");
  if (!(p->M_phi >= 0.0)) return bad("M_phi must be >= 0");
  if (p->bc_y != DUGKS_BC_PERIODIC && p->bc_y != DUGKS_BC_WALLS) return bad("bad bc_y");
  if (p->recon != DUGKS_RECON_CENTRAL && p->recon != DUGKS_RECON_UPWIND) return bad("bad recon");
  if (p->recon == DUGKS_RECON_UPWIND && h->borrowed)
    return bad("the upwind reconstruction runs on single handles only");
  if (h->model == DUGKS_MODEL_AC) {
    if (p->bc_y == DUGKS_BC_WALLS) return bad("walls need the coupled model");
    if (p->vel_kind < DUGKS_VEL_UNIFORM || p->vel_kind > DUGKS_VEL_DEFORM) return bad("bad vel_kind");
    if (p->vel_kind != DUGKS_VEL_UNIFORM && !(p->L0 > 0.0)) return bad("L0 must be > 0");
    if ((p->vel_kind == DUGKS_VEL_SHEAR || p->vel_kind == DUGKS_VEL_DEFORM) && !(p->T_period > 0.0))
      return bad("T_period must be > 0");
  } else {
    if (!(p->rho_H > 0.0 && p->rho_L > 0.0)) return bad("densities must be > 0");
    if (p->visc_mode == DUGKS_VISC_UNIFORM_NU) {
      if (!(p->nu > 0.0)) return bad("nu must be > 0");
    } else if (p->visc_mode == DUGKS_VISC_RECIPROCAL || p->visc_mode == DUGKS_VISC_LINEAR) {
      if (!(p->mu_H > 0.0 && p->mu_L > 0.0)) return bad("viscosities must be > 0");
    } else {
      return bad("bad visc_mode");
    }
    if (p->gravity_form != DUGKS_GRAV_RHO_G && p->gravity_form != DUGKS_GRAV_BUOYANCY)
      return bad("bad gravity_form");
    if (p->bc_y == DUGKS_BC_WALLS && h->ny < 4) return bad("walls need ny >= 4");
  }
  return DUGKS_OK;
}

size_t state_set_bytes(int nx, int ny, int precision, int model) {
  const int e = precision == DUGKS_FP64 ? 8 : 4;
  return (size_t)dugks::state_row_values(nx, model == DUGKS_MODEL_COUPLED, e) * (size_t)ny * e;
}

int ensure_scratch(dugks_handle* h) {
  if (h->scratch) return DUGKS_OK;
  const size_t bytes = (5 * h->n() + (size_t)kDiagBlocks * 7 + 16) * sizeof(double);
  HIPCHK(h, hipMalloc(&h->scratch, bytes));
  return DUGKS_OK;
}

int poll_flag(dugks_handle* h) {
  int v = 0;
  HIPCHK(h, hipMemcpyAsync(&v, h->dflag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (v) h->numeric_err = true;
  return DUGKS_OK;
}

int numeric_fail(dugks_handle* h) {
  return fail(h, DUGKS_ENUMERIC,
              "non-finite values in the state (phi, phi u or p); sticky until init_fields or set_state");
}

int launch_steps(dugks_handle* h, int nsteps) {
  if (h->general()) {
    StepArgs a{};
    a.cases = h->dc;
    a.items = h->uitems;
    a.nitems = h->nuitems;
    a.step_base = h->step_base;
    a.upm_rows = h->upm_rows;
    for (int k = 0; k < nsteps; ++k) {
      a.kofs = k;
      HIPCHK(h, dugks::launch_step_upm(h->fp64(), h->coupled(), h->hc.walls != 0, h->mesh,
                                       !h->upwind(), a, h->stream));
    }
    HIPCHK(h, dugks::launch_advance(h->step_base, nsteps, h->stream));
    return DUGKS_OK;
  }
  StepArgs a{};
  a.cases = h->dc;
  a.items = h->items;
  a.nitems = h->nitems;
  a.step_base = h->step_base;
  a.one_row = h->hc.seg_rows == 1 ? 1 : 0;
  a.two_row = h->hc.seg_rows == 2 ? 1 : 0;
  for (int k = 0; k < nsteps; ++k) {
    a.kofs = k;
    HIPCHK(h, dugks::launch_step(h->fp64(), h->coupled(), h->hc.walls != 0, a, h->stream));
  }
  HIPCHK(h, dugks::launch_advance(h->step_base, nsteps, h->stream));
  return DUGKS_OK;
}

// What the kernels of a handle's step take as launch arguments (variant,
// tiles, device pointers). A captured step sequence stays valid while this
// is unchanged; the case constants themselves are read from device memory.
std::vector<long long> launch_sig(const dugks_handle* h) {
  return {h->general() ? 1 : 0, h->upwind() ? 1 : 0, h->mesh ? 1 : 0, (long long)h->hc.walls,
          h->fp64() ? 1 : 0, h->coupled() ? 1 : 0, (long long)(uintptr_t)h->items,
          (long long)h->nitems, (long long)h->hc.seg_rows, (long long)(uintptr_t)h->dc,
          (long long)(uintptr_t)h->step_base, (long long)(uintptr_t)h->uitems,
          (long long)h->nuitems, (long long)h->upm_rows, (long long)h->nx,
          (long long)h->ny};
}

void drop_graphs(dugks_handle* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
  h->graphs.clear();
}

// Sequences of at least kGraphMin steps on a created stream are recorded once
// in a HIP graph (per step count, at most kGraphCache kept) and replayed: one
// launch from the host instead of one (or two) per step.
constexpr int kGraphMin = 8;
constexpr size_t kGraphCache = 8;

int launch_steps_graph(dugks_handle* h, int nsteps) {
  const std::vector<long long> sig = launch_sig(h);
  if (sig != h->gsig) {
    drop_graphs(h);
    h->gsig = sig;
  }
  hipGraphExec_t ex = nullptr;
  for (auto& g : h->graphs)
    if (g.first == nsteps) ex = g.second;
  if (!ex) {
    if (h->graphs.size() >= kGraphCache) {
      (void)hipGraphExecDestroy(h->graphs.front().second);
      h->graphs.erase(h->graphs.begin());
    }
    hipGraph_t g = nullptr;
    HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch_steps(h, nsteps);
    hipError_t e = hipStreamEndCapture(h->stream, &g);  // always ends the capture
    if (rc) {
      if (e == hipSuccess && g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
    h->graphs.emplace_back(nsteps, ex);
  }
  HIPCHK(h, hipGraphLaunch(ex, h->stream));
  return DUGKS_OK;
}

}  // namespace host
}  // namespace dugks

using namespace dugks::host;

extern "C" {

int dugks_create(int nx, int ny, int precision, int model, dugks_handle** out) {
  if (!out) return fail(nullptr, DUGKS_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 3 || ny < 3) return fail(nullptr, DUGKS_EINVAL, "nx and ny must be >= 3");
  if (precision != DUGKS_FP32 && precision != DUGKS_FP64)
    return fail(nullptr, DUGKS_EINVAL, "bad precision");
  // size limit of the C ABI: 2^28 cells in FP32, 2^27 in FP64
  if ((long long)nx * ny > (1LL << 32) / (4 * (precision == DUGKS_FP64 ? 8 : 4)))
    return fail(nullptr, DUGKS_EINVAL, "grid too large (cells > 2^28 in FP32, 2^27 in FP64)");
  if (model != DUGKS_MODEL_AC && model != DUGKS_MODEL_COUPLED)
    return fail(nullptr, DUGKS_EINVAL, "bad model");
  dugks_handle* h = new (std::nothrow) dugks_handle;
  if (!h) return fail(nullptr, DUGKS_ENOMEM, "host allocation failed");
  h->nx = nx;
  h->ny = ny;
  h->precision = precision;
  h->model = model;
  h->buf_bytes = state_set_bytes(nx, ny, precision, model);
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMalloc(&h->buf[k], h->buf_bytes);
  // zero both buffers once, so that the row padding (never written by the
  // kernels) reads the same in either buffer and the saved state is a pure
  // function of the step
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemset(h->buf[k], 0, h->buf_bytes);
  if (e == hipSuccess) e = hipMalloc(&h->dc, sizeof(CaseDev));
  if (e == hipSuccess) e = hipMalloc(&h->step_base, sizeof(long long));
  if (e == hipSuccess) e = hipMemset(h->step_base, 0, sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&h->dflag, sizeof(int));
  if (e == hipSuccess) e = hipMemset(h->dflag, 0, sizeof(int));
  if (e != hipSuccess) {
    std::string msg = std::string("device allocation failed: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    dugks_destroy(h);
    return fail(nullptr, e == hipErrorOutOfMemory ? DUGKS_ENOMEM : DUGKS_EDEVICE, msg);
  }
  *out = h;
  return DUGKS_OK;
}

int dugks_set_params(dugks_handle* h, const dugks_params* p) {
  if (!h || !p) return fail(h, DUGKS_EINVAL, "NULL argument");
  std::string why;
  if (validate(h, p, why) != DUGKS_OK) return fail(h, DUGKS_EINVAL, why);
  h->params = *p;
  h->has_params = true;
  h->dirty_case = true;
  return upload_case(h);
}

int dugks_set_stream(dugks_handle* h, void* stream) {
  if (!h) return DUGKS_EINVAL;
  h->stream = static_cast<hipStream_t>(stream);
  return DUGKS_OK;
}

// Rows per segment of the step kernel's work items (0 = automatic).
int dugks_set_tile(dugks_handle* h, int seg_rows) {
  if (!h || seg_rows < 0 || seg_rows > 4096) return fail(h, DUGKS_EINVAL, "bad seg_rows");
  h->seg_rows = seg_rows;
  h->dirty_case = true;
  if (h->has_params) return upload_case(h);
  return DUGKS_OK;
}

int dugks_get_tile(const dugks_handle* h) {
  if (!h) return -1;
  return h->general() ? h->upm_rows : h->hc.seg_rows;
}

int dugks_set_mesh(dugks_handle* h, const double* dx, const double* dy) {
  if (!h) return fail(h, DUGKS_EINVAL, "NULL handle");
  if (h->borrowed) return fail(h, DUGKS_EINVAL, "pool cases run on the unit mesh");
  if (!dx && !dy) {  // back to the unit mesh and the fused march
    h->mesh = false;
    h->mdx.clear();
    h->mdy.clear();
    h->dirty_case = true;
    h->has_state = false;
    return h->has_params ? upload_case(h) : DUGKS_OK;
  }
  std::vector<double> wx(h->nx, 1.0), wy(h->ny, 1.0);
  for (int i = 0; i < h->nx; ++i)
    if (dx) wx[i] = dx[i];
  for (int j = 0; j < h->ny; ++j)
    if (dy) wy[j] = dy[j];
  for (double w : wx)
    if (!(w > 0.0 && std::isfinite(w))) return fail(h, DUGKS_EINVAL, "cell widths must be finite and > 0");
  for (double w : wy)
    if (!(w > 0.0 && std::isfinite(w))) return fail(h, DUGKS_EINVAL, "cell widths must be finite and > 0");
  if (!h->dmesh) {
    // the metric arrays in double, then rounded to float
    hipError_t e = hipMalloc(&h->dmesh, dugks::kMeshArrays * (size_t)(h->nx + h->ny) *
                                            (sizeof(double) + sizeof(float)));
    if (e != hipSuccess) {
      h->dmesh = nullptr;
      (void)hipGetLastError();
      return fail(h, DUGKS_ENOMEM, std::string("mesh allocation failed: ") + hipGetErrorString(e));
    }
  }
  h->mesh = true;
  h->mdx.swap(wx);
  h->mdy.swap(wy);
  h->dirty_case = true;
  h->has_state = false;  // the time step and stencils changed: init again
  return h->has_params ? upload_case(h) : DUGKS_OK;
}

int dugks_init_fields_device(dugks_handle* h, const double* phi, const double* u, const double* v,
                             const double* p) {
  if (!h || !phi) return fail(h, DUGKS_EINVAL, "phi is NULL");
  if (!h->has_params) return fail(h, DUGKS_ESTATE, "set_params first");
  int rc = upload_case(h);
  if (rc) return rc;
  // local step 0 lives in buffer 0; the device step counter restarts at 0
  h->hc.cur0 = 0;
  h->hc.step0 = 0;
  HIPCHK(h, hipMemcpyAsync(h->dc, &h->hc, sizeof(CaseDev), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, dugks::launch_reset(h->step_base, 0, h->dflag, h->stream));
  HIPCHK(h, dugks::launch_init(h->fp64(), h->dc, h->hc, phi, u, v, p, h->stream));
  h->steps = 0;
  h->has_state = true;
  h->numeric_err = false;
  return DUGKS_OK;
}

int dugks_init_fields(dugks_handle* h, const double* phi, const double* u, const double* v,
                      const double* p) {
  if (!h || !phi) return fail(h, DUGKS_EINVAL, "phi is NULL");
  if (!h->has_params) return fail(h, DUGKS_ESTATE, "set_params first");
  int rc = ensure_scratch(h);
  if (rc) return rc;
  const size_t n = h->n(), b = n * sizeof(double);
  double* d[4] = {h->scratch, h->scratch + n, h->scratch + 2 * n, h->scratch + 3 * n};
  const double* src[4] = {phi, u, v, p};
  for (int k = 0; k < 4; ++k)
    if (src[k]) HIPCHK(h, hipMemcpyAsync(d[k], src[k], b, hipMemcpyHostToDevice, h->stream));
  rc = dugks_init_fields_device(h, d[0], u ? d[1] : nullptr, v ? d[2] : nullptr, p ? d[3] : nullptr);
  if (rc) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return DUGKS_OK;
}

int dugks_step(dugks_handle* h, int nsteps) {
  if (!h || nsteps < 0) return fail(h, DUGKS_EINVAL, "bad arguments");
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  if (h->numeric_err) return numeric_fail(h);
  if (nsteps == 0) return DUGKS_OK;
  // graph replay on a created stream that is not being captured by the caller
  bool graph = false;
  if (h->stream && nsteps >= kGraphMin) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    HIPCHK(h, hipStreamIsCapturing(h->stream, &st));
    graph = st == hipStreamCaptureStatusNone;
  }
  int rc = graph ? launch_steps_graph(h, nsteps) : launch_steps(h, nsteps);
  if (rc) return rc;
  h->steps += nsteps;
  return DUGKS_OK;
}

int dugks_sync(dugks_handle* h) {
  if (!h) return DUGKS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->has_state) {
    const int rc = poll_flag(h);
    if (rc) return rc;
  }
  return h->numeric_err ? numeric_fail(h) : DUGKS_OK;
}

int dugks_get_macros_device(dugks_handle* h, double* phi, double* u, double* v, double* p,
                            double* rho) {
  if (!h) return DUGKS_EINVAL;
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  HIPCHK(h, dugks::launch_macros(h->fp64(), h->dc, h->hc, h->steps, phi, u, v, p, rho, h->stream));
  return DUGKS_OK;
}

int dugks_get_macros(dugks_handle* h, double* phi, double* u, double* v, double* p, double* rho) {
  if (!h) return DUGKS_EINVAL;
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  int rc = ensure_scratch(h);
  if (rc) return rc;
  const size_t n = h->n(), b = n * sizeof(double);
  double* d[5] = {h->scratch, h->scratch + n, h->scratch + 2 * n, h->scratch + 3 * n,
                  h->scratch + 4 * n};
  double* dst[5] = {phi, u, v, p, rho};
  rc = dugks_get_macros_device(h, phi ? d[0] : nullptr, u ? d[1] : nullptr, v ? d[2] : nullptr,
                               p ? d[3] : nullptr, rho ? d[4] : nullptr);
  if (rc) return rc;
  for (int k = 0; k < 5; ++k)
    if (dst[k]) HIPCHK(h, hipMemcpyAsync(dst[k], d[k], b, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return poll_flag(h);  // a readout, not a failure: the flag only becomes sticky
}

int dugks_get_diagnostics(dugks_handle* h, double out[8]) {
  if (!h || !out) return DUGKS_EINVAL;
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  int rc = ensure_scratch(h);
  if (rc) return rc;
  const size_t n = h->n();
  double* phi = h->scratch;
  double* u = phi + n;
  double* v = u + n;
  double* rho = v + 2 * n;
  double* part = h->scratch + 5 * n;
  double* dout = part + (size_t)kDiagBlocks * 7;
  rc = dugks_get_macros_device(h, phi, u, v, nullptr, rho);
  if (rc) return rc;
  HIPCHK(h, dugks::launch_diag(h->hc, phi, u, v, rho, part, kDiagBlocks, dout, h->stream));
  double tmp[7];
  HIPCHK(h, hipMemcpyAsync(tmp, dout, sizeof(tmp), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int k = 0; k < 7; ++k) out[k] = tmp[k];
  out[7] = h->steps * h->hc.dt;
  rc = poll_flag(h);
  if (rc) return rc;
  if (tmp[6] > 0) h->numeric_err = true;
  return h->numeric_err ? numeric_fail(h) : DUGKS_OK;
}

int dugks_get_diagnostics_noalloc(dugks_handle* h, double* out_dev) {
  if (!h || !out_dev) return fail(h, DUGKS_EINVAL, "NULL argument");
  double* part = nullptr;
  int max_rows = 0;
  HIPCHK(h, dugks::noalloc_scratch(&part, &max_rows));
  if (h->ny > max_rows)
    return fail(h, DUGKS_EINVAL,
                "grid too tall for the diagnostics without allocation (at most " +
                    std::to_string(max_rows) + " rows)");
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  HIPCHK(h, dugks::launch_diag_noalloc(h->fp64(), h->dc, h->hc, h->steps, part, out_dev, h->stream));
  return DUGKS_OK;
}

long long dugks_steps_done(const dugks_handle* h) { return h ? h->steps : -1; }
double dugks_time(const dugks_handle* h) { return h ? h->steps * h->hc.dt : 0.0; }

size_t dugks_state_bytes(const dugks_handle* h) { return h ? h->buf_bytes : 0; }

int dugks_get_state(dugks_handle* h, void* host_buf, size_t bytes, long long* steps) {
  if (!h || !host_buf || bytes != h->buf_bytes) return fail(h, DUGKS_EINVAL, "bad buffer");
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  const int cur = (h->hc.cur0 + (int)(h->steps & 1)) & 1;
  HIPCHK(h, hipMemcpyAsync(host_buf, h->buf[cur], bytes, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (steps) *steps = h->steps;
  return DUGKS_OK;
}

int dugks_set_state(dugks_handle* h, const void* host_buf, size_t bytes, long long steps) {
  if (!h || !host_buf || bytes != h->buf_bytes || steps < 0)
    return fail(h, DUGKS_EINVAL, "bad buffer");
  if (!h->has_params) return fail(h, DUGKS_ESTATE, "set_params first");
  int rc = upload_case(h);
  if (rc) return rc;
  h->hc.cur0 = (int)(steps & 1);  // local step `steps` lands in buffer 0
  h->hc.step0 = 0;
  HIPCHK(h, hipMemcpyAsync(h->dc, &h->hc, sizeof(CaseDev), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(h->buf[0], host_buf, bytes, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, dugks::launch_reset(h->step_base, steps, h->dflag, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->steps = steps;
  h->has_state = true;
  h->numeric_err = false;
  return DUGKS_OK;
}

int dugks_autotune(dugks_handle* h, int probe_steps, int* out_seg_rows, double* out_us) {
  if (!h || probe_steps < 1 || probe_steps > 1000) return fail(h, DUGKS_EINVAL, "bad arguments");
  if (!h->has_state) return fail(h, DUGKS_ESTATE, "init_fields first");
  // candidates: the shortest segments (lowest latency per step), and for
  // k = 1..8, 12, 16, 20, 24 the shortest segment whose tiles fit k rounds of resident waves
  // (more rounds: finer load balance, more repeated halo work); for the
  // reconstruction march (upwind or stretched mesh) with its own strips and
  // resident waves
  const int keep = h->seg_rows;
  int rc = DUGKS_OK;
  const int a = h->general() ? h->upm_rows : h->hc.seg_rows;
  const std::vector<StripShape> shape = {
      StripShape{h->general() ? (h->nx + dugks::kUpmCols - 1) / dugks::kUpmCols : h->hc.nstrips, h->ny}};
  const long long cap =
      h->general() ? cu_count() * dugks::upm_waves_per_cu(h->fp64(), h->coupled(), h->hc.walls != 0,
                                                          h->mesh, !h->upwind())
                   : wave_capacity(h->fp64(), h->coupled(), h->hc.walls != 0);
  std::vector<int> use = {1, 2};
  for (int k : {1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 20, 24}) {
    const int c = fit_seg_rows(shape, k * cap);
    if (std::find(use.begin(), use.end(), c) == use.end()) use.push_back(c);
  }
  // the probe steps run on a copy of the state, which is put back afterwards
  int rc0 = poll_flag(h);  // the probes step the state: clear the flag again if it was clear
  if (rc0) return rc0;
  const int cur = (h->hc.cur0 + (int)(h->steps & 1)) & 1;
  const long long steps0 = h->steps;
  void* saved = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipMalloc(&saved, h->buf_bytes));
  int best = a;
  float best_ms = 0.0f;
  hipError_t e = hipMemcpyAsync(saved, h->buf[cur], h->buf_bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (size_t k = 0; k < use.size() && e == hipSuccess && rc == DUGKS_OK; ++k) {
    h->seg_rows = use[k];
    h->dirty_case = true;
    rc = upload_case(h);
    if (rc) break;
    if (h->stream) {
      // on a stream that can be captured, timed the way dugks_step runs
      // longer sequences there: one captured graph, replayed once untimed
      // and once timed (direct launches can rank the tiles differently)
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) break;
      rc = launch_steps(h, probe_steps);
      e = hipStreamEndCapture(h->stream, &g);  // always ends the capture
      if (rc) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        break;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e == hipSuccess) e = hipGraphLaunch(ex, h->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
      if (e == hipSuccess) e = hipGraphLaunch(ex, h->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (ex) (void)hipGraphExecDestroy(ex);
    } else {
      rc = launch_steps(h, 1);  // warm-up
      if (rc) break;
      e = hipEventRecord(e0, h->stream);
      if (e == hipSuccess) rc = launch_steps(h, probe_steps);
      if (rc) break;
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (k == 0 || ms < best_ms)) {
      best_ms = ms;
      best = use[k];
    }
    // back to the saved state: it sits in buffer 0 as local step steps0
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->buf[0], saved, h->buf_bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->step_base, &steps0, sizeof(long long), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    h->hc.cur0 = (int)(steps0 & 1);
    h->dirty_case = true;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!h->numeric_err) (void)dugks::launch_reset(nullptr, 0, h->dflag, h->stream);
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(saved);
  h->steps = steps0;
  if (e != hipSuccess) {
    h->seg_rows = keep;
    h->dirty_case = true;
    (void)upload_case(h);
    return hip_fail(h, e, "autotune");
  }
  if (rc) return rc;
  h->seg_rows = best;
  h->dirty_case = true;
  rc = upload_case(h);
  if (rc) return rc;
  if (out_seg_rows) *out_seg_rows = best;
  if (out_us) *out_us = 1e3 * (double)best_ms / probe_steps;
  return DUGKS_OK;
}

size_t dugks_footprint_bytes(int nx, int ny, int precision, int model) {
  if (nx < 1 || ny < 1) return 0;
  return 2 * state_set_bytes(nx, ny, precision, model) + sizeof(CaseDev) + 64;
}

const char* dugks_last_error(const dugks_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

int dugks_destroy(dugks_handle* h) {
  if (!h) return DUGKS_OK;
  if (h->borrowed) return fail(h, DUGKS_EINVAL, "a pool case is retired through its pool");
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (int k = 0; k < 2; ++k)
    if (h->buf[k]) (void)hipFree(h->buf[k]);
  if (h->dc) (void)hipFree(h->dc);
  if (h->items) (void)hipFree(h->items);
  if (h->step_base) (void)hipFree(h->step_base);
  if (h->dflag) (void)hipFree(h->dflag);
  if (h->scratch) (void)hipFree(h->scratch);
  if (h->uitems) (void)hipFree(h->uitems);
  if (h->dmesh) (void)hipFree(h->dmesh);
  drop_graphs(h);
  delete h;
  return DUGKS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct dugks_batch {
  std::vector<dugks_handle*> cases;
  bool owns = false;              // cases made by dugks_batch_create: destroyed with the batch
  std::vector<long long> budget;  // remaining steps per case, < 0 = unlimited
  bool fp64 = false, coupled = true;
  hipStream_t stream = nullptr;
  CaseDev* dcases = nullptr;
  Item* items[2] = {nullptr, nullptr};  // work items: periodic cases, wall cases
  int nitems[2] = {0, 0};
  int one_row[2] = {1, 1};              // every case of the group has one-row tiles
  int two_row[2] = {1, 1};              // every case of the group has two-row tiles
  std::vector<int> seg;                 // rows per segment used for each case
  std::vector<long long> bsig;          // what the items were built from (case_sig)
  long long* step_base = nullptr;  // device: global step of the batch
  long long gstep = 0;             // host mirror
  std::vector<CaseDev> hcases;
  std::map<int, hipGraphExec_t> graphs;
  std::string err = "no error";
  // The cases run as two independent chains of launches: cases [0, half) on
  // the batch's stream and [half, n) on `side`, forked from and joined to
  // the batch's stream once per recorded sequence, so that the two chains'
  // kernels overlap each other's start and drain. ofs[w][j] is where chain
  // j's items of boundary group w start (items are case-major).
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  int half = 0;
  int ofs[2][3] = {{0, 0, 0}, {0, 0, 0}};
};

namespace {

int bfail(dugks_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  else g_create_error = m;
  return code;
}

#define BHIPCHK(b, expr)                                                        \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess)                                                       \
      return bfail((b), DUGKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Bring the batch descriptors in line with the handles: local step n of
// case k happens at global step gstep + (n - steps_k).
int sync_descriptors(dugks_batch* b) {
  for (size_t k = 0; k < b->cases.size(); ++k) {
    dugks_handle* h = b->cases[k];
    if (h->general())  // parameters or mesh changed after the batch was made
      return bfail(b, DUGKS_EINVAL,
                   "the upwind reconstruction and stretched meshes run on single handles only");
    CaseDev c = h->hc;
    c.seg_rows = b->seg[k];
    c.nsegs = (c.ny + c.seg_rows - 1) / c.seg_rows;
    c.step0 = b->gstep - h->steps;
    c.nsteps = b->budget[k] < 0 ? LLONG_MAX : h->steps + b->budget[k];
    b->hcases[k] = c;
  }
  BHIPCHK(b, hipMemcpyAsync(b->dcases, b->hcases.data(), b->hcases.size() * sizeof(CaseDev),
                            hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  return DUGKS_OK;
}

// Work items of both boundary groups from the segment length of each case
// (b->seg); (re)allocates the item arrays.
hipError_t build_items(dugks_batch* b) {
  std::vector<Item> it[2];
  b->one_row[0] = b->one_row[1] = 1;
  b->two_row[0] = b->two_row[1] = 1;
  // the chains: the first case at which the running cell count reaches half
  // of the batch's (none for a single case)
  const size_t n = b->cases.size();
  long long total = 0, run = 0;
  for (auto* h : b->cases) total += h->n();
  b->half = (int)n;
  for (size_t k = 0; k + 1 < n && n >= 2; ++k) {
    run += b->cases[k]->n();
    if (2 * run >= total) {
      b->half = (int)k + 1;
      break;
    }
  }
  if (n >= 2 && b->half == (int)n) b->half = (int)n - 1;
  for (size_t k = 0; k < n; ++k) {
    const CaseDev& c = b->cases[k]->hc;
    const int w = c.walls ? 1 : 0;
    if ((int)k == b->half) {
      b->ofs[0][1] = (int)it[0].size();
      b->ofs[1][1] = (int)it[1].size();
    }
    if (b->seg[k] != 1) b->one_row[w] = 0;
    if (b->seg[k] != 2) b->two_row[w] = 0;
    const int nsegs = (c.ny + b->seg[k] - 1) / b->seg[k];
    for (int s = 0; s < nsegs; ++s)
      for (int x = 0; x < c.nstrips; ++x) it[w].push_back(Item{(int)k, x, s, dugks::item_dir(s, w == 1)});
  }
  for (int w = 0; w < 2; ++w) {
    b->ofs[w][0] = 0;
    if (b->half >= (int)n) b->ofs[w][1] = (int)it[w].size();
    b->ofs[w][2] = (int)it[w].size();
  }
  for (int w = 0; w < 2; ++w) {
    if (b->items[w]) (void)hipFree(b->items[w]);
    b->items[w] = nullptr;
    b->nitems[w] = (int)it[w].size();
    if (it[w].empty()) continue;
    hipError_t e = hipMalloc(&b->items[w], it[w].size() * sizeof(Item));
    if (e == hipSuccess)
      e = hipMemcpy(b->items[w], it[w].data(), it[w].size() * sizeof(Item), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
  return hipSuccess;
}

// What the work items of a batch depend on: each case's boundary group and
// explicit tile.
std::vector<long long> case_sig(const dugks_batch* b) {
  std::vector<long long> s;
  for (const auto* h : b->cases) {
    s.push_back(h->params.bc_y == DUGKS_BC_WALLS ? 1 : 0);
    s.push_back(h->seg_rows);
  }
  return s;
}

// Segment lengths and work items, built on first use and again when a
// case's boundary group or explicit tile has changed. Every case needs its
// parameters; the upwind reconstruction and stretched meshes are refused.
int ensure_built(dugks_batch* b) {
  const size_t n = b->cases.size();
  for (size_t k = 0; k < n; ++k) {
    dugks_handle* h = b->cases[k];
    if (!h->has_params) return bfail(b, DUGKS_ESTATE, "case " + std::to_string(k) + " has no params");
    if (h->general())
      return bfail(b, DUGKS_EINVAL,
                   "the upwind reconstruction and stretched meshes run on single handles only");
  }
  const std::vector<long long> sig = case_sig(b);
  if (sig == b->bsig && b->step_base) return DUGKS_OK;
  // one segment length per boundary group, sized to the whole group
  std::vector<StripShape> shapes[2];
  for (size_t k = 0; k < n; ++k) {
    if (upload_case(b->cases[k]) != DUGKS_OK)
      return bfail(b, DUGKS_EDEVICE, b->cases[k]->err);
    const CaseDev& c = b->cases[k]->hc;
    if (b->cases[k]->seg_rows == 0) shapes[c.walls ? 1 : 0].push_back(StripShape{c.nstrips, c.ny});
  }
  int segw[2];
  for (int w = 0; w < 2; ++w)
    segw[w] = shapes[w].empty()
                  ? 1
                  : auto_seg_rows(shapes[w], wave_capacity(b->fp64, b->coupled, w == 1), b->fp64,
                                  w == 1);
  for (size_t k = 0; k < n; ++k) {
    const int w = b->cases[k]->hc.walls ? 1 : 0;
    // a case's explicit tile wins over the group's automatic one
    b->seg[k] = b->cases[k]->seg_rows > 0 ? b->cases[k]->seg_rows : segw[w];
  }
  hipError_t e = hipSuccess;
  if (!b->dcases) e = hipMalloc(&b->dcases, n * sizeof(CaseDev));
  if (e == hipSuccess && !b->step_base) {
    e = hipMalloc(&b->step_base, sizeof(long long));
    if (e == hipSuccess) e = hipMemcpy(b->step_base, &b->gstep, sizeof(long long), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && b->cases.size() >= 2 && !b->side) {
    // default priority, like every stream here
    e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = build_items(b);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, e == hipErrorOutOfMemory ? DUGKS_ENOMEM : DUGKS_EDEVICE,
                 std::string("batch set-up failed: ") + hipGetErrorString(e));
  }
  b->bsig = sig;
  return DUGKS_OK;
}

// ENUMERIC when a case's numeric error is sticky (message names the cases).
int numeric_check(dugks_batch* b) {
  std::string bad;
  for (size_t k = 0; k < b->cases.size(); ++k)
    if (b->cases[k]->numeric_err) bad += (bad.empty() ? "" : ", ") + std::to_string(k);
  if (bad.empty()) return DUGKS_OK;
  return bfail(b, DUGKS_ENUMERIC, "non-finite values in the state of case(s) " + bad);
}

int record_steps(dugks_batch* b, int nsteps) {
  StepArgs a{};
  a.cases = b->dcases;
  a.step_base = b->step_base;
  const bool two = b->side && b->half < (int)b->cases.size();
  if (two) {
    BHIPCHK(b, hipEventRecord(b->fork, b->stream));
    BHIPCHK(b, hipStreamWaitEvent(b->side, b->fork, 0));
  }
  for (int k = 0; k < nsteps; ++k) {
    a.kofs = k;
    for (int j = 0; j < (two ? 2 : 1); ++j) {
      for (int w = 0; w < 2; ++w) {
        const int i0 = two ? b->ofs[w][j] : 0, i1 = two ? b->ofs[w][j + 1] : b->nitems[w];
        if (i1 <= i0) continue;
        a.items = b->items[w] + i0;
        a.nitems = i1 - i0;
        a.one_row = b->one_row[w];
        a.two_row = b->two_row[w];
        BHIPCHK(b, dugks::launch_step(b->fp64, b->coupled, w == 1, a, j ? b->side : b->stream));
      }
    }
  }
  if (two) {
    BHIPCHK(b, hipEventRecord(b->join, b->side));
    BHIPCHK(b, hipStreamWaitEvent(b->stream, b->join, 0));
  }
  BHIPCHK(b, dugks::launch_advance(b->step_base, nsteps, b->stream));
  return DUGKS_OK;
}

dugks_batch* new_batch(int n, dugks_handle* const* cases, bool owns) {
  dugks_batch* b = new (std::nothrow) dugks_batch;
  if (!b) return nullptr;
  b->cases.assign(cases, cases + n);
  b->owns = owns;
  b->budget.assign(n, -1);
  b->hcases.resize(n);
  b->seg.assign(n, 2);
  b->fp64 = cases[0]->fp64();
  b->coupled = cases[0]->coupled();
  return b;
}

}  // namespace

extern "C" {

int dugks_batch_create(int n, const int* nx, const int* ny, int precision, int model,
                       dugks_batch** out) {
  if (!out || n <= 0 || !nx || !ny) return bfail(nullptr, DUGKS_EINVAL, "bad arguments");
  *out = nullptr;
  std::vector<dugks_handle*> hs(n, nullptr);
  for (int k = 0; k < n; ++k) {
    const int rc = dugks_create(nx[k], ny[k], precision, model, &hs[k]);
    if (rc != DUGKS_OK) {
      const std::string m = "case " + std::to_string(k) + ": " + g_create_error;
      for (auto* h : hs) dugks_destroy(h);
      return bfail(nullptr, rc, m);
    }
  }
  dugks_batch* b = new_batch(n, hs.data(), true);
  if (!b) {
    for (auto* h : hs) dugks_destroy(h);
    return bfail(nullptr, DUGKS_ENOMEM, "host allocation failed");
  }
  *out = b;
  return DUGKS_OK;
}

dugks_handle* dugks_batch_case(dugks_batch* b, int k) {
  if (!b || k < 0 || k >= (int)b->cases.size()) return nullptr;
  return b->cases[k];
}

int dugks_batch_create_from(int n, dugks_handle* const* cases, dugks_batch** out) {
  if (!out || n <= 0 || !cases) return bfail(nullptr, DUGKS_EINVAL, "bad arguments");
  *out = nullptr;
  for (int k = 0; k < n; ++k) {
    if (!cases[k]) return bfail(nullptr, DUGKS_EINVAL, "NULL case");
    if (!cases[k]->has_params) return bfail(nullptr, DUGKS_ESTATE, "case without params");
    if (cases[k]->precision != cases[0]->precision || cases[k]->model != cases[0]->model)
      return bfail(nullptr, DUGKS_EINVAL, "cases must share precision and model");
    if (cases[k]->general())
      return bfail(nullptr, DUGKS_EINVAL,
                   "the upwind reconstruction and stretched meshes run on single handles only");
  }
  dugks_batch* b = new_batch(n, cases, false);
  if (!b) return bfail(nullptr, DUGKS_ENOMEM, "host allocation failed");
  const int rc = ensure_built(b);
  if (rc != DUGKS_OK) {
    const std::string m = b->err;
    dugks_batch_destroy(b);
    return bfail(nullptr, rc, m);
  }
  *out = b;
  return DUGKS_OK;
}

int dugks_batch_set_budget(dugks_batch* b, int k, long long steps) {
  if (!b || k < 0 || k >= (int)b->cases.size()) return bfail(b, DUGKS_EINVAL, "bad case index");
  b->budget[k] = steps < 0 ? -1 : steps;
  return DUGKS_OK;
}

int dugks_batch_autotune(dugks_batch* b, int probe_steps, int* seg_periodic, int* seg_walls) {
  if (!b || probe_steps < 1 || probe_steps > 1000) return bfail(b, DUGKS_EINVAL, "bad arguments");
  for (auto* h : b->cases)
    if (!h->has_state) return bfail(b, DUGKS_ESTATE, "a case has no state");
  int brc = ensure_built(b);
  if (brc) return brc;
  for (auto* h : b->cases)
    if (h->stream != b->stream) BHIPCHK(b, hipStreamSynchronize(h->stream));
  // the probes step every case: remember which flags were clear, to clear
  // them again with the states put back
  for (auto* h : b->cases) {
    const int rc = poll_flag(h);
    if (rc) return bfail(b, rc, h->err);
  }
  const size_t n = b->cases.size();
  // the current state of every case, put back after each probe
  std::vector<void*> saved(n, nullptr);
  std::vector<int> curbuf(n);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < n && e == hipSuccess; ++k) {
    dugks_handle* h = b->cases[k];
    curbuf[k] = (h->hc.cur0 + (int)(h->steps & 1)) & 1;
    e = hipMalloc(&saved[k], h->buf_bytes);
    if (e == hipSuccess)
      e = hipMemcpyAsync(saved[k], h->buf[curbuf[k]], h->buf_bytes, hipMemcpyDeviceToDevice, b->stream);
  }
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto restore = [&]() -> hipError_t {
    hipError_t r = hipSuccess;
    for (size_t k = 0; k < n && r == hipSuccess; ++k)
      r = hipMemcpyAsync(b->cases[k]->buf[curbuf[k]], saved[k], b->cases[k]->buf_bytes,
                         hipMemcpyDeviceToDevice, b->stream);
    if (r == hipSuccess)
      r = hipMemcpyAsync(b->step_base, &b->gstep, sizeof(long long), hipMemcpyHostToDevice, b->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(b->stream);
    return r;
  };
  // time `probe_steps` batch steps with the current items (state put back after)
  auto probe = [&](float& ms) -> int {
    int rc = sync_descriptors(b);
    if (rc) return rc;
    if (b->stream) {
      // on a stream that can be captured, the candidate is timed the way
      // dugks_batch_step with use_graph runs it: one captured graph of
      // probe_steps steps, replayed once untimed and once timed (direct
      // launches rank the tiles differently)
      hipGraph_t g;
      BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      rc = record_steps(b, probe_steps);
      hipError_t ce = hipStreamEndCapture(b->stream, &g);
      if (rc) return rc;
      if (ce != hipSuccess) return bfail(b, DUGKS_EDEVICE, hipGetErrorString(ce));
      hipGraphExec_t ex = nullptr;
      ce = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ce == hipSuccess) ce = hipGraphLaunch(ex, b->stream);
      if (ce == hipSuccess) ce = hipEventRecord(e0, b->stream);
      if (ce == hipSuccess) ce = hipGraphLaunch(ex, b->stream);
      if (ce == hipSuccess) ce = hipEventRecord(e1, b->stream);
      if (ce == hipSuccess) ce = hipEventSynchronize(e1);
      if (ex) (void)hipGraphExecDestroy(ex);
      if (ce != hipSuccess) return bfail(b, DUGKS_EDEVICE, hipGetErrorString(ce));
    } else {
      rc = record_steps(b, 1);  // warm-up
      if (rc) return rc;
      BHIPCHK(b, hipEventRecord(e0, b->stream));
      rc = record_steps(b, probe_steps);
      if (rc) return rc;
      BHIPCHK(b, hipEventRecord(e1, b->stream));
      BHIPCHK(b, hipEventSynchronize(e1));
    }
    BHIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
    BHIPCHK(b, restore());
    return DUGKS_OK;
  };
  int rc = e == hipSuccess ? DUGKS_OK : bfail(b, DUGKS_EDEVICE, hipGetErrorString(e));
  int best[2] = {0, 0};
  // one group at a time, the other at its current segment length
  for (int w = 0; w < 2 && rc == DUGKS_OK; ++w) {
    std::vector<StripShape> shapes;
    for (size_t k = 0; k < n; ++k)
      if ((b->cases[k]->hc.walls ? 1 : 0) == w)
        shapes.push_back(StripShape{b->cases[k]->hc.nstrips, b->cases[k]->ny});
    if (shapes.empty()) continue;
    const long long cap = wave_capacity(b->fp64, b->coupled, w == 1);
    std::vector<int> cand = {1, 2};
    for (int r : {1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 20, 24}) {
      const int c = fit_seg_rows(shapes, r * cap);
      if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    }
    float best_ms = -1.0f;
    for (int c : cand) {
      for (size_t k = 0; k < n; ++k)
        if ((b->cases[k]->hc.walls ? 1 : 0) == w) b->seg[k] = c;
      e = build_items(b);
      if (e != hipSuccess) {
        rc = bfail(b, DUGKS_EDEVICE, hipGetErrorString(e));
        break;
      }
      float ms = 0.0f;
      rc = probe(ms);
      if (rc) break;
      if (best_ms < 0.0f || ms < best_ms) {
        best_ms = ms;
        best[w] = c;
      }
    }
    if (rc) break;
    for (size_t k = 0; k < n; ++k)
      if ((b->cases[k]->hc.walls ? 1 : 0) == w) b->seg[k] = best[w];
    e = build_items(b);
    if (e != hipSuccess) rc = bfail(b, DUGKS_EDEVICE, hipGetErrorString(e));
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (auto* h : b->cases)
    if (!h->numeric_err) (void)dugks::launch_reset(nullptr, 0, h->dflag, b->stream);
  (void)hipStreamSynchronize(b->stream);
  for (void* q : saved)
    if (q) (void)hipFree(q);
  if (rc) return rc;
  if (seg_periodic) *seg_periodic = best[0];
  if (seg_walls) *seg_walls = best[1];
  return DUGKS_OK;
}

int dugks_batch_set_stream(dugks_batch* b, void* stream) {
  if (!b) return DUGKS_EINVAL;
  b->stream = static_cast<hipStream_t>(stream);
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
  return DUGKS_OK;
}

int dugks_batch_step(dugks_batch* b, int nsteps, int use_graph) {
  if (!b || nsteps < 0) return bfail(b, DUGKS_EINVAL, "bad arguments");
  if (use_graph && !b->stream)
    return bfail(b, DUGKS_EINVAL,
                 "use_graph needs a stream set with dugks_batch_set_stream "
                 "(the null stream cannot be captured)");
  for (auto* h : b->cases)
    if (!h->has_state) return bfail(b, DUGKS_ESTATE, "a case has no state");
  int rc = numeric_check(b);
  if (rc) return rc;
  if (nsteps == 0) return DUGKS_OK;
  rc = ensure_built(b);
  if (rc) return rc;
  // the handles' own work must be finished before the batch touches them
  for (auto* h : b->cases)
    if (h->stream != b->stream) BHIPCHK(b, hipStreamSynchronize(h->stream));
  rc = sync_descriptors(b);
  if (rc) return rc;
  if (use_graph) {
    auto itg = b->graphs.find(nsteps);
    if (itg == b->graphs.end()) {
      hipGraph_t g;
      BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      rc = record_steps(b, nsteps);
      hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (rc) return rc;
      if (e != hipSuccess) return bfail(b, DUGKS_EDEVICE, hipGetErrorString(e));
      hipGraphExec_t ex;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return bfail(b, DUGKS_EDEVICE, hipGetErrorString(e));
      itg = b->graphs.emplace(nsteps, ex).first;
    }
    BHIPCHK(b, hipGraphLaunch(itg->second, b->stream));
  } else {
    rc = record_steps(b, nsteps);
    if (rc) return rc;
  }
  b->gstep += nsteps;
  // advance every case's own counters by the steps it actually took
  for (size_t k = 0; k < b->cases.size(); ++k) {
    dugks_handle* h = b->cases[k];
    long long took = nsteps;
    if (b->budget[k] >= 0) {
      took = std::min<long long>(nsteps, b->budget[k]);
      b->budget[k] -= took;
    }
    if (took > 0) {
      BHIPCHK(b, dugks::launch_advance(h->step_base, took, b->stream));
      h->steps += took;
    }
  }
  return DUGKS_OK;
}

int dugks_batch_sync(dugks_batch* b) {
  if (!b) return DUGKS_EINVAL;
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  for (auto* h : b->cases) {
    if (!h->has_state) continue;
    const int rc = poll_flag(h);
    if (rc) return bfail(b, rc, h->err);
  }
  return numeric_check(b);
}

int dugks_batch_destroy(dugks_batch* b) {
  if (!b) return DUGKS_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);  // work left unjoined by an error
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  if (b->dcases) (void)hipFree(b->dcases);
  for (int w = 0; w < 2; ++w)
    if (b->items[w]) (void)hipFree(b->items[w]);
  if (b->step_base) (void)hipFree(b->step_base);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->owns)
    for (auto* h : b->cases) dugks_destroy(h);
  delete b;
  return DUGKS_OK;
}

const char* dugks_batch_last_error(const dugks_batch* b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
