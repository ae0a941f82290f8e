// Host-side internals of libdugks shared by the handle API (dugks_api.cpp)
// and the serving pool (dugks_pool.cpp): the handle, and the helpers that
// fill and upload a case descriptor and launch its steps.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dugks.h"
#include "dugks_impl.h"


struct dugks_handle {
  int nx = 0, ny = 0, precision = 0, model = 0;
  dugks_params params{};
  bool has_params = false, has_state = false;
  hipStream_t stream = nullptr;
  void* buf[2] = {nullptr, nullptr};
  size_t buf_bytes = 0;
  dugks::CaseDev hc{};
  dugks::CaseDev* dc = nullptr;
  dugks::Item* items = nullptr;
  int nitems = 0;
  // work items of the reconstruction march (general() handles)
  dugks::Item* uitems = nullptr;
  int nuitems = 0;
  int upm_rows = 0;  // rows per segment of the reconstruction march in use
  int seg_rows = 0;  // 0: automatic
  long long* step_base = nullptr;  // device: steps done
  long long steps = 0;             // host mirror
  int* dflag = nullptr;            // device: non-finite flag of the state (CaseDev::flag)
  bool numeric_err = false;        // sticky: a synchronising call found the flag set
  double* scratch = nullptr;       // 5 n doubles (macros) + diag partials + out
  // stretched mesh: host widths, and the device metric arrays (CaseDev::mesh)
  bool mesh = false;
  std::vector<double> mdx, mdy;
  double* dmesh = nullptr;
  std::string err = "no error";
  bool dirty_case = true;
  // a case of a serving pool: its buffers, descriptor, counter and scratch
  // belong to the pool, which also launches its steps
  bool borrowed = false;
  // step sequences replayed from HIP graphs (a created stream only): nsteps
  // and its graph, valid while the launch signature gsig is unchanged
  std::vector<std::pair<int, hipGraphExec_t>> graphs;
  std::vector<long long> gsig;

  bool fp64() const { return precision == DUGKS_FP64; }
  bool upwind() const { return params.recon == DUGKS_RECON_UPWIND; }
  // steps run as the reconstruction march (k_upm: the upwind reconstruction,
  // or a stretched mesh) instead of k_step's
  bool general() const { return upwind() || mesh; }
  bool coupled() const { return model == DUGKS_MODEL_COUPLED; }
  size_t n() const { return (size_t)nx * ny; }
  size_t elem() const { return fp64() ? 8 : 4; }
};

namespace dugks {
namespace host {

constexpr double kRT = 1.0 / 3.0;
constexpr int kDiagBlocks = 256;

// error of the last failed create (no handle to hold it)
extern thread_local std::string g_create_error;

int fail(dugks_handle* h, int code, const std::string& msg);
int hip_fail(dugks_handle* h, hipError_t e, const char* what);

#define HIPCHK(h, expr)                                    \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail((h), e_, #expr); \
  } while (0)

// Resident step waves on the current device (CUs x waves per CU).
int wave_capacity(bool fp64, bool coupled, bool walls);

// Shape of the step work of one case: strips of 62 columns, and rows.
struct StripShape {
  int nstrips, ny;
};
long long tile_count(const std::vector<StripShape>& cs, int seg);
int fit_seg_rows(const std::vector<StripShape>& cs, long long budget);
// Automatic segment length of a group of cases (fp64, walls: the group's
// precision and boundary, which decide whether the two-row kernel applies).
int auto_seg_rows(const std::vector<StripShape>& cs, long long capacity, bool fp64, bool walls);
// Automatic segment length of the reconstruction march of a handle.
int auto_upm_rows(const dugks_handle* h);
// Compute units of the current device.
long long cu_count();

// Derived constants of the handle's parameters into h->hc, and the upload of
// the descriptor (and, for a plain handle, of its work items).
void fill_case(dugks_handle* h);
int upload_case(dugks_handle* h);
int validate(const dugks_handle* h, const dugks_params* p, std::string& why);
size_t state_set_bytes(int nx, int ny, int precision, int model);
int ensure_scratch(dugks_handle* h);
int launch_steps(dugks_handle* h, int nsteps);
// After the handle's stream has been synchronised: read its non-finite flag;
// a set flag makes the numeric error sticky (until init or set_state).
int poll_flag(dugks_handle* h);

}  // namespace host
}  // namespace dugks
