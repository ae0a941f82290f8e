// Serving pool of libdugks (declared in include/dugks.h): continuous batching
// of solve requests. Cases of different sizes are admitted into one device
// arena while others run, advance together through batched step launches
// (HIP graphs while the set of running cases is unchanged), and are read out
// and retired on their own. Admission and retirement allocate and free no
// device memory (case states are carved from the arena on the host side), so
// they never synchronize the device; a change of the running set costs one
// synchronization of the pool's stream at the next step call.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "dugks_host.h"

using dugks::CaseDev;
using dugks::Item;
using dugks::StepArgs;
using namespace dugks::host;

struct dugks_pool {
  int precision = 0, model = 0;
  hipStream_t stream = nullptr;
  // device arena for the case states, first-fit with coalescing
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> bytes
  struct Pending {
    size_t off, bytes;
    hipEvent_t done;  // recorded at retirement: the block is free once it has passed
  };
  std::vector<Pending> pending;
  // slots
  int max_cases = 0;
  size_t max_cells = 0;
  std::vector<dugks_handle*> slot;  // nullptr: free
  std::vector<long long> target;    // steps to run
  std::vector<long long> start;     // pool step at admission
  std::vector<size_t> off, bytes;   // arena block of the slot
  CaseDev* sdc = nullptr;           // device: per-slot descriptor (init, readout)
  long long* scount = nullptr;      // device: per-slot step counter (init, readout)
  int* sflags = nullptr;            // device: per-slot non-finite flag (CaseDev::flag)
  std::vector<int> hflags;          // host copy of sflags as of the last dugks_pool_sync
  CaseDev* dcases = nullptr;        // device: per-slot descriptor of the pool steps
  long long* step_base = nullptr;   // device: pool step counter
  long long gstep = 0;              // host mirror
  double* staging = nullptr;        // device: 5 max_cells doubles + diagnostics
  // work items of the running cases (periodic, walls)
  Item* items[2] = {nullptr, nullptr};
  size_t items_cap[2] = {0, 0};
  int nitems[2] = {0, 0};
  int seg[2] = {1, 1};        // rows per segment of each group
  std::vector<char> running;  // slot in the current items
  bool dirty = true;
  std::map<int, hipGraphExec_t> graphs;
  std::vector<CaseDev> hcases;
  std::string err = "no error";

  bool fp64() const { return precision == DUGKS_FP64; }
  bool coupled() const { return model == DUGKS_MODEL_COUPLED; }
  long long done(int k) const { return std::min(target[k], std::max(0LL, gstep - start[k])); }
};

namespace {

constexpr size_t kAlign = 256;

int pfail(dugks_pool* p, int code, const std::string& m) {
  if (p) p->err = m;
  else g_create_error = m;
  return code;
}

#define PHIPCHK(p, expr)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return pfail((p), DUGKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Return [o, o + b) to the free list, merged with free neighbours.
void free_insert(dugks_pool* p, size_t o, size_t b) {
  auto next = p->free_blocks.lower_bound(o);
  if (next != p->free_blocks.end() && o + b == next->first) {  // merge with the block after
    b += next->second;
    next = p->free_blocks.erase(next);
  }
  if (next != p->free_blocks.begin()) {  // merge with the block before
    auto prev = std::prev(next);
    if (prev->first + prev->second == o) {
      prev->second += b;
      return;
    }
  }
  p->free_blocks[o] = b;
}

// Blocks whose retirement the stream has passed go back to the free list.
void reclaim(dugks_pool* p) {
  for (size_t i = 0; i < p->pending.size();) {
    if (hipEventQuery(p->pending[i].done) != hipSuccess) {
      ++i;
      continue;
    }
    (void)hipEventDestroy(p->pending[i].done);
    free_insert(p, p->pending[i].off, p->pending[i].bytes);
    p->pending.erase(p->pending.begin() + i);
  }
  (void)hipGetLastError();  // hipEventQuery reports "not ready" through the error state
}

bool arena_alloc(dugks_pool* p, size_t b, size_t& o) {
  for (auto it = p->free_blocks.begin(); it != p->free_blocks.end(); ++it) {
    if (it->second < b) continue;
    o = it->first;
    const size_t rest = it->second - b;
    p->free_blocks.erase(it);
    if (rest) p->free_blocks[o + b] = rest;
    return true;
  }
  return false;
}

// Work items and descriptors of the cases that still have steps to run.
int rebuild(dugks_pool* p) {
  std::vector<char> run(p->max_cases, 0);
  std::vector<StripShape> shapes[2];
  for (int k = 0; k < p->max_cases; ++k) {
    dugks_handle* h = p->slot[k];
    if (!h || p->done(k) >= p->target[k]) continue;
    run[k] = 1;
    shapes[h->hc.walls ? 1 : 0].push_back(StripShape{h->hc.nstrips, h->ny});
  }
  if (!p->dirty && run == p->running) return DUGKS_OK;
  int* seg = p->seg;
  for (int w = 0; w < 2; ++w)
    seg[w] = shapes[w].empty()
                 ? 1
                 : auto_seg_rows(shapes[w], wave_capacity(p->fp64(), p->coupled(), w == 1),
                                 p->fp64(), w == 1);
  std::vector<Item> it[2];
  for (int k = 0; k < p->max_cases; ++k) {
    CaseDev& c = p->hcases[k];
    if (!run[k]) {
      c.nsteps = 0;  // never launched; keeps a stale entry harmless
      continue;
    }
    dugks_handle* h = p->slot[k];
    const int w = h->hc.walls ? 1 : 0;
    c = h->hc;
    c.cur0 = 0;  // local step 0 was built in buffer 0
    c.seg_rows = seg[w];
    c.nsegs = (c.ny + seg[w] - 1) / seg[w];
    c.step0 = p->start[k];
    c.nsteps = p->target[k];
    for (int s = 0; s < c.nsegs; ++s)
      for (int x = 0; x < c.nstrips; ++x) it[w].push_back(Item{k, x, s, dugks::item_dir(s, w == 1)});
  }
  // captured graphs refer to the old items; drop them before the buffers change
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
  p->graphs.clear();
  for (int w = 0; w < 2; ++w) {
    p->nitems[w] = (int)it[w].size();
    if (it[w].empty()) continue;
    if (it[w].size() > p->items_cap[w]) {  // grows rarely (doubling)
      PHIPCHK(p, hipStreamSynchronize(p->stream));
      if (p->items[w]) PHIPCHK(p, hipFree(p->items[w]));
      p->items[w] = nullptr;
      const size_t cap = std::max(it[w].size(), 2 * p->items_cap[w]);
      PHIPCHK(p, hipMalloc(&p->items[w], cap * sizeof(Item)));
      p->items_cap[w] = cap;
    }
    PHIPCHK(p, hipMemcpyAsync(p->items[w], it[w].data(), it[w].size() * sizeof(Item),
                              hipMemcpyHostToDevice, p->stream));
  }
  PHIPCHK(p, hipMemcpyAsync(p->dcases, p->hcases.data(), p->hcases.size() * sizeof(CaseDev),
                            hipMemcpyHostToDevice, p->stream));
  // the host vectors above are reused at the next rebuild
  PHIPCHK(p, hipStreamSynchronize(p->stream));
  p->running = run;
  p->dirty = false;
  return DUGKS_OK;
}

int record(dugks_pool* p, int nsteps) {
  StepArgs a{};
  a.cases = p->dcases;
  a.step_base = p->step_base;
  for (int k = 0; k < nsteps; ++k) {
    a.kofs = k;
    for (int w = 0; w < 2; ++w) {
      if (p->nitems[w] == 0) continue;
      a.items = p->items[w];
      a.nitems = p->nitems[w];
      a.one_row = p->seg[w] == 1 ? 1 : 0;
      a.two_row = p->seg[w] == 2 ? 1 : 0;
      PHIPCHK(p, dugks::launch_step(p->fp64(), p->coupled(), w == 1, a, p->stream));
    }
  }
  PHIPCHK(p, dugks::launch_advance(p->step_base, nsteps, p->stream));
  return DUGKS_OK;
}

}  // namespace

extern "C" {

int dugks_pool_create(size_t hbm_bytes, int max_cases, long long max_cells, int precision, int model,
                      dugks_pool** out) {
  if (!out) return pfail(nullptr, DUGKS_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_bytes < kAlign || max_cases < 1 || max_cases > 65536 || max_cells < 9)
    return pfail(nullptr, DUGKS_EINVAL, "bad pool sizes");
  if (precision != DUGKS_FP32 && precision != DUGKS_FP64) return pfail(nullptr, DUGKS_EINVAL, "bad precision");
  if (model != DUGKS_MODEL_AC && model != DUGKS_MODEL_COUPLED) return pfail(nullptr, DUGKS_EINVAL, "bad model");
  dugks_pool* p = new (std::nothrow) dugks_pool;
  if (!p) return pfail(nullptr, DUGKS_ENOMEM, "host allocation failed");
  p->precision = precision;
  p->model = model;
  p->max_cases = max_cases;
  p->max_cells = (size_t)max_cells;
  p->arena_bytes = hbm_bytes / kAlign * kAlign;
  p->slot.assign(max_cases, nullptr);
  p->target.assign(max_cases, 0);
  p->start.assign(max_cases, 0);
  p->off.assign(max_cases, 0);
  p->bytes.assign(max_cases, 0);
  p->hcases.assign(max_cases, CaseDev{});
  p->running.assign(max_cases, 0);
  p->hflags.assign(max_cases, 0);
  const size_t staging = 5 * (size_t)max_cells + (size_t)kDiagBlocks * 7 + 16;
  hipError_t e = hipMalloc(&p->arena, p->arena_bytes);
  if (e == hipSuccess) e = hipMalloc(&p->sdc, max_cases * sizeof(CaseDev));
  if (e == hipSuccess) e = hipMalloc(&p->dcases, max_cases * sizeof(CaseDev));
  if (e == hipSuccess) e = hipMalloc(&p->scount, max_cases * sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&p->sflags, max_cases * sizeof(int));
  if (e == hipSuccess) e = hipMemset(p->sflags, 0, max_cases * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&p->step_base, sizeof(long long));
  if (e == hipSuccess) e = hipMalloc(&p->staging, staging * sizeof(double));
  if (e == hipSuccess) e = hipMemset(p->step_base, 0, sizeof(long long));
  if (e == hipSuccess) e = hipMemset(p->dcases, 0, max_cases * sizeof(CaseDev));
  if (e != hipSuccess) {
    std::string m = std::string("pool allocation failed: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    dugks_pool_destroy(p);
    return pfail(nullptr, e == hipErrorOutOfMemory ? DUGKS_ENOMEM : DUGKS_EDEVICE, m);
  }
  p->free_blocks[0] = p->arena_bytes;
  *out = p;
  return DUGKS_OK;
}

int dugks_pool_set_stream(dugks_pool* p, void* stream) {
  if (!p) return DUGKS_EINVAL;
  PHIPCHK(p, hipStreamSynchronize(p->stream));
  p->stream = static_cast<hipStream_t>(stream);
  for (auto* h : p->slot)
    if (h) h->stream = p->stream;
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
  p->graphs.clear();
  return DUGKS_OK;
}

size_t dugks_pool_case_bytes(int nx, int ny, int precision, int model) {
  if (nx < 1 || ny < 1) return 0;
  return 2 * round_up(state_set_bytes(nx, ny, precision, model));
}

}  // extern "C"

namespace {

// A slot and an arena block for a case of nx x ny with parameters prm; the
// new handle has the parameters set and both buffers cleared. `fill` then
// builds local step 0 in buffer 0 on the pool's stream. On success the slot
// is taken and *slot_out set.
template <typename Fill>
int admit_case(dugks_pool* p, int nx, int ny, const dugks_params* prm, long long nsteps,
               int* slot_out, Fill fill) {
  if (nx < 3 || ny < 3) return pfail(p, DUGKS_EINVAL, "nx and ny must be >= 3");
  if ((size_t)nx * ny > p->max_cells) return pfail(p, DUGKS_EINVAL, "case larger than max_cells");
  if ((long long)nx * ny > (1LL << 32) / (4 * (p->fp64() ? 8 : 4)))
    return pfail(p, DUGKS_EINVAL, "grid too large (cells > 2^28 in FP32, 2^27 in FP64)");
  int k = 0;
  while (k < p->max_cases && p->slot[k]) ++k;
  if (k == p->max_cases) return pfail(p, DUGKS_EBUSY, "no free slot");
  const size_t half = round_up(state_set_bytes(nx, ny, p->precision, p->model));
  size_t o = 0;
  reclaim(p);
  if (!arena_alloc(p, 2 * half, o)) return pfail(p, DUGKS_EBUSY, "no room in the arena");
  dugks_handle* h = new (std::nothrow) dugks_handle;
  if (!h) {
    free_insert(p, o, 2 * half);  // never used: straight back
    return pfail(p, DUGKS_ENOMEM, "host allocation failed");
  }
  h->nx = nx;
  h->ny = ny;
  h->precision = p->precision;
  h->model = p->model;
  h->borrowed = true;
  h->stream = p->stream;
  h->buf_bytes = state_set_bytes(nx, ny, p->precision, p->model);
  h->buf[0] = p->arena + o;
  h->buf[1] = p->arena + o + half;
  // the row padding of both buffers reads zero, whatever the arena held
  if (hipMemsetAsync(p->arena + o, 0, 2 * half, p->stream) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    free_insert(p, o, 2 * half);
    return pfail(p, DUGKS_EDEVICE, "clearing the slot's state failed");
  }
  h->dc = p->sdc + k;
  h->step_base = p->scount + k;
  h->dflag = p->sflags + k;
  h->scratch = p->staging;
  int rc = dugks_set_params(h, prm);
  if (rc == DUGKS_OK) rc = fill(h);
  if (rc != DUGKS_OK) {
    std::string m = h->err;
    delete h;
    // the failed init may still be queued: free the block once the stream passes it
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(ev, p->stream) == hipSuccess)
      p->pending.push_back(dugks_pool::Pending{o, 2 * half, ev});
    else
      (void)hipStreamSynchronize(p->stream), free_insert(p, o, 2 * half);
    return pfail(p, rc, m);
  }
  p->slot[k] = h;
  p->hflags[k] = 0;
  p->target[k] = nsteps;
  p->start[k] = p->gstep;
  p->off[k] = o;
  p->bytes[k] = 2 * half;
  p->dirty = true;
  *slot_out = k;
  return DUGKS_OK;
}

}  // namespace

extern "C" {

int dugks_pool_admit(dugks_pool* p, int nx, int ny, const dugks_params* prm, const double* phi,
                     const double* u, const double* v, const double* pr, long long nsteps,
                     int* slot_out) {
  if (!p || !prm || !phi || !slot_out || nsteps < 0) return pfail(p, DUGKS_EINVAL, "bad arguments");
  return admit_case(p, nx, ny, prm, nsteps, slot_out, [&](dugks_handle* h) {
    // host fields into the staging area, then the initial state; all on the
    // pool stream, so the staging area is reused in order
    const size_t n = h->n(), b = n * sizeof(double);
    const double* src[4] = {phi, u, v, pr};
    double* d[4] = {p->staging, p->staging + n, p->staging + 2 * n, p->staging + 3 * n};
    for (int i = 0; i < 4; ++i)
      if (src[i] && hipMemcpyAsync(d[i], src[i], b, hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return hip_fail(h, hipGetLastError(), "hipMemcpyAsync");
    return dugks_init_fields_device(h, d[0], u ? d[1] : nullptr, v ? d[2] : nullptr,
                                    pr ? d[3] : nullptr);
  });
}

int dugks_pool_admit_handle(dugks_pool* p, dugks_handle* src, long long nsteps, int* slot_out) {
  if (!p || !src || !slot_out || nsteps < 0) return pfail(p, DUGKS_EINVAL, "bad arguments");
  if (src->borrowed) return pfail(p, DUGKS_EINVAL, "the handle is a pool case");
  if (src->precision != p->precision || src->model != p->model)
    return pfail(p, DUGKS_EINVAL, "the handle's precision and model must be the pool's");
  if (src->general())
    return pfail(p, DUGKS_EINVAL,
                 "the upwind reconstruction and stretched meshes run on single handles only");
  if (!src->has_state) return pfail(p, DUGKS_ESTATE, "the handle has no state (init_fields first)");
  // the handle's queued steps must be done before its state is copied
  if (hipStreamSynchronize(src->stream) != hipSuccess)
    return pfail(p, DUGKS_EDEVICE, "synchronising the handle's stream failed");
  if (poll_flag(src) != DUGKS_OK) return pfail(p, DUGKS_EDEVICE, src->err);
  if (src->numeric_err) return pfail(p, DUGKS_ENUMERIC, "the handle's state is non-finite");
  const int cur = (src->hc.cur0 + (int)(src->steps & 1)) & 1;
  return admit_case(p, src->nx, src->ny, &src->params, nsteps, slot_out, [&](dugks_handle* h) {
    // the handle's current state becomes local step 0 (buffer 0) at its time
    h->hc.cur0 = 0;
    h->hc.step0 = 0;
    h->hc.t0 = src->hc.t0 + (double)src->steps * src->hc.dt;
    HIPCHK(h, hipMemcpyAsync(h->dc, &h->hc, sizeof(CaseDev), hipMemcpyHostToDevice, p->stream));
    HIPCHK(h, hipMemcpyAsync(h->buf[0], src->buf[cur], src->buf_bytes, hipMemcpyDeviceToDevice,
                             p->stream));
    HIPCHK(h, dugks::launch_reset(h->step_base, 0, h->dflag, p->stream));
    // h->hc is a member of the new handle: the copy above may run later
    HIPCHK(h, hipStreamSynchronize(p->stream));
    h->steps = 0;
    h->has_state = true;
    return DUGKS_OK;
  });
}

int dugks_pool_step(dugks_pool* p, int nsteps, int use_graph) {
  if (!p || nsteps < 0) return pfail(p, DUGKS_EINVAL, "bad arguments");
  if (use_graph && !p->stream)
    return pfail(p, DUGKS_EINVAL,
                 "use_graph needs a stream set with dugks_pool_set_stream "
                 "(the null stream cannot be captured)");
  if (nsteps == 0) return DUGKS_OK;
  int rc = rebuild(p);
  if (rc) return rc;
  if (p->nitems[0] + p->nitems[1] == 0) return DUGKS_OK;  // nothing to run
  if (use_graph) {
    auto itg = p->graphs.find(nsteps);
    if (itg == p->graphs.end()) {
      hipGraph_t g;
      PHIPCHK(p, hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
      rc = record(p, nsteps);
      hipError_t e = hipStreamEndCapture(p->stream, &g);
      if (rc) return rc;
      if (e != hipSuccess) return pfail(p, DUGKS_EDEVICE, hipGetErrorString(e));
      hipGraphExec_t ex;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return pfail(p, DUGKS_EDEVICE, hipGetErrorString(e));
      itg = p->graphs.emplace(nsteps, ex).first;
    }
    PHIPCHK(p, hipGraphLaunch(itg->second, p->stream));
  } else {
    rc = record(p, nsteps);
    if (rc) return rc;
  }
  p->gstep += nsteps;
  return DUGKS_OK;
}

long long dugks_pool_steps_done(const dugks_pool* p, int k) {
  if (!p || k < 0 || k >= p->max_cases || !p->slot[k]) return -1;
  return p->done(k);
}

long long dugks_pool_remaining(const dugks_pool* p, int k) {
  if (!p || k < 0 || k >= p->max_cases || !p->slot[k]) return -1;
  return p->target[k] - p->done(k);
}

int dugks_pool_get_macros(dugks_pool* p, int k, double* phi, double* u, double* v, double* pr,
                          double* rho) {
  if (!p || k < 0 || k >= p->max_cases || !p->slot[k]) return pfail(p, DUGKS_EINVAL, "bad slot");
  dugks_handle* h = p->slot[k];
  h->steps = p->done(k);  // local step the state is at once the stream has run
  const int rc = dugks_get_macros(h, phi, u, v, pr, rho);
  if (rc) return pfail(p, rc, h->err);
  if (h->numeric_err) {
    p->hflags[k] = 1;
    return pfail(p, DUGKS_ENUMERIC, "non-finite values in the state of slot " + std::to_string(k));
  }
  return DUGKS_OK;
}

int dugks_pool_status(const dugks_pool* p, int k) {
  if (!p || k < 0 || k >= p->max_cases || !p->slot[k]) return DUGKS_EINVAL;
  return p->hflags[k] ? DUGKS_ENUMERIC : DUGKS_OK;
}

int dugks_pool_retire(dugks_pool* p, int k) {
  if (!p || k < 0 || k >= p->max_cases || !p->slot[k]) return pfail(p, DUGKS_EINVAL, "bad slot");
  hipEvent_t ev;
  PHIPCHK(p, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  PHIPCHK(p, hipEventRecord(ev, p->stream));
  p->pending.push_back(dugks_pool::Pending{p->off[k], p->bytes[k], ev});
  delete p->slot[k];
  p->slot[k] = nullptr;
  p->target[k] = 0;
  p->dirty = true;
  return DUGKS_OK;
}

size_t dugks_pool_bytes_free(dugks_pool* p) {
  if (!p) return 0;
  reclaim(p);
  size_t f = 0;
  for (auto& b : p->free_blocks) f += b.second;
  return f;
}

int dugks_pool_sync(dugks_pool* p) {
  if (!p) return DUGKS_EINVAL;
  PHIPCHK(p, hipMemcpyAsync(p->hflags.data(), p->sflags, p->hflags.size() * sizeof(int),
                            hipMemcpyDeviceToHost, p->stream));
  PHIPCHK(p, hipStreamSynchronize(p->stream));
  for (int k = 0; k < p->max_cases; ++k) {
    if (!p->slot[k]) p->hflags[k] = 0;
    else if (p->hflags[k]) p->slot[k]->numeric_err = true;
  }
  return DUGKS_OK;
}

const char* dugks_pool_last_error(const dugks_pool* p) {
  return p ? p->err.c_str() : g_create_error.c_str();
}

int dugks_pool_destroy(dugks_pool* p) {
  if (!p) return DUGKS_OK;
  (void)hipStreamSynchronize(p->stream);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
  for (auto& q : p->pending) (void)hipEventDestroy(q.done);
  for (auto* h : p->slot) delete h;
  if (p->arena) (void)hipFree(p->arena);
  if (p->sdc) (void)hipFree(p->sdc);
  if (p->dcases) (void)hipFree(p->dcases);
  if (p->scount) (void)hipFree(p->scount);
  if (p->sflags) (void)hipFree(p->sflags);
  if (p->step_base) (void)hipFree(p->step_base);
  if (p->staging) (void)hipFree(p->staging);
  for (int w = 0; w < 2; ++w)
    if (p->items[w]) (void)hipFree(p->items[w]);
  delete p;
  return DUGKS_OK;
}

}  // extern "C"
