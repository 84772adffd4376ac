// api.cpp -- host runtime behind the C ABI of include/links.h: argument checks,
// workspace management, the crank table and the launch sequence of one call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/links.h"
#include "common.h"
#include "kernels.h"

namespace {

// The largest double t with sqrt(t) <= 1e-12: a link of squared length d2 is
// longer than 1e-12 exactly when d2 > t (sqrt is monotone and correctly rounded).
double len2_min() {
  static const double t = [] {
    double v = 1e-12 * 1e-12;
    while (std::sqrt(v) > 1e-12) v = std::nextafter(v, 0.0);
    while (std::sqrt(std::nextafter(v, 1.0)) <= 1e-12) v = std::nextafter(v, 1.0);
    return v;
  }();
  return t;
}


thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_CHECK(expr)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(LINKS_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

constexpr int kTimingRing = 64;
struct TimingSet {
  hipEvent_t ev[LINKS_TIMING_PASSES + 1] = {};
  bool used[LINKS_TIMING_PASSES] = {};
};

struct links_ctx {
  int device = 0;
  int num_cu = 0;
  std::map<std::string, Buf> bufs;
  std::map<int, bool> tables;  // crank tables uploaded, by T
  // launch parameters (see links_set_tuning)
  int waves32 = 4;
  int refill_min = 32;
  int waves64 = 1;
  int refill64 = 32;           // refill threshold of the FP64 passes
  int spread = 1;              // FP32 waves start spread over the solve-order buckets
  int chunk = 128;             // list items a wave claims per atomic
  int deesc = 0;               // FP64 steps after a hand-over before returning to FP32 (0: never)
  bool exact_handover = false;  // FP64 hand-over pass with the correctly rounded sequence (else rsq + Newton)
  // FP64 passes computed parallel in time (16-lane segments per candidate):
  // 0 none, 1 the hand-over pass, 2 every FP64 pass.  The return to FP32 after a
  // hand-over (deesc > 0) keeps the step-by-step pass.
  int par64 = 1;
  int seg64 = 8;  // lanes per candidate of the parallel hand-over pass
  // the FP32 pass computed parallel in time (with deesc > 0 the step-by-step pass);
  // off by default: its larger LDS footprint per wave costs more than the idle
  // lanes it saves on the measured workloads
  bool par32 = false;
  // drain hand-off of the FP32 pass: once the work list is exhausted, waves of the
  // step-by-step pass with fewer than drain32 active lanes hand their candidates
  // to the parallel-in-time pass (0: never; 65: every wave at once)
  int drain32 = 0;
  // the FP64 hand-over pass takes the queue ordered by hand-over step, earliest
  // first (the candidates with the most FP64 steps ahead start first); off by
  // default: on the measured workloads the queue as handed over is faster
  bool sort_esc = false;
  // path rows computed in chunks of kPathChunk steps from the sides the decision
  // passes record (else whole, step by step)
  bool path_chunks = true;
  // FP64 passes with one candidate per wave and its positions in registers
  // (up to 20 joints): bit 0 the hand-over pass, bit 1 the path pass (whole rows),
  // bit 2 the FP64 decision pass of FP64 precision
  int wave64 = 0;
  std::map<std::string, int> occ_cache;
  // last call's statistics
  int last_grid32 = 0, last_grid64 = 0;
  // profiling: events around the passes of the last kTimingRing profiled
  // links_simulate calls, one set per call, so that a caller can time many calls
  // and read them afterwards without synchronising in between
  bool profile = false;
  TimingSet ev_ring[kTimingRing];
  int ev_cur = 0;      // set the current profiled call records into
  int ev_last = 0;     // set of the last completed profiled call
  int ev_count = 0;    // completed profiled calls held, at most kTimingRing
  bool ev_open = false;
  // graph capture: passes are enqueued without profiling events, and workspace
  // held by live graphs is never reallocated
  bool capturing = false;
  int graphs = 0;
  // workspace carved from caller-provided device memory instead of allocated
  // (the allocation-free entry point); null: ordinary allocations
  links::Arena* arena = nullptr;
  // pinned host copy of the running retrieval result (FIRST scans)
  uint64_t* hkeys = nullptr;
  size_t hkeys_bytes = 0;
};

struct links_graph {
  links_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int ensure(links_ctx* ctx, const char* name, size_t bytes, void** out) {
  if (links::Arena* ar = ctx->arena) {
    // the next 256-byte aligned piece of the arena; a dry pass only measures
    const size_t off = (ar->used + 255) & ~(size_t)255;
    ar->used = off + bytes;
    if (ar->used > ar->peak) ar->peak = ar->used;
    if (ar->dry) {
      *out = nullptr;
      return LINKS_OK;
    }
    if (ar->used > ar->cap)
      return fail(LINKS_ERR_ARG, "workspace %s does not fit the %zu-byte scratch area", name, ar->cap);
    *out = ar->base + off;
    return LINKS_OK;
  }
  Buf& b = ctx->bufs[name];
  if (b.bytes < bytes) {
    if (ctx->graphs > 0)
      return fail(LINKS_ERR_ARG, "workspace %s must grow but %d graph(s) of this context use it; destroy them first",
                  name, ctx->graphs);
    if (ctx->capturing) return fail(LINKS_ERR_ARG, "workspace %s would be allocated during capture", name);
    if (b.p) {
      hipError_t e = hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
      if (e != hipSuccess) return fail(LINKS_ERR_DEVICE, "hipFree(%s): %s", name, hipGetErrorString(e));
    }
    size_t want = bytes + bytes / 8 + 256;
    if (hipMalloc(&b.p, want) != hipSuccess) {
      b.p = nullptr;
      (void)hipGetLastError();
      return fail(LINKS_ERR_OOM, "workspace allocation of %zu bytes for %s failed", want, name);
    }
    b.bytes = want;
  }
  *out = b.p;
  return LINKS_OK;
}

template <typename T>
int ensure_t(links_ctx* ctx, const char* name, size_t count, T** out) {
  void* p = nullptr;
  int rc = ensure(ctx, name, count * sizeof(T) + 16, &p);
  *out = static_cast<T*>(p);
  return rc;
}

int set_device(links_ctx* ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(LINKS_ERR_DEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
  return LINKS_OK;
}

int check_batch(const links_batch* b) {
  if (!b) return fail(LINKS_ERR_ARG, "batch is NULL");
  if (b->B < 0) return fail(LINKS_ERR_ARG, "B = %d < 0", b->B);
  if (b->J < 1 || b->J > links::kMaxJ) return fail(LINKS_ERR_ARG, "J = %d outside [1, 32]", b->J);
  if (b->B > 0 && (!b->n || !b->adj || !b->fixed || !b->motor))
    return fail(LINKS_ERR_ARG, "batch has a NULL array");
  return LINKS_OK;
}

// The crank table of the allocation-free path: at the start of the arena, room
// for kArenaTableMax steps; uploaded through a fixed host staging buffer in
// pieces (no allocation on either side), and kept while T stays the same.
constexpr int kStage = 512;
std::mutex g_stage_mu;
double2 g_stage64[kStage];
float2 g_stage32[kStage];

int arena_crank_table(links_ctx* ctx, links::Arena* ar, int T, hipStream_t st, float2** cs32, double2** cs64) {
  (void)ctx;
  if (T > links::kArenaTableMax)
    return fail(LINKS_ERR_ARG, "T = %d above %d, the most the allocation-free path holds", T, links::kArenaTableMax);
  if (ar->dry) {
    *cs64 = nullptr;
    *cs32 = nullptr;
    return LINKS_OK;
  }
  *cs64 = reinterpret_cast<double2*>(ar->base);
  *cs32 = reinterpret_cast<float2*>(ar->base + (size_t)links::kArenaTableMax * sizeof(double2));
  if (*ar->table_T == T) return LINKS_OK;
  std::lock_guard<std::mutex> lock(g_stage_mu);
  for (int t0 = 0; t0 < T; t0 += kStage) {
    const int m = T - t0 < kStage ? T - t0 : kStage;
    for (int i = 0; i < m; i++) {
      const int t = t0 + i;
      double theta = 2.0 * M_PI * (double)t / (double)T;
      double c = cos(theta), s = sin(theta);
      g_stage64[i] = make_double2(c, s);
      g_stage32[i] = make_float2((float)c, (float)s);
    }
    HIP_CHECK(hipMemcpyAsync(*cs64 + t0, g_stage64, sizeof(double2) * m, hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(*cs32 + t0, g_stage32, sizeof(float2) * m, hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));  // the staging buffer is reused
  }
  *ar->table_T = T;
  return LINKS_OK;
}

// theta_t = 2 pi t / T, counter-clockwise, evaluated in double on the host; one
// table per T, so that a recorded graph keeps its own table
int crank_table(links_ctx* ctx, int T, hipStream_t st, float2** cs32, double2** cs64) {
  if (links::Arena* ar = ctx->arena) return arena_crank_table(ctx, ar, T, st, cs32, cs64);
  const std::string k64 = "cs64:" + std::to_string(T), k32 = "cs32:" + std::to_string(T);
  int rc = ensure_t(ctx, k64.c_str(), (size_t)T, cs64);
  if (rc) return rc;
  rc = ensure_t(ctx, k32.c_str(), (size_t)T, cs32);
  if (rc) return rc;
  if (!ctx->tables[T]) {
    if (ctx->capturing) return fail(LINKS_ERR_ARG, "crank table would be uploaded during capture");
    std::vector<double> h64(2 * (size_t)T);
    std::vector<float> h32(2 * (size_t)T);
    for (int t = 0; t < T; t++) {
      double theta = 2.0 * M_PI * (double)t / (double)T;
      double c = cos(theta), s = sin(theta);
      h64[2 * t] = c;
      h64[2 * t + 1] = s;
      h32[2 * t] = (float)c;
      h32[2 * t + 1] = (float)s;
    }
    HIP_CHECK(hipMemcpyAsync(*cs64, h64.data(), sizeof(double) * 2 * T, hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(*cs32, h32.data(), sizeof(float) * 2 * T, hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
    ctx->tables[T] = true;
  }
  return LINKS_OK;
}

// records the boundary event before pass i (i == LINKS_TIMING_PASSES: after the last)
int mark(links_ctx* ctx, int i, hipStream_t st) {
  if (!ctx->ev_open) return LINKS_OK;
  TimingSet& s = ctx->ev_ring[ctx->ev_cur];
  if (!s.ev[i]) HIP_CHECK(hipEventCreate(&s.ev[i]));
  HIP_CHECK(hipEventRecord(s.ev[i], st));
  return LINKS_OK;
}

void mark_used(links_ctx* ctx, int i) {
  if (ctx->ev_open) ctx->ev_ring[ctx->ev_cur].used[i] = true;
}

// elapsed milliseconds of each pass of one recorded set
int read_set(links_ctx* ctx, const TimingSet& s, float* ms, int k) {
  HIP_CHECK(hipEventSynchronize(s.ev[LINKS_TIMING_PASSES]));
  for (int i = 0; i < k; i++) {
    ms[i] = 0.f;
    if (s.used[i]) HIP_CHECK(hipEventElapsedTime(&ms[i], s.ev[i], s.ev[i + 1]));
  }
  (void)ctx;
  return LINKS_OK;
}

int grid_for(links_ctx* ctx, const std::string& key, int per_cu) {
  (void)key;
  int g = ctx->num_cu * (per_cu > 0 ? per_cu : 1);
  return g > 0 ? g : 1;
}

}  // namespace

extern "C" {

const char* links_last_error(void) { return g_err.c_str(); }

const char* links_version(void) { return "links-mi355x 0.1 (gfx950)"; }

int links_create(int device, links_ctx** out) {
  if (!out) return fail(LINKS_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return fail(LINKS_ERR_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
  if (device < 0 || device >= count) return fail(LINKS_ERR_ARG, "device %d outside [0, %d)", device, count);
  links_ctx* ctx = new links_ctx();
  ctx->device = device;
  int rc = set_device(ctx);
  if (rc) {
    delete ctx;
    return rc;
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete ctx;
    return fail(LINKS_ERR_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  ctx->num_cu = prop.multiProcessorCount;
  // the device address of this device's allocation-free scratch area, once per device
  if ((rc = links::noalloc_setup(device))) {
    delete ctx;
    return rc;
  }
  *out = ctx;
  return LINKS_OK;
}

void links_destroy(links_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto& set : ctx->ev_ring)
    for (auto& e : set.ev)
      if (e) (void)hipEventDestroy(e);
  for (auto& kv : ctx->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (ctx->hkeys) (void)hipHostFree(ctx->hkeys);
  delete ctx;
}

void links_sim_opts_default(links_sim_opts* o) {
  if (!o) return;
  o->T = 200;
  o->precision = LINKS_FP32_RECHECK;
  o->eps_disc = 1e-6;
  o->eps_branch = 1e-5;
  o->tau_drift = 1e-4;
  o->out_joint = -1;
  o->write = LINKS_WRITE_NONE;
  o->path_dtype = LINKS_F32;
  o->T_prefilter = 0;
  o->branch = LINKS_BRANCH_CONTINUITY;
}

int links_set_tuning(links_ctx* ctx, int waves32, int refill_min, int waves64) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (waves32 < 1 || waves32 > 4 || waves64 < 1 || waves64 > 4 || refill_min < 1 || refill_min > 64)
    return fail(LINKS_ERR_ARG, "tuning out of range (waves 1..4, refill_min 1..64)");
  ctx->waves32 = waves32;
  ctx->refill_min = refill_min;
  ctx->waves64 = waves64;
  return LINKS_OK;
}

int links_set_option(links_ctx* ctx, const char* name, int value) {
  if (!ctx || !name) return fail(LINKS_ERR_ARG, "NULL argument");
  const std::string k(name);
  if (k == "waves32") return links_set_tuning(ctx, value, ctx->refill_min, ctx->waves64);
  if (k == "refill_min") return links_set_tuning(ctx, ctx->waves32, value, ctx->waves64);
  if (k == "waves64") return links_set_tuning(ctx, ctx->waves32, ctx->refill_min, value);
  if (k == "deesc") {
    if (value < 0 || value > 32767) return fail(LINKS_ERR_ARG, "deesc must be in 0..32767");
    ctx->deesc = value;
    return LINKS_OK;
  }
  if (k == "chunk") {
    if (value < 1 || value > 4096) return fail(LINKS_ERR_ARG, "chunk must be in 1..4096");
    ctx->chunk = value;
    return LINKS_OK;
  }
  if (k == "spread") {
    if (value != 0 && value != 1) return fail(LINKS_ERR_ARG, "spread must be 0 or 1");
    ctx->spread = value;
    return LINKS_OK;
  }
  if (k == "refill64") {
    if (value < 1 || value > 64) return fail(LINKS_ERR_ARG, "refill64 must be in 1..64");
    ctx->refill64 = value;
    return LINKS_OK;
  }
  if (k == "exact_handover") {
    if (value != 0 && value != 1) return fail(LINKS_ERR_ARG, "exact_handover must be 0 or 1");
    ctx->exact_handover = value != 0;
    return LINKS_OK;
  }
  if (k == "par32") {
    if (value != 0 && value != 1) return fail(LINKS_ERR_ARG, "par32 must be 0 or 1");
    ctx->par32 = value != 0;
    return LINKS_OK;
  }
  if (k == "path_chunks") {
    if (value != 0 && value != 1) return fail(LINKS_ERR_ARG, "path_chunks must be 0 or 1");
    ctx->path_chunks = value != 0;
    return LINKS_OK;
  }
  if (k == "sort_esc") {
    if (value != 0 && value != 1) return fail(LINKS_ERR_ARG, "sort_esc must be 0 or 1");
    ctx->sort_esc = value != 0;
    return LINKS_OK;
  }
  if (k == "drain32") {
    if (value < 0 || value > 65) return fail(LINKS_ERR_ARG, "drain32 must be in 0..65");
    ctx->drain32 = value;
    return LINKS_OK;
  }
  if (k == "seg64") {
    if (value != 4 && value != 8 && value != 16) return fail(LINKS_ERR_ARG, "seg64 must be 4, 8 or 16");
    ctx->seg64 = value;
    return LINKS_OK;
  }
  if (k == "par64") {
    if (value < 0 || value > 2) return fail(LINKS_ERR_ARG, "par64 must be 0, 1 or 2");
    ctx->par64 = value;
    return LINKS_OK;
  }
  if (k == "wave64") {
    if (value < 0 || value > 7) return fail(LINKS_ERR_ARG, "wave64 must be in 0..7");
    ctx->wave64 = value;
    return LINKS_OK;
  }
  return fail(LINKS_ERR_ARG, "unknown option '%s'", name);
}

int links_get_option(links_ctx* ctx, const char* name, int* value) {
  if (!ctx || !name || !value) return fail(LINKS_ERR_ARG, "NULL argument");
  const std::string k(name);
  if (k == "waves32") *value = ctx->waves32;
  else if (k == "refill_min") *value = ctx->refill_min;
  else if (k == "waves64") *value = ctx->waves64;
  else if (k == "refill64") *value = ctx->refill64;
  else if (k == "chunk") *value = ctx->chunk;
  else if (k == "spread") *value = ctx->spread;
  else if (k == "deesc") *value = ctx->deesc;
  else if (k == "exact_handover") *value = ctx->exact_handover ? 1 : 0;
  else if (k == "par64") *value = ctx->par64;
  else if (k == "seg64") *value = ctx->seg64;
  else if (k == "par32") *value = ctx->par32 ? 1 : 0;
  else if (k == "drain32") *value = ctx->drain32;
  else if (k == "sort_esc") *value = ctx->sort_esc ? 1 : 0;
  else if (k == "path_chunks") *value = ctx->path_chunks ? 1 : 0;
  else if (k == "wave64") *value = ctx->wave64;
  else return fail(LINKS_ERR_ARG, "unknown option '%s'", name);
  return LINKS_OK;
}

int links_get_tuning(links_ctx* ctx, int* waves32, int* refill_min, int* waves64, int* grid32, int* grid64) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (waves32) *waves32 = ctx->waves32;
  if (refill_min) *refill_min = ctx->refill_min;
  if (waves64) *waves64 = ctx->waves64;
  if (grid32) *grid32 = ctx->last_grid32;
  if (grid64) *grid64 = ctx->last_grid64;
  return LINKS_OK;
}

int links_solve_order(links_ctx* ctx, const links_batch* batch, int8_t* order, uint8_t* n_dyads, uint8_t* depth,
                      uint8_t* status, void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  int rc = check_batch(batch);
  if (rc) return rc;
  if (batch->B > 0 && !status) return fail(LINKS_ERR_ARG, "status is NULL");
  rc = set_device(ctx);
  if (rc) return rc;
  if (batch->B == 0) return LINKS_OK;
  links::PrepArgs a;
  memset(&a, 0, sizeof(a));
  a.B = batch->B;
  a.J = batch->J;
  a.n = batch->n;
  a.adj = batch->adj;
  a.fixed = batch->fixed;
  a.motor = batch->motor;
  a.x0 = batch->x0;
  a.order = order;
  a.n_dyads = n_dyads;
  a.depth = depth;
  a.status = status;
  a.sim = 0;
  HIP_CHECK(links::launch_solve_order(a, (hipStream_t)stream));
  return LINKS_OK;
}

}  // extern "C"

namespace {

enum Phase { kPrepare = 0, kRun = 1 };

// kPrepare: argument checks, workspace and crank table only; kRun: the whole call
int simulate_impl(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts, links_sim_out* out,
                  void* stream, int phase, int pre_ratio = 0) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  int rc = check_batch(batch);
  if (rc) return rc;
  if (!opts || !out) return fail(LINKS_ERR_ARG, "opts or out is NULL");
  const int B = batch->B, J = batch->J, T = opts->T;
  if (T < 1 || T > 32767) return fail(LINKS_ERR_ARG, "T = %d outside [1, 32767]", T);
  if (opts->precision < 0 || opts->precision > 2) return fail(LINKS_ERR_ARG, "bad precision %d", opts->precision);
  if (opts->write < 0 || opts->write > 2) return fail(LINKS_ERR_ARG, "bad write mode %d", opts->write);
  if (opts->path_dtype != LINKS_F32 && opts->path_dtype != LINKS_F64)
    return fail(LINKS_ERR_ARG, "bad path dtype %d", opts->path_dtype);
  if (opts->branch != LINKS_BRANCH_CONTINUITY && opts->branch != LINKS_BRANCH_ORIENTATION)
    return fail(LINKS_ERR_ARG, "bad branch rule %d", opts->branch);
  if (opts->out_joint < -1 || opts->out_joint >= J)
    return fail(LINKS_ERR_ARG, "out_joint %d outside [-1, J)", opts->out_joint);
  if (!(opts->eps_disc >= 0) || !(opts->eps_branch >= 0) || !(opts->tau_drift >= 0))
    return fail(LINKS_ERR_ARG, "negative or NaN tolerance");
  if (opts->T_prefilter != 0) {
    const int Tp = opts->T_prefilter;
    if (Tp < 1 || Tp >= T || T % Tp != 0)
      return fail(LINKS_ERR_ARG, "T_prefilter = %d must divide T = %d and be smaller", Tp, T);
    // low-fidelity pass: decisions only, into the caller's status arrays
    links_sim_opts lo = *opts;
    lo.T = Tp;
    lo.T_prefilter = 0;
    lo.write = LINKS_WRITE_NONE;
    links_sim_out lo_out = *out;
    lo_out.path = nullptr;
    lo_out.path_index = nullptr;
    lo_out.n_written = nullptr;
    lo_out.cap = 0;
    int r = simulate_impl(ctx, batch, &lo, &lo_out, stream, phase);
    if (r) return r;
    links_sim_opts hi = *opts;
    hi.T_prefilter = 0;
    return simulate_impl(ctx, batch, &hi, out, stream, phase, T / Tp);
  }
  if (B > 0 && !out->status) return fail(LINKS_ERR_ARG, "status is NULL");
  if (B > 0 && (batch->x0 == nullptr) == (batch->x0_f32 == nullptr))
    return fail(LINKS_ERR_ARG, "exactly one of x0 and x0_f32 must be given");
  if (opts->write == LINKS_WRITE_ALL && B > 0 && !out->path) return fail(LINKS_ERR_ARG, "path is NULL");
  if (opts->write == LINKS_WRITE_VALID &&
      (out->cap < 0 || !out->n_written || (out->cap > 0 && (!out->path_index || !out->path))))
    return fail(LINKS_ERR_ARG, "WRITE_VALID needs cap >= 0, n_written, and path and path_index when cap > 0");
  rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (B == 0) {
    if (opts->write == LINKS_WRITE_VALID) HIP_CHECK(links::launch_fill_u32(out->n_written, 1, 0u, st));
    return LINKS_OK;
  }

  using namespace links;
  // each pass of a call (a low-fidelity screen runs two) carves the arena anew
  // after the crank tables
  if (ctx->arena) ctx->arena->used = kArenaTableBytes;
  // single-precision positions: widened to double once (exactly), then the same path
  links_batch wide;
  if (!batch->x0) {
    double* x0w;
    if ((rc = ensure_t(ctx, "x0_wide", (size_t)B * J * 2, &x0w))) return rc;
    if (phase == kRun) HIP_CHECK(launch_widen(batch->x0_f32, x0w, (size_t)B * J * 2, st));
    wide = *batch;
    wide.x0 = x0w;
    batch = &wide;
  }
  CandMeta* meta;
  CandF32* cf;
  CandF64* cd;
  DyadF32* df;
  DyadF64* dd;
  float2* x0s;
  uint8_t* sj;
  int32_t* perm;
  int32_t* counters;
  EscEntry* esc;
  float2* esc_pos;
  EscEntry* res;
  float2* res_pos;
  EscEntry* esc2;
  float2* esc2_pos;
  int32_t* counters2;
  int16_t* fail_ws;
  int32_t* path_list;
  int32_t* path_row;
  uint8_t* dlen;
  double* scale_ws;
  int16_t* movable_ws;
  int32_t* block_hist;
  int32_t* block_off;
  int32_t* scratch;
  uint32_t* side_ck = nullptr;
  const size_t nblocks = (size_t)prep_blocks(B);
  // Path rows in chunks of kPathChunk steps, each on a lane of its own, starting
  // from the sides the decision passes record at the chunk boundaries (the FP32
  // pass, step by step or parallel in time, for the steps it decides, the FP64
  // passes for theirs).  Rows are computed whole with the return to FP32 after a
  // hand-over or par64 = 2; and without escalation (FP32_ONLY), whose FP32 sides
  // near a tie need not be those the FP64 path pass takes.
  const int ck_n = (T + kPathChunk - 1) / kPathChunk;
  // the FP64 passes a wave-per-candidate kernel runs (up to 20 joints; not with the
  // return to FP32 after a hand-over)
  const bool wave_ok = sim64_wave_fits(J) && ctx->deesc == 0;
  const bool wave_esc = wave_ok && (ctx->wave64 & 1) && ctx->par64 >= 1;
  const bool wave_path = wave_ok && (ctx->wave64 & 2);
  const bool wave_perm = wave_ok && (ctx->wave64 & 4);
  const bool chunks = !wave_path && ctx->path_chunks && opts->write != LINKS_WRITE_NONE &&
                      !(opts->write == LINKS_WRITE_VALID && out->cap == 0) && ck_n > 1 && ctx->par64 != 2 &&
                      (opts->precision == LINKS_FP64 ||
                       (opts->precision == LINKS_FP32_RECHECK && ctx->deesc == 0));
  if (chunks && (rc = ensure_t(ctx, "side_ck", (size_t)B * ck_n, &side_ck))) return rc;
  // drain hand-off: the parallel-in-time pass's counters, its work queue and the
  // handed-on error bounds
  const bool drain = opts->precision != LINKS_FP64 && ctx->drain32 > 0 && !ctx->par32 && ctx->deesc == 0;
  int32_t* cnt_drain = nullptr;
  EscEntry* drain_q = nullptr;
  uint16_t* drain_err = nullptr;
  const bool sort_esc = opts->precision != LINKS_FP64 && ctx->sort_esc && ctx->deesc == 0;
  EscEntry* esc_sorted = nullptr;
  int32_t* esc_work = nullptr;
  if (sort_esc && ((rc = ensure_t(ctx, "esc_sorted", B, &esc_sorted)) ||
                   (rc = ensure_t(ctx, "esc_work", 2 * kEscBins, &esc_work))))
    return rc;
  if (drain && ((rc = ensure_t(ctx, "cnt_drain", kCntSize, &cnt_drain)) ||
                (rc = ensure_t(ctx, "drain_q", B, &drain_q)) ||
                (rc = ensure_t(ctx, "drain_err", (size_t)B * J, &drain_err))))
    return rc;
  if ((rc = ensure_t(ctx, "meta", B, &meta)) || (rc = ensure_t(ctx, "cf", B, &cf)) ||
      (rc = ensure_t(ctx, "cd", B, &cd)) || (rc = ensure_t(ctx, "df", (size_t)B * J, &df)) ||
      (rc = ensure_t(ctx, "dd", (size_t)B * J, &dd)) || (rc = ensure_t(ctx, "x0s", (size_t)B * J, &x0s)) ||
      (rc = ensure_t(ctx, "sj", (size_t)B * J, &sj)) || (rc = ensure_t(ctx, "perm", B, &perm)) ||
      (rc = ensure_t(ctx, "counters", kCntSize, &counters)) || (rc = ensure_t(ctx, "esc", B, &esc)) ||
      (rc = ensure_t(ctx, "esc_pos", (size_t)B * J, &esc_pos)) || (rc = ensure_t(ctx, "fail_ws", B, &fail_ws)) ||
      (rc = ensure_t(ctx, "res", B, &res)) || (rc = ensure_t(ctx, "res_pos", (size_t)B * J, &res_pos)) ||
      (rc = ensure_t(ctx, "esc2", B, &esc2)) || (rc = ensure_t(ctx, "esc2_pos", (size_t)B * J, &esc2_pos)) ||
      (rc = ensure_t(ctx, "counters2", kCntSize, &counters2)) ||
      (rc = ensure_t(ctx, "path_list", B, &path_list)) || (rc = ensure_t(ctx, "path_row", B, &path_row)) ||
      (rc = ensure_t(ctx, "dlen", B, &dlen)) || (rc = ensure_t(ctx, "scale_ws", B, &scale_ws)) ||
      (rc = ensure_t(ctx, "movable_ws", B, &movable_ws)) ||
      (rc = ensure_t(ctx, "block_hist", nblocks * kMaxJ, &block_hist)) ||
      (rc = ensure_t(ctx, "block_off", nblocks * kMaxJ, &block_off)) ||
      (rc = ensure_t(ctx, "compact", compact_scratch_ints(B), &scratch)))
    return rc;
  float2* cs32;
  double2* cs64;
  if ((rc = crank_table(ctx, T, st, &cs32, &cs64))) return rc;
  if (phase == kPrepare) return LINKS_OK;

  const size_t elt = opts->path_dtype == LINKS_F64 ? sizeof(double2) : sizeof(float2);
  if (opts->write == LINKS_WRITE_ALL)
    HIP_CHECK(launch_fill_u32(out->path, (size_t)B * T * elt / 4, 0xFFFFFFFFu, st));  // NaN rows
  HIP_CHECK(launch_fill_u32(counters, kCntSize, 0u, st));
  if (drain) HIP_CHECK(launch_fill_u32(cnt_drain, kCntSize, 0u, st));
  int16_t* fail_step = out->fail_step ? out->fail_step : fail_ws;

  PrepArgs pa;
  memset(&pa, 0, sizeof(pa));
  pa.B = B;
  pa.J = J;
  pa.n = batch->n;
  pa.adj = batch->adj;
  pa.fixed = batch->fixed;
  pa.motor = batch->motor;
  pa.x0 = batch->x0;
  pa.status = out->status;
  pa.sim = 1;
  pa.pre_ratio = pre_ratio;
  pa.out_joint = opts->out_joint;
  pa.eps_disc = opts->eps_disc;
  pa.eps_branch = opts->eps_branch;
  pa.tau_drift = opts->tau_drift;
  pa.len2_min = len2_min();
  pa.fail_step = fail_step;
  pa.esc_step = out->esc_step;
  pa.meta = meta;
  pa.cf = cf;
  pa.cd = cd;
  pa.df = df;
  pa.dd = dd;
  pa.x0s = x0s;
  pa.slot_joint = sj;
  pa.counters = counters;
  pa.Bs = B;
  pa.dlen = dlen;
  pa.scale_ws = scale_ws;
  pa.movable_ws = movable_ws;
  pa.block_hist = block_hist;
  pa.block_off = block_off;
  pa.perm = perm;
  // a profiled call takes the next event set of the ring
  ctx->ev_open = ctx->profile && !ctx->capturing;
  if (ctx->ev_open) {
    ctx->ev_cur = ctx->ev_count == 0 ? 0 : (ctx->ev_last + 1) % kTimingRing;
    if (ctx->ev_count == kTimingRing) ctx->ev_count--;  // the oldest set is re-recorded
    for (int i = 0; i < LINKS_TIMING_PASSES; i++) ctx->ev_ring[ctx->ev_cur].used[i] = false;
  }
  // set-up: validation and solve-order length, bucket offsets, then the records
  // written at each candidate's sorted position (largest solve order first)
  if ((rc = mark(ctx, 0, st))) return rc;
  HIP_CHECK(launch_prep_count(pa, st));
  HIP_CHECK(launch_prep_offsets(pa, st));
  mark_used(ctx, 0);
  if ((rc = mark(ctx, 1, st))) return rc;
  HIP_CHECK(launch_prep_fill(pa, st));
  mark_used(ctx, 1);
  if ((rc = mark(ctx, 2, st))) return rc;

  SimArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.B = B;
  sa.J = J;
  sa.T = T;
  sa.Bs = B;
  sa.n = batch->n;
  sa.adj = batch->adj;
  sa.fixed = batch->fixed;
  sa.motor = batch->motor;
  sa.x0 = batch->x0;
  sa.meta = meta;
  sa.cf = cf;
  sa.cd = cd;
  sa.df = df;
  sa.dd = dd;
  sa.x0s = x0s;
  sa.slot_joint = sj;
  sa.perm = perm;
  sa.counters = counters;
  sa.esc = esc;
  sa.esc_pos = esc_pos;
  sa.path_list = path_list;
  sa.path_row = path_row;
  sa.write_all = opts->write == LINKS_WRITE_ALL;
  sa.cs32 = cs32;
  sa.cs64 = cs64;
  sa.status = out->status;
  sa.fail_step = fail_step;
  sa.esc_step = out->esc_step;
  sa.path = out->path;
  sa.path_f64 = opts->path_dtype == LINKS_F64;
  sa.nslot = J;
  sa.refill_min = ctx->refill_min;
  sa.spread = ctx->spread;
  sa.res = res;
  sa.res_pos = res_pos;
  sa.deesc = 0;
  sa.resume = 0;
  sa.esc_cnt = counters + kCntEsc;
  sa.mig_min = 0;
  sa.chunk = ctx->chunk;
  sa.branch = opts->branch;
  sa.side_ck = side_ck;
  sa.ck_n = chunks ? ck_n : 1;

  LaunchCfg c64;
  c64.waves = ctx->waves64;
  c64.refill_min = 1;
  const int lds64 = sim64_lds_bytes(J, c64.waves);
  const bool fp64 = opts->precision == LINKS_FP64;
  // ---- decisions
  SimArgs sa64 = sa;
  sa64.refill_min = ctx->refill64;
  // an FP64 pass, step by step or parallel in time
  auto run64 = [&](const SimArgs& a, int source, bool exact, LaunchCfg cfg, bool par, bool wave = false) -> hipError_t {
    if (wave) {
      cfg.grid = grid_for(ctx, "wave64", sim64_wave_blocks_per_cu(J, source, exact, cfg.waves));
      return launch_sim64_wave(a, source, exact, cfg, st);
    }
    if (par) {
      cfg.seg = source == kFromEsc ? ctx->seg64 : 16;
      cfg.grid = grid_for(ctx, "par64", sim64_par_blocks_per_cu(J, source, exact, cfg.waves, cfg.seg));
      return launch_sim64_par(a, source, exact, cfg, st);
    }
    cfg.grid = grid_for(ctx, "sim64", sim64_blocks_per_cu(J, source, exact, cfg.waves, lds64));
    return launch_sim64(a, source, exact, cfg, st);
  };
  if (fp64) {
    c64.grid = grid_for(ctx, "sim64", sim64_blocks_per_cu(J, kFromPerm, true, c64.waves, lds64));
    if ((rc = mark(ctx, 3, st))) return rc;
    HIP_CHECK(run64(sa64, kFromPerm, true, c64, ctx->par64 == 2, wave_perm));
    mark_used(ctx, 3);
    ctx->last_grid32 = 0;
  } else {
    LaunchCfg c32;
    c32.waves = ctx->waves32;
    c32.refill_min = ctx->refill_min;
    // mode bit 0: no escalation; bit 2: the pass records the sides at chunk ends;
    // bit 3: the orientation branch rule
    const int mode = (opts->precision == LINKS_FP32_ONLY ? 1 : 0) | (chunks ? 4 : 0) |
                     (opts->branch == LINKS_BRANCH_ORIENTATION ? 8 : 0);
    if (ctx->par32 && ctx->deesc == 0) {
      c32.grid = grid_for(ctx, "par32", sim32_par_blocks_per_cu(J, mode, T, c32.waves));
      HIP_CHECK(launch_sim32_par(sa, mode, c32, st));
    } else {
      const int lds32 = sim32_lds_bytes(J, c32.waves, T);
      c32.grid = grid_for(ctx, "sim32", sim32_blocks_per_cu(J, mode, T, c32.waves, lds32));
      SimArgs s0 = sa;
      if (drain) {
        s0.mig_min = ctx->drain32;
        s0.mig_out = drain_q;
        s0.mig_cnt = cnt_drain + kCntItems;
        s0.mig_err = drain_err;
      }
      HIP_CHECK(launch_sim32(s0, mode, c32, st));
      if (drain) {
        // the candidates the waves handed on, parallel in time from their step
        SimArgs sp = sa;
        sp.counters = cnt_drain;
        sp.resume = 2;
        sp.mig_in = drain_q;
        sp.mig_err = drain_err;
        LaunchCfg cp = c32;
        cp.grid = grid_for(ctx, "par32", sim32_par_blocks_per_cu(J, mode, T, cp.waves));
        HIP_CHECK(launch_sim32_par(sp, mode, cp, st));
      }
    }
    mark_used(ctx, 2);
    c64.grid = grid_for(ctx, "sim64", sim64_blocks_per_cu(J, kFromEsc, ctx->exact_handover, c64.waves, lds64));
    if ((rc = mark(ctx, 3, st))) return rc;
    SimArgs h1 = sa64;
    h1.deesc = ctx->deesc;
    if (sort_esc) {
      HIP_CHECK(launch_sort_esc(B, counters, esc, esc_work, esc_sorted, st));
      h1.esc = esc_sorted;
    }
    const bool par_h = ctx->par64 >= 1 && ctx->deesc == 0;
    HIP_CHECK(run64(h1, kFromEsc, ctx->exact_handover, c64, par_h, wave_esc));
    if (ctx->deesc > 0) {
      // the returned candidates continue in FP32 (their own counters and
      // hand-over queue), and what they hand over again is finished in FP64
      HIP_CHECK(launch_resume_setup(counters, counters2, st));
      SimArgs r32 = sa;
      r32.counters = counters2;
      r32.esc_cnt = counters2 + kCntEsc;
      r32.resume = 1;
      r32.esc = esc2;
      r32.esc_pos = esc2_pos;
      HIP_CHECK(launch_sim32(r32, mode, c32, st));
      SimArgs h2 = sa64;
      h2.counters = counters2;
      h2.esc = esc2;
      h2.esc_pos = esc2_pos;
      h2.deesc = 0;
      HIP_CHECK(launch_sim64(h2, kFromEsc, ctx->exact_handover, c64, st));
    }
    mark_used(ctx, 3);
    ctx->last_grid32 = c32.grid;
  }
  ctx->last_grid64 = c64.grid;
  // ---- compaction of the valid candidates and the list of paths to write
  if ((rc = mark(ctx, 4, st))) return rc;
  if (opts->write == LINKS_WRITE_VALID) {
    HIP_CHECK(launch_compact(B, out->status, scratch, out->path_index, out->cap, out->n_written, path_row, st));
    if (out->cap > 0)
      HIP_CHECK(launch_select_paths(B, perm, out->status, path_row, 0, scratch, path_list, counters, st));
    mark_used(ctx, 4);
  } else if (opts->write == LINKS_WRITE_ALL) {
    HIP_CHECK(launch_select_paths(B, perm, out->status, path_row, 1, scratch, path_list, counters, st));
    mark_used(ctx, 4);
  }
  // ---- path pass: the output joint of every selected candidate, step by step,
  // written straight into its output row
  if ((rc = mark(ctx, 5, st))) return rc;
  if (opts->write != LINKS_WRITE_NONE && !(opts->write == LINKS_WRITE_VALID && out->cap == 0)) {
    HIP_CHECK(run64(sa64, kFromPath, fp64, c64, ctx->par64 == 2, wave_path));
    mark_used(ctx, 5);
  }
  if ((rc = mark(ctx, 6, st))) return rc;
  if (ctx->ev_open) {
    ctx->ev_last = ctx->ev_cur;
    ctx->ev_count++;
  }
  ctx->ev_open = false;
  return LINKS_OK;
}

}  // namespace

extern "C" {

int links_simulate(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts, links_sim_out* out,
                   void* stream) {
  return simulate_impl(ctx, batch, opts, out, stream, kRun);
}

}  // extern "C"

namespace links {

int ctx_device(const links_ctx* ctx) { return ctx->device; }

int report_error(int code, const char* msg) { return fail(code, "%s", msg); }

// links_simulate with every workspace buffer carved from [base, base + cap): a dry
// pass measures the call's needs (no device work), then the call runs with
// profiling events off (creating them would allocate)
int simulate_in_arena(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts, links_sim_out* out,
                      void* stream, unsigned char* base, size_t cap, int* table_T) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (ctx->capturing) return fail(LINKS_ERR_ARG, "the context is capturing a graph");
  Arena dry{nullptr, cap, kArenaTableBytes, kArenaTableBytes, true, table_T};
  ctx->arena = &dry;
  int rc = simulate_impl(ctx, batch, opts, out, stream, kPrepare);
  ctx->arena = nullptr;
  if (rc) return rc;
  if (dry.peak > cap)
    return fail(LINKS_ERR_ARG,
                "B = %d, J = %d needs %zu bytes of workspace, above the %zu-byte allocation-free scratch area",
                batch->B, batch->J, dry.peak, cap);
  Arena run{base, cap, kArenaTableBytes, kArenaTableBytes, false, table_T};
  const bool prof = ctx->profile;
  ctx->profile = false;
  ctx->arena = &run;
  rc = simulate_impl(ctx, batch, opts, out, stream, kRun);
  ctx->arena = nullptr;
  ctx->profile = prof;
  return rc;
}

}  // namespace links

extern "C" {

int links_generate_dyads(links_ctx* ctx, uint64_t seed, int64_t first, int32_t B, int32_t J, int32_t n_lo,
                         int32_t n_hi, int32_t paper_mode, uint8_t* n, uint32_t* adj, uint32_t* fixed,
                         uint8_t* motor, double* x0, void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (B < 0 || first < 0) return fail(LINKS_ERR_ARG, "B = %d or first = %lld is negative", B, (long long)first);
  if (J < 3 || J > links::kMaxJ) return fail(LINKS_ERR_ARG, "J = %d outside [3, 32]", J);
  if (n_lo < 3 || n_lo > n_hi || n_hi > J)
    return fail(LINKS_ERR_ARG, "joint counts [%d, %d] not within [3, J = %d]", n_lo, n_hi, J);
  if (paper_mode < 0 || paper_mode > 3) return fail(LINKS_ERR_ARG, "paper_mode must be in 0..3");
  if ((paper_mode & 2) && n_lo < 5) return fail(LINKS_ERR_ARG, "the topology rules need at least 5 joints");
  if (B > 0 && (!n || !adj || !fixed || !motor || !x0)) return fail(LINKS_ERR_ARG, "NULL output array");
  int rc = set_device(ctx);
  if (rc) return rc;
  links::GenArgs g;
  g.seed = seed;
  g.first = first;
  g.B = B;
  g.J = J;
  g.n_lo = n_lo;
  g.n_hi = n_hi;
  g.paper_mode = paper_mode & 1;
  g.rules = (paper_mode >> 1) & 1;
  g.n = n;
  g.adj = adj;
  g.fixed = fixed;
  g.motor = motor;
  g.x0 = x0;
  HIP_CHECK(links::launch_gen_dyads(g, (hipStream_t)stream));
  return LINKS_OK;
}

int links_curate(links_ctx* ctx, const links_batch* batch, const int32_t* path_index, const int32_t* count,
                 int32_t cap, int32_t out_joint, const float* norm_paths, int32_t T, double circle_var,
                 uint8_t* flags, float* radial_var, uint32_t* keep, void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  int rc = check_batch(batch);
  if (rc) return rc;
  if (cap < 0) return fail(LINKS_ERR_ARG, "cap = %d < 0", cap);
  if (T < 1) return fail(LINKS_ERR_ARG, "T = %d < 1", T);
  if (out_joint < -1 || out_joint >= batch->J) return fail(LINKS_ERR_ARG, "out_joint %d outside [-1, J)", out_joint);
  if (!path_index && cap > batch->B) return fail(LINKS_ERR_ARG, "cap %d > B %d without path_index", cap, batch->B);
  if (cap > 0 && (!norm_paths || !flags || !radial_var || !keep)) return fail(LINKS_ERR_ARG, "NULL array");
  if (!(circle_var >= 0)) return fail(LINKS_ERR_ARG, "circle_var must be >= 0");
  if ((rc = set_device(ctx))) return rc;
  links::CurateArgs a;
  a.J = batch->J;
  a.T = T;
  a.cap = cap;
  a.out_joint = out_joint;
  a.n = batch->n;
  a.adj = batch->adj;
  a.fixed = batch->fixed;
  a.motor = batch->motor;
  a.path_index = path_index;
  a.count = count;
  a.norm = norm_paths;
  a.circle_var = circle_var;
  a.flags = flags;
  a.radial_var = radial_var;
  a.keep = keep;
  HIP_CHECK(links::launch_curate(a, (hipStream_t)stream));
  return LINKS_OK;
}

int links_graph_create(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts, links_sim_out* out,
                       links_graph** graph) {
  if (!graph) return fail(LINKS_ERR_ARG, "graph is NULL");
  *graph = nullptr;
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (ctx->capturing) return fail(LINKS_ERR_ARG, "context is already capturing");
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t st = nullptr;
  HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  // workspace and crank table first, outside the capture
  rc = simulate_impl(ctx, batch, opts, out, st, kPrepare);
  if (rc == LINKS_OK) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(LINKS_ERR_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  hipGraph_t g = nullptr;
  if (rc == LINKS_OK) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      rc = fail(LINKS_ERR_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    } else {
      ctx->capturing = true;
      rc = simulate_impl(ctx, batch, opts, out, st, kRun);
      ctx->capturing = false;
      e = hipStreamEndCapture(st, &g);
      if (rc == LINKS_OK && e != hipSuccess) rc = fail(LINKS_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
  }
  hipGraphExec_t x = nullptr;
  if (rc == LINKS_OK) {
    hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail(LINKS_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  (void)hipStreamDestroy(st);
  if (rc != LINKS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  links_graph* out_g = new links_graph();
  out_g->ctx = ctx;
  out_g->graph = g;
  out_g->exec = x;
  ctx->graphs++;
  *graph = out_g;
  return LINKS_OK;
}

int links_gather(links_ctx* ctx, const uint8_t* buf, const links_piece* pieces, int32_t npieces, int32_t count,
                 const links_batch* out, void* stream) {
  if (!ctx || !out) return fail(LINKS_ERR_ARG, "ctx or out is NULL");
  if (out->J < 1 || out->J > links::kMaxJ) return fail(LINKS_ERR_ARG, "out J = %d outside [1, 32]", out->J);
  if (count < 0 || count > out->B) return fail(LINKS_ERR_ARG, "count = %d outside [0, B = %d]", count, out->B);
  if (count > 0 && (npieces < 1 || !buf || !pieces)) return fail(LINKS_ERR_ARG, "no pieces for %d rows", count);
  if (out->B > 0 && (!out->n || !out->adj || !out->fixed || !out->motor || !out->x0))
    return fail(LINKS_ERR_ARG, "output batch has a NULL array (x0 must be f64)");
  int rc = set_device(ctx);
  if (rc) return rc;
  HIP_CHECK(links::launch_gather(buf, pieces, npieces, count, out->B, out->J, const_cast<uint8_t*>(out->n),
                                 const_cast<uint32_t*>(out->adj), const_cast<uint32_t*>(out->fixed),
                                 const_cast<uint8_t*>(out->motor), const_cast<double*>(out->x0),
                                 (hipStream_t)stream));
  return LINKS_OK;
}

int links_graph_launch(links_graph* graph, void* stream) {
  if (!graph || !graph->exec) return fail(LINKS_ERR_ARG, "graph is NULL");
  int rc = set_device(graph->ctx);
  if (rc) return rc;
  HIP_CHECK(hipGraphLaunch(graph->exec, (hipStream_t)stream));
  return LINKS_OK;
}

void links_graph_destroy(links_graph* graph) {
  if (!graph) return;
  (void)hipSetDevice(graph->ctx->device);
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  graph->ctx->graphs--;
  delete graph;
}

int links_profile(links_ctx* ctx, int enable) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  ctx->profile = enable != 0;
  ctx->ev_count = 0;
  ctx->ev_cur = ctx->ev_last = 0;
  ctx->ev_open = false;
  return LINKS_OK;
}

int links_last_timings(links_ctx* ctx, float* ms, int n) {
  if (!ctx || (!ms && n > 0)) return fail(LINKS_ERR_ARG, "NULL argument");
  if (ctx->ev_count == 0) return fail(LINKS_ERR_ARG, "no profiled links_simulate call");
  int rc = set_device(ctx);
  if (rc) return rc;
  const int k = n < LINKS_TIMING_PASSES ? (n > 0 ? n : 0) : LINKS_TIMING_PASSES;
  if ((rc = read_set(ctx, ctx->ev_ring[ctx->ev_last], ms, k))) return rc;
  return k;
}

int links_mean_timings(links_ctx* ctx, int calls, float* ms, int n) {
  if (!ctx || (!ms && n > 0)) return fail(LINKS_ERR_ARG, "NULL argument");
  if (calls < 1 || calls > ctx->ev_count)
    return fail(LINKS_ERR_ARG, "calls = %d outside [1, %d profiled calls held]", calls, ctx->ev_count);
  int rc = set_device(ctx);
  if (rc) return rc;
  const int k = n < LINKS_TIMING_PASSES ? (n > 0 ? n : 0) : LINKS_TIMING_PASSES;
  float sum[LINKS_TIMING_PASSES] = {}, one[LINKS_TIMING_PASSES];
  for (int c = 0; c < calls; c++) {
    const int slot = ((ctx->ev_last - c) % kTimingRing + kTimingRing) % kTimingRing;
    if ((rc = read_set(ctx, ctx->ev_ring[slot], one, k))) return rc;
    for (int i = 0; i < k; i++) sum[i] += one[i];
  }
  for (int i = 0; i < k; i++) ms[i] = sum[i] / (float)calls;
  return k;
}

int links_normalize_paths(links_ctx* ctx, const float* paths, int32_t P, int32_t T, int32_t mode, float* out,
                          float* xform, void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (P < 0) return fail(LINKS_ERR_ARG, "P = %d < 0", P);
  if (T < 1 || T > 4096) return fail(LINKS_ERR_ARG, "T = %d outside [1, 4096]", T);
  if (mode != LINKS_NORM_PCA && mode != LINKS_NORM_DIAMETER) return fail(LINKS_ERR_ARG, "bad mode %d", mode);
  if (P > 0 && (!paths || !out || !xform)) return fail(LINKS_ERR_ARG, "NULL array");
  int rc = set_device(ctx);
  if (rc) return rc;
  HIP_CHECK(links::launch_normalize(paths, P, nullptr, T, mode, out, xform, (hipStream_t)stream));
  return LINKS_OK;
}

int links_normalize_paths_n(links_ctx* ctx, const float* paths, const int32_t* count, int32_t cap, int32_t T,
                            int32_t mode, float* out, float* xform, void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  if (cap < 0) return fail(LINKS_ERR_ARG, "cap = %d < 0", cap);
  if (T < 1 || T > 4096) return fail(LINKS_ERR_ARG, "T = %d outside [1, 4096]", T);
  if (mode != LINKS_NORM_PCA && mode != LINKS_NORM_DIAMETER) return fail(LINKS_ERR_ARG, "bad mode %d", mode);
  if (cap > 0 && (!paths || !out || !xform || !count)) return fail(LINKS_ERR_ARG, "NULL array");
  int rc = set_device(ctx);
  if (rc) return rc;
  HIP_CHECK(links::launch_normalize(paths, cap, count, T, mode, out, xform, (hipStream_t)stream));
  return LINKS_OK;
}


namespace {

int check_chamfer(const float* bank, int32_t P, int32_t T, const float* queries, int32_t Q) {
  if (P < 0) return fail(LINKS_ERR_ARG, "P = %d < 0", P);
  if (Q < 0) return fail(LINKS_ERR_ARG, "Q = %d < 0", Q);
  if (T < 1 || T > links::kChamferMaxT) return fail(LINKS_ERR_ARG, "T = %d outside [1, %d]", T, links::kChamferMaxT);
  if (P > 0 && Q > 0 && (!bank || !queries)) return fail(LINKS_ERR_ARG, "NULL array");
  return LINKS_OK;
}

// waves per query: twice the resident waves of the chip over all queries, at
// most one per bank path
int32_t chamfer_waves(links_ctx* ctx, int32_t T, int64_t Q, int64_t P) {
  const std::string key = "chamfer" + std::to_string(links::chamfer_na(T));
  auto it = ctx->occ_cache.find(key);
  if (it == ctx->occ_cache.end()) it = ctx->occ_cache.emplace(key, links::chamfer_blocks_per_cu(T)).first;
  const int64_t resident = (int64_t)ctx->num_cu * it->second * 4;
  int64_t w = (2 * resident + Q - 1) / std::max<int64_t>(Q, 1);
  w = std::min<int64_t>(w, std::max<int64_t>(P, 1));
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(w, 1 << 20));
}

}  // namespace

int links_chamfer(links_ctx* ctx, const float* bank, int32_t P, int32_t T, const float* queries, int32_t Q,
                  float* dist, void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  int rc = check_chamfer(bank, P, T, queries, Q);
  if (rc) return rc;
  if (P == 0 || Q == 0) return LINKS_OK;
  if (!dist) return fail(LINKS_ERR_ARG, "dist is NULL");
  rc = set_device(ctx);
  if (rc) return rc;
  links::ChamferArgs a{};
  a.bank = reinterpret_cast<const float2*>(bank);
  a.P = P;
  a.T = T;
  a.queries = reinterpret_cast<const float2*>(queries);
  a.Q = Q;
  a.p_lo = 0;
  a.p_hi = P;
  a.waves_per_query = chamfer_waves(ctx, T, Q, P);
  a.dist = dist;
  HIP_CHECK(links::launch_chamfer(a, (hipStream_t)stream));
  return LINKS_OK;
}

int links_chamfer_search(links_ctx* ctx, const float* bank, int32_t P, int32_t T, const float* queries,
                         int32_t Q, int32_t k, float cutoff, int32_t order, int64_t* idx, float* dist,
                         void* stream) {
  if (!ctx) return fail(LINKS_ERR_ARG, "ctx is NULL");
  int rc = check_chamfer(bank, P, T, queries, Q);
  if (rc) return rc;
  if (k < 1 || k > links::kChamferKeep) return fail(LINKS_ERR_ARG, "k = %d outside [1, %d]", k, links::kChamferKeep);
  if (cutoff != cutoff) return fail(LINKS_ERR_ARG, "cutoff is NaN");
  if (order != LINKS_SEARCH_FIRST && order != LINKS_SEARCH_BEST) return fail(LINKS_ERR_ARG, "bad order %d", order);
  if (Q == 0) return LINKS_OK;
  if (!idx || !dist) return fail(LINKS_ERR_ARG, "NULL output array");
  rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  links::ChamferArgs a{};
  a.bank = reinterpret_cast<const float2*>(bank);
  a.P = P;
  a.T = T;
  a.queries = reinterpret_cast<const float2*>(queries);
  a.Q = Q;
  a.k = k;
  a.cutoff = cutoff;
  a.order = order == LINKS_SEARCH_FIRST ? links::kChamferFirst : links::kChamferBest;
  a.waves_per_query = P > 0 ? chamfer_waves(ctx, T, Q, P) : 0;
  const size_t nrun = (size_t)Q * links::kChamferKeep;
  void *part = nullptr, *running = nullptr;
  rc = ensure(ctx, "chamfer_part", std::max<size_t>(1, nrun * a.waves_per_query) * sizeof(uint64_t), &part);
  if (rc) return rc;
  rc = ensure(ctx, "chamfer_run", nrun * sizeof(uint64_t), &running);
  if (rc) return rc;
  a.part = static_cast<uint64_t*>(part);
  a.running = static_cast<const uint64_t*>(running);
  uint64_t* run = static_cast<uint64_t*>(running);
  HIP_CHECK(links::launch_chamfer_clear(run, (int64_t)nrun, st));
  if (a.order == links::kChamferBest || P == 0) {
    a.p_lo = 0;
    a.p_hi = P;
    HIP_CHECK(links::launch_chamfer(a, st));
    HIP_CHECK(links::launch_chamfer_merge(a, run, idx, dist, st));
    HIP_CHECK(hipStreamSynchronize(st));
    return LINKS_OK;
  }
  // FIRST: chunks in bank order, growing geometrically; after each, the host
  // reads the running result and stops once every query holds k matches
  if (ctx->hkeys_bytes < nrun * sizeof(uint64_t)) {
    if (ctx->hkeys) (void)hipHostFree(ctx->hkeys);
    ctx->hkeys = nullptr;
    ctx->hkeys_bytes = 0;
    void* h = nullptr;
    if (hipHostMalloc(&h, nrun * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
      return fail(LINKS_ERR_OOM, "hipHostMalloc(%zu) failed", nrun * sizeof(uint64_t));
    ctx->hkeys = static_cast<uint64_t*>(h);
    ctx->hkeys_bytes = nrun * sizeof(uint64_t);
  }
  int64_t chunk = (int64_t)a.waves_per_query * 2;
  for (int64_t lo = 0; lo < P;) {
    a.p_lo = lo;
    a.p_hi = std::min<int64_t>(P, lo + chunk);
    HIP_CHECK(links::launch_chamfer(a, st));
    HIP_CHECK(links::launch_chamfer_merge(a, run, idx, dist, st));
    lo = a.p_hi;
    if (lo >= P) break;
    HIP_CHECK(hipMemcpyAsync(ctx->hkeys, run, nrun * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    bool all = true;
    for (int32_t q = 0; q < Q && all; q++) all = ctx->hkeys[(size_t)q * links::kChamferKeep + k - 1] != ~0ull;
    if (all) break;
    chunk = std::min<int64_t>(chunk * 2, (int64_t)a.waves_per_query * 1024);
  }
  HIP_CHECK(hipStreamSynchronize(st));
  return LINKS_OK;
}

}  // extern "C"
