// kernels.h -- launchers of the device kernels (internal to liblinks.so).
#pragma once
#include "common.h"
#include "links.h"

namespace links {

// counters[] layout (int32 in device memory)
constexpr int kCntNext = 0;     // next work item of the simulation pass
constexpr int kCntItems = 1;    // work items of the simulation pass
constexpr int kCntEsc = 2;      // candidates handed to FP64
constexpr int kCntEscNext = 3;  // next hand-over item taken by the FP64 pass
constexpr int kCntValid = 4;    // valid candidates (compaction)
constexpr int kCntPath = 5;     // candidates whose path is written
constexpr int kCntPathNext = 6;
constexpr int kCntHist = 8;     // [32] histogram of solve-order lengths
constexpr int kCntOff = 40;     // [32] bucket offsets
constexpr int kCntCur = 72;     // [32] next item of each bucket (FP32 pass)
constexpr int kCntRes = 104;    // candidates returned from the FP64 hand-over to FP32
constexpr int kCntSize = 112;

// Workspace carved from a fixed device area instead of allocated (the
// allocation-free entry point).  The area starts with the crank tables of up to
// kArenaTableMax steps (FP64 then FP32); the call's buffers follow, each at a
// 256-byte boundary.  A dry pass only measures what a call needs.
constexpr int kArenaTableMax = 4096;
constexpr size_t kArenaTableBytes = (size_t)kArenaTableMax * (sizeof(double2) + sizeof(float2));
struct Arena {
  unsigned char* base;  // device address of the area (null on a dry pass)
  size_t cap;           // its size in bytes
  size_t used;          // end of the last piece carved
  size_t peak;          // largest end over the passes of one call
  bool dry;
  int* table_T;         // steps of the crank table the area holds now (-1: none)
};

struct PrepArgs {
  int32_t B, J;
  const uint8_t* n;
  const uint32_t* adj;
  const uint32_t* fixed;
  const uint8_t* motor;
  const double* x0;
  // solve-order outputs (nullable)
  int8_t* order;
  uint8_t* n_dyads;
  uint8_t* depth;
  uint8_t* status;
  // simulation records (sim != 0)
  int32_t sim;
  int32_t pre_ratio;  // > 0: candidates whose status is not VALID keep it (low-fidelity rejects)
  int32_t out_joint;
  double eps_disc, eps_branch, tau_drift;
  double len2_min;  // largest double whose square root is at most 1e-12 (shortest link)
  int16_t* fail_step;
  int16_t* esc_step;
  CandMeta* meta;
  CandF32* cf;
  CandF64* cd;
  DyadF32* df;
  DyadF64* dd;
  float2* x0s;
  uint8_t* slot_joint;
  int32_t* counters;
  // sorting by solve-order length (records are written at the sorted position)
  int32_t Bs;            // stride of the per-entry record arrays
  uint8_t* dlen;         // [B] solve-order length, 0xFF when not simulated
  int32_t* block_hist;   // [32][blocks]: candidates of each solve-order length per count workgroup
  int32_t* block_off;    // [32][blocks]: their exclusive prefix within the bucket
  int32_t* perm;         // [B] candidate at each sorted position
  double* scale_ws;      // [B] longest link of each pending candidate (count -> fill)
  int16_t* movable_ws;   // [B] its links not between two fixed joints (count -> fill)
};

hipError_t launch_solve_order(const PrepArgs& a, hipStream_t st);
int prep_blocks(int32_t B);
hipError_t launch_prep_count(const PrepArgs& a, hipStream_t st);
hipError_t launch_prep_offsets(const PrepArgs& a, hipStream_t st);
hipError_t launch_prep_fill(const PrepArgs& a, hipStream_t st);
hipError_t launch_fill_u32(void* p, size_t n_u32, uint32_t v, hipStream_t st);
hipError_t launch_widen(const float* in, double* out, size_t n, hipStream_t st);
// counters of a resume round: every returned candidate in one bucket (prep.hip)
hipError_t launch_resume_setup(const int32_t* counters, int32_t* counters2, hipStream_t st);

// on-device candidate generation (gen.hip)
struct GenArgs {
  uint64_t seed;
  int64_t first;   // index of the first candidate in the seed's sequence
  int64_t B;
  int32_t J, n_lo, n_hi, paper_mode;
  int32_t rules;   // the paper's topology rules (irreducible, last joint not on a fixed joint)
  uint8_t* n;
  uint32_t* adj;
  uint32_t* fixed;
  uint8_t* motor;
  double* x0;
};
hipError_t launch_gen_dyads(const GenArgs& g, hipStream_t st);

// curation of normalised coupler paths (prep.hip)
struct CurateArgs {
  int32_t J, T, cap, out_joint;
  const uint8_t* n;
  const uint32_t* adj;
  const uint32_t* fixed;
  const uint8_t* motor;
  const int32_t* path_index;  // nullable: row i belongs to candidate i
  const int32_t* count;       // nullable: cap rows
  const float* norm;          // [cap][T][2] DIAMETER-normalised
  double circle_var;
  uint8_t* flags;
  float* radial_var;
  uint32_t* keep;
};
hipError_t launch_curate(const CurateArgs& a, hipStream_t st);
size_t compact_scratch_ints(int32_t B);
// the hand-over queue (counters[kCntEsc] entries of q) into out, ordered by
// hand-over step in groups of 8 steps, earliest first; work: 2 kEscBins ints
constexpr int kEscBins = 4096;
hipError_t launch_sort_esc(int32_t B, const int32_t* counters, const EscEntry* q, int32_t* work, EscEntry* out,
                           hipStream_t st);
hipError_t launch_compact(int32_t B, const uint8_t* status, int32_t* scratch, int32_t* index, int32_t cap,
                          int32_t* total, int32_t* row_of, hipStream_t st);
// path list over sorted positions: valid candidates with a row (all_simulated = 0)
// or every simulated candidate (1); count in counters[kCntPath]
hipError_t launch_select_paths(int32_t B, const int32_t* perm, const uint8_t* status, const int32_t* row_of,
                               int all_simulated, int32_t* scratch, int32_t* list, int32_t* counters,
                               hipStream_t st);

// Simulation passes.  `grid` = persistent workgroups; block = waves * 64 lanes.
struct LaunchCfg {
  int grid;
  int waves;
  int refill_min;
  int seg = 16;  // lanes per candidate of a parallel-in-time pass (4, 8 or 16)
};
// FP32 pass: mode 0 escalates to FP64, mode 1 never escalates.
hipError_t launch_sim32(const SimArgs& a, int mode, const LaunchCfg& cfg, hipStream_t st);
// the FP32 pass computed parallel in time (16-lane segments per candidate)
hipError_t launch_sim32_par(const SimArgs& a, int mode, const LaunchCfg& cfg, hipStream_t st);
int sim32_par_blocks_per_cu(int J, int mode, int T, int waves);
int sim32_lds_bytes(int nslot, int waves, int T);
constexpr int kTableLds = 1024;  // crank tables up to this many steps live in LDS
int sim32_dmax(int J);
// FP64 pass work sources
constexpr int kFromPerm = 0;    // every pending candidate from t = 0 (plain FP64 precision)
constexpr int kFromEsc = 1;     // candidates handed over by the FP32 pass, from their step
constexpr int kFromPath = 2;    // path pass: candidates whose path is output, from t = 0
// exact: the correctly rounded IEEE sequence (else reciprocal square roots refined
// by Newton steps)
hipError_t launch_sim64(const SimArgs& a, int source, bool exact, const LaunchCfg& cfg, hipStream_t st);
int sim64_lds_bytes(int nslot, int waves);
// occupancy helper: resident workgroups per CU for a kernel variant
int sim32_blocks_per_cu(int J, int mode, int T, int waves, int lds_bytes);
int sim64_blocks_per_cu(int J, int source, bool exact, int waves, int lds_bytes);
// the same passes computed parallel in time (16-lane segments per candidate)
hipError_t launch_sim64_par(const SimArgs& a, int source, bool exact, const LaunchCfg& cfg, hipStream_t st);
int sim64_par_blocks_per_cu(int J, int source, bool exact, int waves, int seg);
// the same passes with one candidate per wave and its positions in registers
// (simwave.hip); up to 20 joints (sim64_wave_fits)
bool sim64_wave_fits(int J);
hipError_t launch_sim64_wave(const SimArgs& a, int source, bool exact, const LaunchCfg& cfg, hipStream_t st);
int sim64_wave_blocks_per_cu(int J, int source, bool exact, int waves);

// Path normalisation, one wave per path.
hipError_t launch_normalize(const float* paths, int32_t P, const int32_t* count, int32_t T, int32_t mode,
                            float* out, float* xform, hipStream_t st);

// Bidirectional chamfer distance and retrieval (chamfer.hip).
constexpr int kChamferKeep = 16;  // largest k of a search
constexpr int kChamferFirst = 0;  // k lowest bank positions under the cut-off
constexpr int kChamferBest = 1;   // k smallest distances under the cut-off
constexpr int kChamferMaxT = 256;

struct ChamferArgs {
  const float2* bank;     // [P][T]
  int64_t P;
  int32_t T;
  const float2* queries;  // [Q][T]
  int64_t Q;
  int64_t p_lo, p_hi;     // bank rows of this launch
  int32_t waves_per_query;
  float* dist;            // [Q][P] or null
  int32_t k;              // 0: no selection
  float cutoff;
  int32_t order;
  uint64_t* part;         // [Q][waves_per_query][kChamferKeep] per-wave lists
  const uint64_t* running;  // [Q][kChamferKeep] result of earlier launches (FIRST: a full one ends the scan)
};

int chamfer_na(int T);
int chamfer_blocks_per_cu(int T);
hipError_t launch_chamfer(const ChamferArgs& a, hipStream_t st);
hipError_t launch_chamfer_merge(const ChamferArgs& a, uint64_t* running, int64_t* idx, float* dist,
                                hipStream_t st);
hipError_t launch_chamfer_clear(uint64_t* running, int64_t n, hipStream_t st);

// serving: the tick's batch gathered from request blocks of their own strides (serve.hip)
hipError_t launch_gather(const uint8_t* buf, const links_piece* pieces, int32_t npieces, int32_t count,
                         int32_t rows, int32_t J, uint8_t* n, uint32_t* adj, uint32_t* fixed, uint8_t* motor,
                         double* x0, hipStream_t st);

// set-up and entry of the allocation-free variant of links_simulate
// (noalloc.hip, api.cpp)
int noalloc_setup(int device);
int simulate_in_arena(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts, links_sim_out* out,
                      void* stream, unsigned char* base, size_t cap, int* table_T);
int ctx_device(const links_ctx* ctx);
int report_error(int code, const char* msg);

}  // namespace links
