// common.h -- internal definitions shared by the kernels and the host runtime of
// liblinks.so.  Nothing here is part of the public ABI (include/links.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace links {

constexpr int kMaxJ = 32;
constexpr int kWave = 64;

// internal status of a candidate that still has to be simulated
constexpr uint8_t kPending = 255;

// per-candidate flags written by the prep kernel
constexpr uint32_t kFlagRedundant = 1u;  // has links outside the solve order (drift checks)
constexpr uint32_t kFlagNoPath = 2u;     // requested output joint does not exist

// ---------------------------------------------------------------------------
// Per-candidate records produced once per mechanism by the prep kernel.  Slots
// are the LDS positions used during simulation: joint of solve-order entry s is
// in slot s, the tip in slot D, the fixed joints after it in ascending index.
struct CandMeta {
  uint8_t D;         // placed joints (solve-order entries)
  uint8_t n;         // joints
  uint8_t out_slot;  // slot of the output joint
  uint8_t flags;     // kFlag*
};

// relative rounding unit of an FP32 placement: four units of 2^-24
constexpr float kRoundUnit = 0x1p-22f;

// FP32 constants of one candidate (thresholds are already scaled)
struct CandF32 {
  float px, py;  // pivot
  float vx, vy;  // tip - pivot at t = 0
  float U;       // rounding-error unit of a computed position
  float KB;      // escalation band on K: 4 eps_disc scale^4
  float CD;      // escalation band on d^2: eps_disc scale^2
  float EB;      // escalation band on the branch distance: eps_branch scale
  float U2;      // rounding of one placement relative to the link lengths: u 2 scale
  float TS;      // 2 scale, a bound on 2 ra in the branch error term
  float u;       // relative rounding unit of a placement (kRoundUnit)
  float DG;      // degenerate threshold 1e-12 scale^2 (FP32-only mode)
  uint32_t side; // bit s: placed joint s starts left of its parents' line a->b
  float pad[3];
};

// FP64 constants of one candidate
struct CandF64 {
  double px, py, vx, vy;
  double scale;
  double deg_thr;  // 1e-12 scale^2
  double drift_thr;  // tau scale
  uint64_t side;     // as CandF32::side
};

// FP32 per-entry constants, rounded from FP64: S = (ra + rb)^2, Dm = (ra - rb)^2,
// Kc = (ra^2 - rb^2)/2; parent slots packed as a | b << 8.
struct DyadF32 {
  float S, Dm, Kc;
  uint32_t slots;
};

// FP64 per-entry constants, computed exactly as the reference arithmetic does
struct DyadF64 {
  double ra2, rb2;  // squared initial link lengths to parents a and b
  double S, Dm;     // (ra + rb)^2 and (ra - rb)^2 with ra = sqrt(ra2), rb = sqrt(rb2)
};

// A candidate handed from the FP32 pass to the FP64 pass.
struct EscEntry {
  int32_t item;   // sorted position of the candidate (its records)
  int16_t t;      // step to recompute in FP64
  int8_t from_x0;    // 1: start from x0 at step 0 (links outside the solve order)
  int8_t pad;
};

// steps per chunk of a path row (a power of two, and a multiple of the 8- and
// 4-step write groups of the path pass)
constexpr int kPathChunk = 32;

// Pointers of the workspace and of the caller's batch, passed by value to kernels.
struct SimArgs {
  // batch
  int32_t B, J, T;
  const uint8_t* n;
  const uint32_t* adj;
  const uint32_t* fixed;
  const uint8_t* motor;
  const double* x0;
  // records, stored at the sorted position p: per candidate [p], per entry or
  // slot [s * Bs + p]
  int32_t Bs;
  CandMeta* meta;
  CandF32* cf;
  CandF64* cd;
  DyadF32* df;      // [J][Bs]
  DyadF64* dd;      // [J][Bs]
  float2* x0s;      // [J][Bs] initial positions in slot order (FP32)
  uint8_t* slot_joint;  // [J][Bs] joint in each slot
  // scheduling
  int32_t* perm;    // [B] candidate at each sorted position (largest D first)
  int32_t* counters;  // [0] next work item, [1] work items, [2] escalations, [3] next esc item, [4..] D histogram
  EscEntry* esc;    // [B]
  int32_t* path_list;  // [B] sorted positions of the candidates whose path is written
  int32_t* path_row;   // [B] output row of each valid candidate (WRITE_VALID), -1 beyond cap
  int32_t write_all;   // every simulated candidate's path is output (row = candidate)
  float2* esc_pos;  // [B][J] FP32 slot positions at hand-over, row = the candidate's sorted position
  // crank table
  const float2* cs32;   // [T] (cos, sin) rounded from FP64
  const double2* cs64;  // [T]
  // outputs
  uint8_t* status;
  int16_t* fail_step;
  int16_t* esc_step;
  void* path;          // [rows][T][2] or null
  int32_t path_f64;    // element type
  int32_t nslot;       // LDS slots per lane (max n)
  int32_t refill_min;  // refill a wave when at least this many lanes are idle
  int32_t spread;      // FP32 pass: waves start spread over the buckets (1) or all in the largest (0)
  int32_t chunk;       // items a wave claims with one atomic
  int32_t branch;      // LINKS_BRANCH_CONTINUITY or LINKS_BRANCH_ORIENTATION (side bits of the records)
  // Side bits of every placed joint (bit s: dyad s on the left of its parents'
  // line) after step k * kPathChunk - 1, k = 1 .. ck_n - 1, by candidate
  // ([B][ck_n], entry 0 unused): written by the step-by-step FP64 decision pass,
  // read by the path pass, which then computes each chunk of kPathChunk steps of
  // a row on its own lane (null: rows computed whole).
  uint32_t* side_ck;
  int32_t ck_n;
  // returning to FP32 after a hand-over: the FP64 pass stops a candidate deesc
  // steps after its hand-over step and queues it (res, res_pos); a resume round of
  // the FP32 pass (resume = 1) takes its work items from that queue
  EscEntry* res;       // [B] (sorted position, next step)
  float2* res_pos;     // [B][J] slot positions at the end of the last FP64 step
  int32_t deesc;       // 0: the FP64 pass finishes every candidate it takes
  int32_t resume;      // FP32 pass work items: 0 the sorted list, 1 the FP64 pass's returns (res),
                       // 2 (parallel-in-time pass) the candidates the step-by-step pass handed on
  // Drain hand-off of the FP32 pass.  Once the work list is exhausted, a wave of
  // the step-by-step pass with fewer than mig_min active lanes stops: each active
  // lane's column goes to esc_pos and its error bounds to mig_err (at the
  // candidate's sorted position), and (sorted position, next step) to mig_out,
  // counted in *mig_cnt.  The parallel-in-time pass (resume = 2) then carries
  // them on bit for bit from mig_in, with full segments.  mig_min = 0: none.
  int32_t mig_min;
  EscEntry* mig_out;
  int32_t* mig_cnt;
  const EscEntry* mig_in;
  uint16_t* mig_err;       // [B][J] error bounds (as the pass stores them) by sorted position
  int32_t* esc_cnt;        // hand-over queue counter shared by the launches of the FP32 pass
};

}  // namespace links
