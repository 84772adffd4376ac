/* links.h -- C ABI of liblinks.so: batched kinematic simulation of one-degree-of-
 * freedom planar linkages on AMD Instinct MI355X (gfx950).
 *
 * The operations follow the LINKS paper (Nobari, Srivastava, Gutfreund, Ahmed,
 * arXiv 2208.14567):
 *   - a mechanism is an undirected graph given by its adjacency matrix plus, per
 *     joint, a type (fixed, free, actuated) and an initial position; link lengths
 *     are the initial distances (Methodology, "Mechanism Representation");
 *   - the actuator arm joins a fixed pivot and an actuated tip, joints 0 and 1 in
 *     the paper's dataset (Methodology, "Dataset Features & Statistics", item 1);
 *   - the graphical solver finds, once per mechanism, the order in which joints
 *     with two known neighbours can be placed (Methodology, "Graphical
 *     Simulator");
 *   - a mechanism is valid when the actuator completes a full rotation, sampled
 *     at T equally spaced positions (200 in the dataset, 50 in the low-fidelity
 *     pass), without locking (Methodology, "Finding Valid Initial Positions",
 *     "Scale of Infeasibilities", "Dataset Features & Statistics" item 2);
 *   - paths are normalised for comparison (Methodology, "Dataset Curation &
 *     Processing").
 *
 * General conventions
 *   - Every entry point returns LINKS_OK (0) or a negative error code; the text
 *     of the last error on the calling thread is in links_last_error().
 *   - Problems of a single candidate never fail a call: they are reported in its
 *     status entry.
 *   - All array pointers are DEVICE pointers (hipMalloc'd or equivalent) owned by
 *     the caller; the library never keeps them after the call returns and never
 *     frees them.  Calls are asynchronous on `stream` (a hipStream_t passed as
 *     void*, NULL = the null stream); outputs are valid once the stream has
 *     completed, and inputs must stay alive until then.
 *   - A context owns device workspace that grows on demand; one context must not
 *     be used by two threads at the same time.  Calls that overlap on one context
 *     through different streams are not supported.
 */
#ifndef LINKS_H
#define LINKS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define LINKS_OK 0
#define LINKS_ERR_ARG (-1)    /* null pointer, size out of range, bad option */
#define LINKS_ERR_DEVICE (-2) /* a HIP runtime call failed */
#define LINKS_ERR_OOM (-3)    /* workspace allocation failed */

/* ---- per-candidate status ---- */
#define LINKS_VALID 0       /* full rotation without locking */
#define LINKS_LOCKED 1      /* two parent circles do not meet at some step */
#define LINKS_DEGENERATE 2  /* the two parents coincide (d^2 <= 1e-12 scale^2) */
#define LINKS_DRIFT 3       /* a redundant link changed length by > tau*scale */
#define LINKS_UNSOLVABLE 4  /* the graphical solver cannot place every joint */
#define LINKS_BAD_MECH 5    /* malformed input (see links_solve_order) */

/* ---- precisions for links_simulate ---- */
#define LINKS_FP32_RECHECK 0 /* FP32 with escalation to FP64 (default) */
#define LINKS_FP64 1         /* plain FP64 throughout */
#define LINKS_FP32_ONLY 2    /* FP32 without escalation (diagnostic) */

/* ---- path output modes ---- */
#define LINKS_WRITE_NONE 0
#define LINKS_WRITE_ALL 1   /* path[B][T][2]; NaN from fail_step on */
#define LINKS_WRITE_VALID 2 /* compacted: path[cap][T][2] + path_index[cap] */

/* ---- path element types ---- */
#define LINKS_F32 0
#define LINKS_F64 1

/* ---- normalisation ---- */
#define LINKS_NORM_PCA 0      /* centroid, RMS radius 1, principal axis on +x */
#define LINKS_NORM_DIAMETER 1 /* longest chord on +x, length 1, box centred at (0.5, 0.5) */
#define LINKS_NF_CONSTANT 1   /* all points coincide: output zeros */
#define LINKS_NF_ISOTROPIC 2  /* principal axis undefined (circle-like): no rotation */
#define LINKS_NF_SIGN_TIE 4   /* third moment ~ 0: axis sign kept as found */
#define LINKS_NF_DIAM_TIE 8   /* another chord within 1e-6 of the longest */

typedef struct links_ctx links_ctx;

/* Creates a context bound to HIP device `device` (the device is made current for
 * the calls of this context).  *out receives the context. */
int links_create(int device, links_ctx** out);
void links_destroy(links_ctx* ctx);

/* Message of the last failing call on this thread ("" if none).  The pointer is
 * valid until the next call on the same thread. */
const char* links_last_error(void);

/* Version string of the library (static storage). */
const char* links_version(void);

/* A batch of B candidates with a per-candidate joint stride J (1 <= J <= 32).
 * Layout of the representation in the paper's Methodology, "Mechanism
 * Representation": adjacency matrix rows as bitmasks, a fixed-joint mask in
 * place of type 0, the motor pair in place of the actuated type, and x0.
 *   n     uint8  [B]       joint count, 3 <= n <= J
 *   adj   uint32 [B][J]    bit j of adj[c][i] set iff joints i and j are linked
 *   fixed uint32 [B]       bit i set iff joint i is a ground (fixed) joint
 *   motor uint8  [B][2]    (pivot, tip): pivot fixed, tip free, link pivot-tip present
 *   x0    double [B][J][2] initial positions; entries beyond n are ignored
 *   x0_f32 float  [B][J][2] the same in single precision, used when x0 is NULL
 *                          (the values are widened to double exactly, so results
 *                          equal those of x0 holding the same numbers); exactly
 *                          one of x0 and x0_f32 must be non-NULL when B > 0      */
typedef struct {
  int32_t B, J;
  const uint8_t* n;
  const uint32_t* adj;
  const uint32_t* fixed;
  const uint8_t* motor;
  const double* x0;
  const float* x0_f32;
} links_batch;

/* Graphical solve order (Methodology, "Graphical Simulator"): starting from the
 * fixed joints and the tip, each round places, in ascending joint index, every
 * unknown joint with at least two known neighbours, using the two smallest known
 * neighbours as parents.
 * Outputs (device, [B] unless stated):
 *   order   int8 [B][J][3]  (joint, parent a, parent b) per placed joint, -1 padded
 *   n_dyads placed joints; depth = number of rounds
 *   status  LINKS_VALID (all joints placed), LINKS_UNSOLVABLE, or LINKS_BAD_MECH
 *           when n is outside [3, J], adj is not symmetric, has a diagonal bit or
 *           a bit at or beyond n, fixed has a bit at or beyond n, or the motor
 *           pair is not (fixed pivot, free tip) joined by a link.
 * Any output pointer except status may be NULL. */
int links_solve_order(links_ctx* ctx, const links_batch* batch, int8_t* order, uint8_t* n_dyads,
                      uint8_t* depth, uint8_t* status, void* stream);

typedef struct {
  int32_t T;           /* actuator positions per revolution, theta_t = 2 pi t / T, 1..32767 */
  int32_t precision;   /* LINKS_FP32_RECHECK | LINKS_FP64 | LINKS_FP32_ONLY */
  double eps_disc;     /* escalation band on disc = K/(4 scale^2), in units of scale^2 (1e-6) */
  double eps_branch;   /* escalation band on the branch distance, in units of scale (1e-5) */
  double tau_drift;    /* redundant-link drift limit, in units of scale (1e-4) */
  int32_t out_joint;   /* joint whose path is written; -1 = last joint of the solve order */
  int32_t write;       /* LINKS_WRITE_NONE | LINKS_WRITE_ALL | LINKS_WRITE_VALID */
  int32_t path_dtype;  /* LINKS_F32 | LINKS_F64 */
  int32_t T_prefilter; /* 0: off.  Otherwise the low-fidelity check of "Scale of
                        * Infeasibilities": every candidate is first simulated at
                        * T_prefilter positions (T must be a multiple of it); those
                        * that fail keep that status, with fail_step converted to the
                        * same angle on the T grid (t * T / T_prefilter) and
                        * esc_step -1, and only the survivors are simulated at T */
  int32_t branch;      /* side of each placed joint, which the paper leaves open
                        * (Methodology, "Graphical Simulator"; "Computational Cost of
                        * Simulations"): LINKS_BRANCH_CONTINUITY (default) the
                        * intersection nearer the joint's previous position (ties:
                        * left of a->b); LINKS_BRANCH_ORIENTATION the side of its
                        * parents' line a->b on which the joint lies in x0 (decided
                        * once per candidate in FP64, so no band is needed for it) */
} links_sim_opts;

#define LINKS_BRANCH_CONTINUITY 0
#define LINKS_BRANCH_ORIENTATION 1

/* Fills opts with the defaults above (T = 200, WRITE_NONE, F32). */
void links_sim_opts_default(links_sim_opts* opts);

typedef struct {
  uint8_t* status;     /* [B] required */
  int16_t* fail_step;  /* [B] nullable; step of the first failure, -1 if none */
  int16_t* esc_step;   /* [B] nullable; step at which FP32 handed over to FP64, -1 if never */
  void* path;          /* see write mode; element type path_dtype */
  int32_t* path_index; /* WRITE_VALID: [cap] candidate index of each written path, ascending */
  int32_t* n_written;  /* WRITE_VALID: [1] number of valid candidates (may exceed cap) */
  int32_t cap;         /* WRITE_VALID: rows available in path / path_index */
} links_sim_out;

/* Full-rotation simulation of every candidate.  Decisions (status, fail_step) come
 * from the FP32 pass and the FP64 hand-over pass (or the FP64 pass alone); the
 * paths of the selected candidates are then recomputed by a path pass in FP64
 * (the correctly rounded sequence in FP64 precision, reciprocal square roots with
 * a Newton step otherwise) and written straight into their rows.  Per step t the tip is turned by
 * theta_t about the pivot, fixed joints stay at x0, and every joint of the solve
 * order is placed at an intersection of the circles about its two parents (radii
 * = initial link lengths).  Of the two intersections the one nearer the joint's
 * previous position is taken (the initial position at t = 0).  A candidate fails
 * at the first step where two circles miss (LOCKED), its parents coincide
 * (DEGENERATE) or a link outside the solve order drifts (DRIFT); decisions are
 * taken in step order, then solve order.  Link lengths must exceed 1e-12 and
 * positions must be finite, else BAD_MECH.
 * FP32_RECHECK runs FP32 and hands a candidate over to the FP64 arithmetic at the
 * first step where a decision lies within eps (or within the tracked FP32 error
 * bound) of its threshold; FP64 results are identical to a correctly rounded
 * double evaluation of the same formulas. */
int links_simulate(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts,
                   links_sim_out* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): links_simulate with the
 * same arguments, kernels and results, whose workspace (records, work lists,
 * hand-over queues, crank tables) lives in one fixed device array of
 * LINKS_NOALLOC_SCRATCH_BYTES per GPU instead of memory the context allocates.
 * The call allocates nothing, on the device or the host, and records no timing
 * events.  The array is held by each GPU the library runs on until the process
 * ends; links_create looks up its address on the context's device.  A call
 * needs about (185 + 81 J) bytes per candidate (plus 16 J with x0_f32 input, and
 * 4 ceil(T / 32) when path rows are written) after 96 KiB of crank tables: at
 * J = 20 and T = 200 about 37,000 candidates fit.  Errors:
 * those of links_simulate; LINKS_ERR_ARG, before any device work, when the call
 * needs more than the array holds or T > 4096.  Every call on a GPU shares that
 * GPU's array and leaves its contents behind (what must start at zero is cleared
 * by each call): calls that overlap in time on one GPU race, so issue them on one
 * stream or synchronise them. */
#define LINKS_NOALLOC_SCRATCH_BYTES (64u << 20)
int links_simulate_noalloc(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts,
                           links_sim_out* out, void* stream);

/* Serving support (no operation of the paper: the batching step of a serving
 * loop that runs the simulation of the Methodology over requests of any size).
 * Gathers into one batch the candidates of several requests,
 * each stored in a byte buffer at its own joint stride, so that a request takes
 * the device memory of its own layout.  A request block of `size` candidates at
 * stride J (1..32) holds, each part starting 16-byte aligned from the block's
 * start (itself 16-byte aligned in buf): x0 [size][J][2] f64, adj [size][J]
 * u32, fixed [size] u32, n [size] u8, motor [size][2] u8.  Piece p fills rows
 * dst[p] .. dst[p+1]-1 (the last piece up to `count`) of the output batch with
 * candidates first[p], first[p]+1, ... of its request; pieces are in ascending
 * dst from 0.  Rows count .. out->B-1 get n = 0 (BAD_MECH, never simulated).
 * adj words and x0 pairs beyond a request's stride are zero.  buf, pieces and
 * the output arrays are device pointers (out->x0 as f64), owned by the caller;
 * the call is asynchronous on `stream`.  Pieces are device data and are not
 * checked on the host: each must describe a block inside buf; a row whose piece
 * has J outside [1, out->J] or a candidate index outside [0, size) is left
 * empty (n = 0), and so is a candidate with more joints than its request's
 * stride (links_simulate at that stride reports it BAD_MECH, as it does n = 0).  Errors: LINKS_ERR_ARG for NULL arrays, count outside
 * [0, out->B], npieces < 1 with count > 0, or out->J outside [1, 32]. */
typedef struct {
  int64_t src;   /* byte offset of the request's block in buf */
  int32_t dst;   /* first output row of the piece */
  int32_t first; /* index within the request of the piece's first candidate */
  int32_t size;  /* candidates in the request's block */
  int32_t J;     /* the request's stride */
} links_piece;
int links_gather(links_ctx* ctx, const uint8_t* buf, const links_piece* pieces, int32_t npieces, int32_t count,
                 const links_batch* out, void* stream);

/* Launch parameters of the simulation passes (chosen by the autotuner in the
 * Python layer, or set by hand): waves32 / waves64 = wavefronts per workgroup of
 * the FP32 / FP64 pass (1..4); refill_min = idle lanes a wave waits for before it
 * fetches new candidates (1..64).  Returns LINKS_ERR_ARG outside these ranges. */
int links_set_tuning(links_ctx* ctx, int waves32, int refill_min, int waves64);
/* Named integer options (LINKS_ERR_ARG for an unknown name or value):
 *   "waves32", "refill_min", "waves64"  as in links_set_tuning;
 *   "deesc"           FP32_RECHECK: a candidate handed over to FP64 returns to FP32
 *                     after this many FP64 steps (positions rounded to FP32, error
 *                     bounds restarted as at t = 0); what it hands over again is
 *                     finished in FP64.  0 (default) keeps it in FP64 to the end;
 *   "chunk"           list items a wave claims with one atomic operation and
 *                     then hands to its lanes as they free up (1..4096, default 128);
 *   "spread"          1 (default): waves of the FP32 pass start spread over the
 *                     solve-order buckets in proportion to their sizes; 0: all
 *                     start in the largest bucket and move down together;
 *   "refill64"        idle lanes a wave of the FP64 passes waits for before it
 *                     fetches new candidates (1..64, default 32);
 *   "exact_handover"  0 (default): the FP64 hand-over pass uses reciprocal square
 *                     roots refined by a Newton step (relative error ~5e-15); 1: the
 *                     correctly rounded sequence of the FP64 precision (the
 *                     operations of an IEEE double evaluation, as in LINKS_FP64);
 *   "par64"           which FP64 passes run parallel in time: 16 lanes share one
 *                     candidate, each computing one step with every dyad on an
 *                     assumed side, checked against the continuity rule and
 *                     restarted where the rule changes side (results identical to
 *                     the step-by-step pass).  0: none; 1 (default): the hand-over
 *                     pass (whose long FP64 runs are few); 2: every FP64 pass;
 *   "seg64"           lanes per candidate of the parallel hand-over pass: 4, 8
 *                     (default) or 16 (the other parallel passes use 16);
 *   "par32"           1: the FP32 pass runs parallel in time the same way (same
 *                     decisions and hand-over steps as the step-by-step pass);
 *                     0 (default).  Ignored when "deesc" > 0;
 *   "drain32"         once the FP32 pass's work list is exhausted, its waves with
 *                     fewer active lanes than this hand their candidates (column,
 *                     error bounds, next step) to the parallel-in-time FP32 pass,
 *                     which carries them on with the same decisions (0..65; 0,
 *                     the default: never; 65: every wave at once);
 *   "sort_esc"        1: the FP64 hand-over pass takes its queue ordered by
 *                     hand-over step, earliest first; 0 (default): as handed over;
 *   "wave64"          FP64 passes with one candidate per wave, its joint
 *                     positions in registers and 63 steps decided per round (up to
 *                     20 joints; not with "deesc" > 0), a bit mask: 1 the hand-over
 *                     pass, 2 the path pass (rows whole), 4 the FP64 decision pass
 *                     of LINKS_FP64; 0 (default): none.  Results are the same
 *                     either way;
 *   "path_chunks"     1 (default): path rows are computed in chunks of 32 steps,
 *                     each on a lane of its own, from the sides of every placed
 *                     joint that the decision passes record at the chunk ends
 *                     (FP64 and FP32_RECHECK precision; not with "deesc" > 0,
 *                     "par64" = 2 or the path pass of "wave64"); 0: whole rows.
 *                     Rows are the same either way. */
int links_set_option(links_ctx* ctx, const char* name, int value);
/* Current value of a named option in *value (LINKS_ERR_ARG for an unknown name). */
int links_get_option(links_ctx* ctx, const char* name, int* value);

/* Current launch parameters and the persistent grid sizes of the last call (any
 * pointer may be NULL). */
int links_get_tuning(links_ctx* ctx, int* waves32, int* refill_min, int* waves64, int* grid32, int* grid64);

/* Path normalisation (Methodology, "Dataset Curation & Processing"), FP32.
 *   paths [P][T][2] in, out [P][T][2], xform [P][5] = (cx, cy, s, phi, flags) with
 *   out = R(-phi) (p - c) / s, plus (0.5, 0.5) in DIAMETER mode.
 * PCA: c = centroid, s = RMS radius, phi = principal axis angle turned so that the
 *   third moment along +x is positive.  DIAMETER: the paper's rule -- the longest
 *   chord is turned to +x and scaled to length 1, and the bounding box is centred
 *   at (0.5, 0.5).  out may alias paths. */
int links_normalize_paths(links_ctx* ctx, const float* paths, int32_t P, int32_t T, int32_t mode,
                          float* out, float* xform, void* stream);

/* Same as links_normalize_paths for the first min(*count, cap) rows, where count
 * is a DEVICE int32 (for instance n_written of a WRITE_VALID simulation), so a
 * simulate -> normalise pipeline needs no host synchronisation. */
int links_normalize_paths_n(links_ctx* ctx, const float* paths, const int32_t* count, int32_t cap, int32_t T,
                            int32_t mode, float* out, float* xform, void* stream);

/* On-device generation of B dyad-built candidates (Methodology, "1-DOF Operator"
 * and "Generating Valid Topologies"; positions as in "Finding Valid Initial
 * Positions"): joint 0 fixed pivot, joint 1 actuated tip (link 0-1), joint 2
 * fixed, and each joint k = 3..n-1 linked to two earlier joints that are not both
 * fixed (21 draws of a pair, then the arm 0-1 as a fallback); n ~ U{n_lo..n_hi};
 * every coordinate uniform in [0,1) with 24 random bits.  paper_mode is a bit
 * set: bit 0 adds, with probability 1/4, a fixed joint in place of a linked one
 * and sets the arm to pivot (0.5, 0.5), tip (0.55, 0.5); bit 1 applies the
 * paper's topology rules (the last joint depends on every other joint, so the
 * mechanism is not reducible, and is linked to no fixed joint): a draw is kept
 * only if the rules can still be met by the joints left to add, else the
 * deterministic choice that uses up the most joints not yet used by any later
 * joint is taken, and the last joint takes those left (needs n_lo >= 5).
 * Candidate i of the call is candidate
 * first + i of the seed's sequence (SplitMix64 streams, Steele, Lea and Flood
 * 2014), identical to the host generator of the Python package for the same
 * seed, so a long stream can be generated in independent chunks.
 * Outputs are device arrays in the links_batch layout (x0 as double), written
 * asynchronously on `stream`.  Errors: LINKS_ERR_ARG for B < 0, first < 0,
 * J outside [3, 32], joint counts outside [3, J], paper_mode outside 0..3, the
 * rules with n_lo < 5, or a NULL array. */
int links_generate_dyads(links_ctx* ctx, uint64_t seed, int64_t first, int32_t B, int32_t J, int32_t n_lo,
                         int32_t n_hi, int32_t paper_mode, uint8_t* n, uint32_t* adj, uint32_t* fixed,
                         uint8_t* motor, double* x0, void* stream);

/* Curation of coupler paths (Methodology, "Dataset Curation & Processing").  Row i
 * of norm_paths ([cap][T][2], DIAMETER-normalised by links_normalize_paths) is the
 * path of joint out_joint (-1: the last joint of the solve order) of candidate
 * path_index[i] of batch (path_index NULL: candidate i); only the first
 * min(*count, cap) rows are processed (count: a DEVICE int32, for instance the
 * n_written of a WRITE_VALID simulation; NULL: all cap rows).  Outputs per row:
 *   flags      uint8   LINKS_CURATE_ARC when the joint is linked to a fixed joint
 *                      (its path is an arc about that joint); LINKS_CURATE_CIRCLE
 *                      when the population variance of the distances of the
 *                      points from (0.5, 0.5) is below circle_var (the paper uses
 *                      5e-4), computed in double
 *   radial_var float   that variance
 *   keep       uint32  joints of the reduced mechanism: the path's joint, its
 *                      solve-order parents recursively, and the pivot when the
 *                      actuated tip is among them (0 for an unsolvable candidate)
 * Errors: LINKS_ERR_ARG for NULL arrays, cap < 0, T < 1, a bad out_joint, or
 * cap > B without path_index. */
#define LINKS_CURATE_ARC 1
#define LINKS_CURATE_CIRCLE 2
int links_curate(links_ctx* ctx, const links_batch* batch, const int32_t* path_index, const int32_t* count,
                 int32_t cap, int32_t out_joint, const float* norm_paths, int32_t T, double circle_var,
                 uint8_t* flags, float* radial_var, uint32_t* keep, void* stream);

/* Bidirectional chamfer distance between paths ("A Case Study of Mechanism
 * Retrieval"): for two paths A and B of T points each,
 *   CD(A, B) = mean_a min_b |a - b| + mean_b min_a |a - b|   (Euclidean norm),
 * computed in FP32 from exact coordinate differences.  A path with a NaN
 * coordinate has CD = NaN against everything.
 *   bank    [P][T][2] float  normalised paths (DIAMETER mode in the paper)
 *   queries [Q][T][2] float  normalised target paths
 *   dist    [Q][P]    float  CD of every (query, bank path) pair
 * Errors: LINKS_ERR_ARG for P < 0, Q < 0, T outside [1, 256], or a NULL array
 * when P and Q are both > 0.  Asynchronous on `stream`. */
int links_chamfer(links_ctx* ctx, const float* bank, int32_t P, int32_t T, const float* queries, int32_t Q,
                  float* dist, void* stream);

/* Path retrieval over a bank ("A Case Study of Mechanism Retrieval": a bank path
 * matches a query when its CD is below a cut-off, 0.03 in the paper).
 *   LINKS_SEARCH_FIRST  go through the bank in order (the paper shuffles the
 *                       curated set first: pass it shuffled) until k matches are
 *                       found: the k lowest bank positions with CD < cutoff;
 *                       the scan stops early once every query has k matches
 *   LINKS_SEARCH_BEST   the k smallest CDs below cutoff over the whole bank,
 *                       equal CDs in bank order (cutoff = INFINITY: plain top k)
 * Outputs (device): idx [Q][k] int64 bank positions (-1 where fewer than k
 * matches exist) and dist [Q][k] float their CD (NaN where idx is -1).  The
 * call returns when the search has finished (it synchronises `stream`: the
 * FIRST scan decides on the host when to stop).  Errors: those of
 * links_chamfer, k outside [1, 16], a NaN cutoff or a bad order. */
#define LINKS_SEARCH_FIRST 0
#define LINKS_SEARCH_BEST 1
int links_chamfer_search(links_ctx* ctx, const float* bank, int32_t P, int32_t T, const float* queries,
                         int32_t Q, int32_t k, float cutoff, int32_t order, int64_t* idx, float* dist,
                         void* stream);

/* Replayable launch sequence.  links_graph_create records the passes of one
 * links_simulate call with exactly these arguments into a HIP graph (captured on
 * a private stream; nothing runs yet) and returns it in *graph.  Every replay by
 * links_graph_launch on `stream` recomputes the outputs from whatever the batch
 * arrays hold at that time, so a caller may refill the same input buffers and
 * replay.  The graph keeps the device pointers of batch, out and of the
 * context's workspace: they must stay valid until links_graph_destroy, and a
 * links_simulate on the same context that would need a larger workspace fails
 * with LINKS_ERR_ARG while graphs exist.  Replays of graphs of one context share
 * its workspace, so they must not overlap in time (same stream, or synchronised).
 * Profiling events are not recorded in graphs.  Destroy graphs before their
 * context.  Errors: those of links_simulate, or LINKS_ERR_DEVICE from capture. */
typedef struct links_graph links_graph;
int links_graph_create(links_ctx* ctx, const links_batch* batch, const links_sim_opts* opts, links_sim_out* out,
                       links_graph** graph);
int links_graph_launch(links_graph* graph, void* stream);
void links_graph_destroy(links_graph* graph);

/* Kernel timing.  With profiling enabled every links_simulate records HIP
 * events around each of its passes on the call's stream, into the next of 64
 * event sets held by the context (a call with a low-fidelity screen records two
 * sets, the screen's first).  Recording never synchronises the host, so a caller
 * can time a run of calls and read them afterwards.  links_profile clears the
 * sets.  links_last_timings synchronises with the last completed call's final
 * event and writes the elapsed milliseconds of up to n passes, in this order:
 * set-up count (validation, solve-order length, bucket offsets), set-up fill
 * (solve order and records at the sorted position), FP32 pass, FP64 pass
 * (hand-over list, or every candidate in FP64 precision), compaction and path
 * selection, path pass.  links_mean_timings writes the mean of each pass over
 * the last `calls` completed profiled calls (1 <= calls <= the number held,
 * at most 64).  A pass that did not run counts as 0.  Both return the number of
 * values written, or LINKS_ERR_ARG when no (or too few) profiled calls are held. */
#define LINKS_TIMING_PASSES 6
int links_profile(links_ctx* ctx, int enable);
int links_last_timings(links_ctx* ctx, float* ms, int n);
int links_mean_timings(links_ctx* ctx, int calls, float* ms, int n);

#ifdef __cplusplus
}
#endif
#endif
