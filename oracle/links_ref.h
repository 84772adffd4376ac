/* links_ref.h -- FP64 CPU oracle for batched 1-DOF planar linkage simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * HIP path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 *
 * All pointers are host pointers owned by the caller.  Layouts match the product
 * library's inputs (row bitmask adjacency, fixed-joint mask, motor pair, x0).
 * Return value: 0 on success, -1 on a bad argument (null pointer, J outside
 * [1,32], T < 1, B < 0).  Per-candidate problems go to `status`.
 */
#ifndef LINKS_REF_H
#define LINKS_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-candidate status codes */
#define LREF_VALID 0
#define LREF_LOCKED 1
#define LREF_DEGENERATE 2
#define LREF_DRIFT 3
#define LREF_UNSOLVABLE 4
#define LREF_BAD_MECH 5

/* normalisation modes and flags */
#define LREF_NORM_PCA 0
#define LREF_NORM_DIAMETER 1
#define LREF_NF_CONSTANT 1
#define LREF_NF_ISOTROPIC 2
#define LREF_NF_SIGN_TIE 4
#define LREF_NF_DIAM_TIE 8

/* Graphical solve order (Methodology, "Graphical Simulator"): rounds of joints
 * with two known neighbours.  order: [B][J][3] int8 (joint, parent a, parent b),
 * -1 padded; n_dyads, depth, status: [B]. */
int links_ref_solve_order(int32_t B, int32_t J, const uint8_t* n, const uint32_t* adj,
                          const uint32_t* fixed, const uint8_t* motor, int8_t* order,
                          uint8_t* n_dyads, uint8_t* depth, uint8_t* status);

/* Full-rotation simulation in FP64.
 * x0: [B][J][2].  T steps, crank angle 2*pi*t/T.  out_joint -1 = last solved joint.
 * tau_drift: a redundant link whose length moves by more than tau_drift*scale
 *   (scale = longest link) fails the candidate.
 * status [B], fail_step [B] (-1 when valid or never simulated).
 * path (nullable): [B][T][2] output joint positions, NaN from fail_step on.
 * pos_all (nullable): [B][T][J][2] every joint, NaN from fail_step on.
 * margins (nullable): [B][4] = min |disc|/scale^2 with disc = K/(4 scale^2) and
 *   K = ((ra+rb)^2 - d^2)(d^2 - (ra-rb)^2) the intersection discriminant, min d^2/scale^2,
 *   min branch distance/scale, min |drift - tau*scale|/scale over evaluated steps
 *   (+inf where nothing was evaluated).
 * nthreads: host threads over candidates (<=0: 1). */
int links_ref_simulate(int32_t B, int32_t J, const uint8_t* n, const uint32_t* adj,
                       const uint32_t* fixed, const uint8_t* motor, const double* x0,
                       int32_t T, int32_t out_joint, double tau_drift, uint8_t* status,
                       int16_t* fail_step, double* path,
                       double* pos_all, double* margins, int32_t nthreads);

/* The same with the branch rule chosen: LREF_BRANCH_CONTINUITY (the intersection
 * nearer the previous position, as links_ref_simulate) or LREF_BRANCH_ORIENTATION
 * (every placed joint stays on the side of its parents' line a->b where it is in
 * x0; margins[2] is then +inf).  Returns -1 for any other value. */
#define LREF_BRANCH_CONTINUITY 0
#define LREF_BRANCH_ORIENTATION 1
int links_ref_simulate_branch(int32_t B, int32_t J, const uint8_t* n, const uint32_t* adj,
                              const uint32_t* fixed, const uint8_t* motor, const double* x0,
                              int32_t T, int32_t out_joint, double tau_drift, uint8_t* status,
                              int16_t* fail_step, double* path,
                              double* pos_all, double* margins, int32_t nthreads, int32_t branch);

/* Path normalisation in FP64.  paths, out: [P][T][2]; xform: [P][5] =
 * (cx, cy, s, phi, flags) such that out = R(-phi)(p - c)/s, plus (0.5, 0.5) in
 * DIAMETER mode. */
int links_ref_normalize_paths(const double* paths, int32_t P, int32_t T, int32_t mode,
                              double* out, double* xform);

/* Curation of coupler paths (Methodology, "Dataset Curation & Processing").
 * Path i belongs to candidate cand[i] (cand NULL: candidate i); its joint is
 * out_joint, or the last joint of the solve order when out_joint < 0.
 *   flags[i]: bit 1 (ARC) when the joint is linked to a fixed joint (it turns
 *     about that joint); bit 2 (CIRCLE) when the population variance of the
 *     distances of the DIAMETER-normalised path norm[i] ([T][2]) from (0.5, 0.5)
 *     is below circle_var.
 *   radial_var[i]: that variance.
 *   keep[i]: the joints needed to move the path joint: the joint, its solve-order
 *     parents recursively, and the pivot when the tip is among them (the
 *     reduced mechanism).
 * Returns -1 on bad arguments (an unsolvable candidate gets keep = 0, flags 0). */
#define LREF_CUR_ARC 1
#define LREF_CUR_CIRCLE 2
int links_ref_curate(int32_t J, const uint8_t* n, const uint32_t* adj, const uint32_t* fixed,
                     const uint8_t* motor, int32_t out_joint, const int32_t* cand, int32_t P,
                     const double* norm, int32_t T, double circle_var, uint8_t* flags, double* radial_var,
                     uint32_t* keep);

#ifdef __cplusplus
}
#endif
#endif
