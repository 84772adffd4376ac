// gen.hip -- on-device generation of dyad-built candidates, draw for draw the
// same as the host generator (paper_2208_14567_amd/gen.py), so large streams of
// candidates never cross PCIe.
//
// Topologies follow the paper's dyadic J operator (Methodology, "1-DOF Operator"
// and "Generating Valid Topologies"): ground joint 0, actuated tip 1 (link 0-1)
// and a floating ground joint 2, then each further joint is linked to two
// existing joints that are not both fixed; in paper mode a linkless ground joint
// is added instead with probability 1/4 and the actuator arm is standardised
// ("Finding Valid Initial Positions").  Positions are uniform in [0,1)^2 with 24
// random bits per coordinate.
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).  Candidate c
// owns the stream whose state is output c of SplitMix64(seed); draw k of that
// candidate is output k of SplitMix64(state).  Draw numbering: 0 joint count,
// 1 + 2j and 2 + 2j the coordinates of joint j, 65 + 64 (k - 3) + 3 a + r the
// topology draws of joint k at attempt a (r = 0 operator choice, 1 first
// partner, 2 second partner).
//
// With the topology rules (Methodology, "Generating Valid Topologies": the last
// joint depends on every other joint, and is linked to no fixed joint) a draw is
// kept only if the rules can still be met by the joints left to add; otherwise
// the deterministic choice that uses up the most pending joints is taken, and the
// last joint takes the pending ones (with a partner among the other non-fixed
// joints when one is left).
#include "common.h"
#include "kernels.h"

namespace links {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kTopoAttempts = 21;
constexpr int kGenBlock = 64;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// the 24-bit integer m of draw k; the uniform value is m * 2^-24
__device__ __forceinline__ uint32_t draw24(uint64_t state, uint32_t k) {
  return (uint32_t)(mix64(state + (uint64_t)(k + 1) * kGamma) >> 40);
}

// Pending joints U: placed or fixed joints no later joint uses yet.  With r joints
// left to add after the current one, each of them but the last can use up two
// pending joints (at most one fixed) and adds itself, and the last must use up
// what remains (at most two, none fixed): the rules can still be met iff
// |U| <= r + 1 and at most r - 1 pending joints are fixed.
__device__ __forceinline__ bool rules_feasible(uint32_t U, uint32_t fixed, int r) {
  return __popc(U) <= r + 1 && __popc(U & fixed) <= r - 1;
}

// index of the lowest set bit (32 when none)
__device__ __forceinline__ int lowest(uint32_t m) { return m ? __ffs(m) - 1 : 32; }

__global__ void __launch_bounds__(kGenBlock) gen_dyads_kernel(GenArgs g) {
  __shared__ uint32_t adj_l[kMaxJ * kGenBlock];
  const int tid = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * kGenBlock + tid;
  if (c >= g.B) return;
  const int J = g.J;
  const uint64_t cand = (uint64_t)(g.first + c);
  const uint64_t st = mix64(g.seed + (cand + 1) * kGamma);
  // n = lo + floor(u * (hi - lo + 1)), exact in integers for a 24-bit u
  const int n = g.n_lo + (int)(((uint64_t)draw24(st, 0) * (uint64_t)(g.n_hi - g.n_lo + 1)) >> 24);
  uint32_t* A = adj_l + tid;
  for (int i = 0; i < J; i++) A[i * kGenBlock] = 0u;
  uint32_t fixed = 0b101u;
  uint32_t U = 0b110u;  // pending joints (rules): the tip and fixed joint 2
  A[0] |= 1u << 1;
  A[1 * kGenBlock] |= 1u << 0;
  for (int k = 3; k < n; k++) {
    const uint32_t base = 65u + 64u * (uint32_t)(k - 3);
    const uint32_t bit = 1u << k;
    const int r = n - 1 - k;  // joints still to add after this one
    const bool last = r == 0;
    if (g.paper_mode && draw24(st, base) < (1u << 22)) {  // u < 1/4: a new ground joint
      if (!g.rules || (!last && rules_feasible(U | bit, fixed | bit, r))) {
        fixed |= bit;
        if (g.rules) U |= bit;
        continue;
      }
    }
    int pi = 0, pj = 1;  // the actuator arm when no attempt succeeds (no rules)
    bool done = false;
    for (int a = 0; a < kTopoAttempts && !(g.rules && last); a++) {
      const uint32_t mi = draw24(st, base + 3u * a + 1u);
      const uint32_t mj = draw24(st, base + 3u * a + 2u);
      const int i = (int)(((uint64_t)mi * (uint64_t)k) >> 24);
      int j = (int)(((uint64_t)mj * (uint64_t)(k - 1)) >> 24);
      if (j >= i) j++;
      if (((fixed >> i) & 1u) && ((fixed >> j) & 1u)) continue;
      if (g.rules && !rules_feasible((U & ~((1u << i) | (1u << j))) | bit, fixed, r)) continue;
      pi = i;
      pj = j;
      done = true;
      break;
    }
    if (g.rules) {
      const uint32_t nonfixed = (bit - 1u) & ~fixed;
      const uint32_t uf = U & fixed, un = U & ~fixed;
      if (!done && !last) {
        // the choice that uses up the most pending joints, a pending fixed one
        // first, then pending non-fixed ones, then the lowest non-fixed joint
        pi = uf ? lowest(uf) : un ? lowest(un) : lowest(nonfixed);
        const uint32_t m1 = 1u << pi;
        pj = (un & ~m1) ? lowest(un & ~m1) : lowest(nonfixed & ~m1);
      } else if (last) {
        // the pending joints; with one left, the q-th of the other non-fixed
        // joints in index order, q from the first attempt's first-partner draw
        pi = lowest(un);
        const uint32_t ml = 1u << pi;
        if (un & ~ml) {
          pj = lowest(un & ~ml);
        } else {
          const uint32_t others = nonfixed & ~ml;
          const uint32_t cnt = (uint32_t)__popc(others);
          const uint32_t q = (uint32_t)(((uint64_t)draw24(st, base + 1u) * (uint64_t)(cnt ? cnt : 1u)) >> 24);
          uint32_t o = others;
          for (uint32_t s = 0; s < q; s++) o &= o - 1u;  // drop the q lowest bits
          pj = lowest(o);
        }
      }
      if (pi > 31 || pj > 31) {  // cannot happen from a state that meets the rules
        pi = 0;
        pj = 1;
      }
      U = (U & ~((1u << pi) | (1u << pj))) | bit;
    }
    A[k * kGenBlock] |= (1u << pi) | (1u << pj);
    A[pi * kGenBlock] |= 1u << k;
    A[pj * kGenBlock] |= 1u << k;
  }
  g.n[c] = (uint8_t)n;
  g.fixed[c] = fixed;
  g.motor[2 * c] = 0;
  g.motor[2 * c + 1] = 1;
  uint32_t* adj_out = g.adj + c * J;
  for (int i = 0; i < J; i++) adj_out[i] = A[i * kGenBlock];
  double2* x = reinterpret_cast<double2*>(g.x0 + c * J * 2);
  const double inv24 = 1.0 / 16777216.0;
  for (int j = 0; j < J; j++) {
    double2 v = make_double2(0.0, 0.0);
    if (j < n) {
      v.x = (double)draw24(st, 1u + 2u * j) * inv24;
      v.y = (double)draw24(st, 2u + 2u * j) * inv24;
    }
    if (g.paper_mode && j == 0) v = make_double2(0.5, 0.5);
    if (g.paper_mode && j == 1) v = make_double2(0.55, 0.5);
    x[j] = v;
  }
}

}  // namespace

hipError_t launch_gen_dyads(const GenArgs& g, hipStream_t st) {
  if (g.B <= 0) return hipSuccess;
  const int64_t blocks = (g.B + kGenBlock - 1) / kGenBlock;
  hipLaunchKernelGGL(gen_dyads_kernel, dim3((unsigned)blocks), dim3(kGenBlock), 0, st, g);
  return hipGetLastError();
}

}  // namespace links
