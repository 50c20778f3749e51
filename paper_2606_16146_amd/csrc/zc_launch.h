// Round-kernel launch helpers shared by the host API and the per-gate
// instantiation units (zc_inst.hip is compiled once per gate so that the
// large unrolled kernels build in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "zc_device.h"

namespace zc {

struct RoundArgs;
struct BatchStep;
struct ServeStep;

constexpr int kTailQ = 32;  // the tail runs rounds with at most this many pairs

// Rounds with at most this many pairs use sixteen lanes per pair: one thread
// per pair is the faster of the two down to 16384 pairs (measured at mu = 20
// for degree 9; for degree 3, whose lane-split rounds are speculative, 16384
// and 8192 measured the same and 4096 slower).
inline uint64_t split_q(uint32_t) { return 16384u; }

// Folding thread-per-pair rounds run two waves per 64 pairs when they have at
// most this many pairs: 32768 pairs are 512 waves, one for half the SIMDs of
// 256 CUs.  kHalfQ for the gates that fold inside their evaluation (whose two
// waves both fold every table), kHalfQVanilla for the vanilla gate (whose
// waves split its terms and tables).
constexpr uint64_t kHalfQ = 32768;
constexpr uint64_t kHalfQVanilla = 32768;

enum RoundKind { kPerPair = 0, kSplit = 1, kSplitTail = 2, kInTail = 3, kSpec = 4, kSpecTail = 5 };

// Fused lane-split rounds: round i is evaluated in the same launch as the
// finisher of round i-1.  Gates of degree <= 3 (whose (d+1)^2 evaluations per
// pair fit the 16 lanes of a pair) evaluate it for every candidate
// alpha_{i-1} in 0..d, and its own finisher interpolates (speculation); the
// other gates' blocks wait for alpha_{i-1}, which the finisher block posts
// when it has it, with their first loads already issued.  s0 is the first
// lane-split round, r the round whose finisher starts the tail; rounds
// s0..r-1 are kSpec, r is kSpecTail.  Used when s0 >= 3 and r > s0.
struct SpecPlan {
  uint32_t s0, r;
  bool on;
};
inline SpecPlan spec_plan(uint32_t mu, uint32_t degree) {
  SpecPlan p{0, 0, false};
  for (uint32_t i = 1; i <= mu; ++i) {
    const uint64_t q = 1ull << (mu - i);
    if (!p.s0 && q <= split_q(degree)) p.s0 = i;
    if (!p.r && q <= 2 * (uint64_t)kTailQ) p.r = i;
  }
  p.on = p.s0 >= 3 && p.r > p.s0;
  return p;
}

// Which kernel evaluates round i of a whole proof (zc_prove).
inline RoundKind prove_round_kind(uint32_t mu, uint32_t i, uint32_t degree) {
  const uint64_t q = 1ull << (mu - i);
  const uint64_t first_tail_q = 2 * (uint64_t)kTailQ;
  if (q > split_q(degree)) return kPerPair;
  const SpecPlan sp = spec_plan(mu, degree);
  if (sp.on && i >= sp.s0 && i <= sp.r) return i < sp.r ? kSpec : kSpecTail;
  if (q > first_tail_q) return kSplit;
  // the first round with q <= 2 kTailQ launches the tail; later rounds run inside it
  const uint64_t prev_q = q * 2;
  return (i == 1 || prev_q > first_tail_q) ? kSplitTail : kInTail;
}

// The launches of a fused schedule: the last thread-per-pair round without
// its finisher; the finisher of round r-1 beside round r (first or later);
// the finisher of the last fused round, which runs the tail.  *blocks
// receives the number of partial-sum blocks written.
enum SpecStep { kSpecRoundOnly = 0, kSpecFirst = 1, kSpecNext = 2, kSpecFinishTail = 3 };
constexpr uint32_t kSpecBlocks = 1024;  // partial-sum blocks of a speculative round, at most

// One launcher per gate instantiation (defined in zc_inst.hip).  `after`, if
// not null, is recorded on the stream between the round kernel and its
// finisher (profiling).
int launch_round_vanilla(bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src, const TabPtrs& dst,
                         hipStream_t st, hipEvent_t after);
#define ZC_DECL_PROD(M)                                                                                      \
  int launch_round_prod##M(bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src, const TabPtrs& dst, \
                           hipStream_t st, hipEvent_t after);
ZC_DECL_PROD(1)
ZC_DECL_PROD(2)
ZC_DECL_PROD(3)
ZC_DECL_PROD(4)
ZC_DECL_PROD(5)
ZC_DECL_PROD(6)
ZC_DECL_PROD(7)
ZC_DECL_PROD(8)
#undef ZC_DECL_PROD

// One gate's share of one batch step: the round kernel over `blocks` blocks,
// then one finisher block per instance (with tail LDS when `tail` is set).
int launch_batch_vanilla(const BatchStep& bs, uint32_t blocks, bool fold, bool tail, hipStream_t st);
#define ZC_DECL_BPROD(M) \
  int launch_batch_prod##M(const BatchStep& bs, uint32_t blocks, bool fold, bool tail, hipStream_t st);
ZC_DECL_BPROD(1)
ZC_DECL_BPROD(2)
ZC_DECL_BPROD(3)
ZC_DECL_BPROD(4)
ZC_DECL_BPROD(5)
ZC_DECL_BPROD(6)
ZC_DECL_BPROD(7)
ZC_DECL_BPROD(8)
#undef ZC_DECL_BPROD

// The same for a serving step (instances at their own rounds).
int launch_serve_vanilla(const ServeStep& ss, uint32_t blocks, bool fold, bool tail, hipStream_t st);
#define ZC_DECL_SPROD(M) \
  int launch_serve_prod##M(const ServeStep& ss, uint32_t blocks, bool fold, bool tail, hipStream_t st);
ZC_DECL_SPROD(1)
ZC_DECL_SPROD(2)
ZC_DECL_SPROD(3)
ZC_DECL_SPROD(4)
ZC_DECL_SPROD(5)
ZC_DECL_SPROD(6)
ZC_DECL_SPROD(7)
ZC_DECL_SPROD(8)
#undef ZC_DECL_SPROD

#define ZC_SPEC_ARGS                                                                                  \
  SpecStep step, const RoundArgs &fa, const TabPtrs &fdst, const RoundArgs &sa, const TabPtrs &src, \
      const TabPtrs &dst, hipStream_t st, uint32_t *blocks
int launch_spec_vanilla(ZC_SPEC_ARGS);
int launch_spec_prod1(ZC_SPEC_ARGS);
int launch_spec_prod2(ZC_SPEC_ARGS);
int launch_spec_prod3(ZC_SPEC_ARGS);
int launch_spec_prod4(ZC_SPEC_ARGS);
int launch_spec_prod5(ZC_SPEC_ARGS);
int launch_spec_prod6(ZC_SPEC_ARGS);
int launch_spec_prod7(ZC_SPEC_ARGS);
int launch_spec_prod8(ZC_SPEC_ARGS);

// Table 1 shapes, one set per m = P + 16 A.
#define ZC_DECL_SUM(C)                                                                                            \
  int launch_round_sum##C(bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src, const TabPtrs& dst, \
                          hipStream_t st, hipEvent_t after);                                                     \
  int launch_batch_sum##C(const BatchStep& bs, uint32_t blocks, bool fold, bool tail, hipStream_t st);          \
  int launch_serve_sum##C(const ServeStep& ss, uint32_t blocks, bool fold, bool tail, hipStream_t st);          \
  int launch_spec_sum##C(ZC_SPEC_ARGS);
ZC_DECL_SUM(2)
ZC_DECL_SUM(18)
ZC_DECL_SUM(34)
ZC_DECL_SUM(50)
ZC_DECL_SUM(3)
ZC_DECL_SUM(4)
#undef ZC_DECL_SUM

}  // namespace zc
