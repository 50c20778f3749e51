// Round-kernel instantiations for one gate.  Built once per gate with
// -DZC_INST_VANILLA, -DZC_INST_PROD=<m> or -DZC_INST_SUM=<P + 16 A>, so the
// unrolled kernels compile in parallel.
#include <hip/hip_runtime.h>

#include "zc_kernels.h"
#include "zc_launch.h"

namespace zc {
namespace {

inline int launch_ok() { return hipGetLastError() == hipSuccess ? 0 : -3; }

template <class Gate>
size_t tail_lds_bytes() {
  return (size_t)tail_lds_words<Gate>() * sizeof(uint32_t);
}

// The tail's dynamic LDS can pass 64 KiB (gfx950 has 160 KiB per CU): allow
// it for a kernel once, before its first launch with a tail.
template <class KernelTag>
void allow_tail_lds(const void* kernel, size_t bytes) {
  static const bool done = [kernel, bytes] {
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipGetLastError();
    return true;
  }();
  (void)done;
}

// Blocks of `kernel` (kBlock threads, no dynamic LDS) resident per CU; the
// answer depends only on the compiled kernel, so it is asked once.
template <class KernelTag>
int resident_blocks(const void* kernel) {
  static const int n = [kernel] {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, kBlock, 0) != hipSuccess || b < 1) b = 1;
    return b;
  }();
  return n;
}

template <class Gate, bool FOLD, bool SPLIT, int X0 = 0, bool HALF = false>
struct RoundTag {};

template <class Gate>
constexpr uint64_t half_q() {
  return Gate::kFoldInGate ? kHalfQ : kHalfQVanilla;
}
template <class Gate>
struct FinishTag {};
template <class Gate>
struct FinishSpecTag {};
template <class Gate>
struct BatchFinishTag {};
template <class Gate>
struct ServeFinishTag {};

// Grid of a round kernel: enough blocks for the work, at most one resident
// generation (CUs x resident blocks per CU) and at most kMaxBlocks.  With
// `share` (ZC_FLAG_SHARED_GPU) a round may use more generations, down to
// kSharePairs pairs per thread, still at most kMaxBlocks: shorter-lived
// blocks, so that compute units come free during the round for the kernels
// of other streams (the sums are exact, so the bytes do not change).  Each
// generation costs a block start and a block reduction; kSharePairs keeps
// that overhead to a few percent of the round.
constexpr uint64_t kSharePairs = 2;
inline uint32_t round_grid(uint64_t blocks_for_work, int per_cu, int* rc, bool share = false) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
    *rc = -3;
    return 0;
  }
  uint64_t cap = (uint64_t)cus * (uint64_t)per_cu;
  if (share && (blocks_for_work + kSharePairs - 1) / kSharePairs > cap)
    cap = (blocks_for_work + kSharePairs - 1) / kSharePairs;
  if (cap > (uint64_t)kMaxBlocks) cap = kMaxBlocks;
  if (blocks_for_work < 1) blocks_for_work = 1;
  return (uint32_t)(blocks_for_work < cap ? blocks_for_work : cap);
}

// Launches round a.round: the round kernel (partial sums per block), then
// k_finish (one block: sums, G_i, alpha_i, and with kSplitTail the rest of
// the proof).
template <class Gate>
int launch_round(bool fold, RoundKind kind, RoundArgs a, const TabPtrs& src, const TabPtrs& dst, hipStream_t st,
                 hipEvent_t after) {
  int rc = 0;
  uint32_t blocks;
  // round 1 under ZC_FLAG_ASSUME_SATISFIED: the kernels that skip X = 0, 1
  const bool skip = !fold && a.skip01 != 0;
  if (kind == kPerPair && fold && a.q <= half_q<Gate>() && src.p[0] != dst.p[0]) {
    // two waves per 64 pairs (round_body HALF), never in place: both waves
    // read every pair that one of them then overwrites
    const void* kern = reinterpret_cast<const void*>(&k_round<Gate, true, 0, true>);
    const int per_cu = resident_blocks<RoundTag<Gate, true, false, 0, true>>(kern);
    blocks = round_grid((2 * a.q + kBlock - 1) / kBlock, per_cu, &rc, a.share != 0);
    if (rc) return rc;
    hipLaunchKernelGGL((k_round<Gate, true, 0, true>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
  } else if (kind == kPerPair) {
    const void* kern = fold ? reinterpret_cast<const void*>(&k_round<Gate, true>)
                       : skip ? reinterpret_cast<const void*>(&k_round<Gate, false, 2>)
                              : reinterpret_cast<const void*>(&k_round<Gate, false>);
    const int per_cu = fold ? resident_blocks<RoundTag<Gate, true, false>>(kern)
                       : skip ? resident_blocks<RoundTag<Gate, false, false, 2>>(kern)
                              : resident_blocks<RoundTag<Gate, false, false>>(kern);
    blocks = round_grid((a.q + kBlock - 1) / kBlock, per_cu, &rc, a.share != 0);
    if (rc) return rc;
    if (fold)
      hipLaunchKernelGGL((k_round<Gate, true>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
    else if (skip)
      hipLaunchKernelGGL((k_round<Gate, false, 2>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
    else
      hipLaunchKernelGGL((k_round<Gate, false>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
  } else {
    const void* kern = fold ? reinterpret_cast<const void*>(&k_round_split<Gate, true>)
                       : skip ? reinterpret_cast<const void*>(&k_round_split<Gate, false, 2>)
                              : reinterpret_cast<const void*>(&k_round_split<Gate, false>);
    const int per_cu = fold ? resident_blocks<RoundTag<Gate, true, true>>(kern)
                       : skip ? resident_blocks<RoundTag<Gate, false, true, 2>>(kern)
                              : resident_blocks<RoundTag<Gate, false, true>>(kern);
    blocks = round_grid((a.q + kSplitPairs - 1) / kSplitPairs, per_cu, &rc);
    if (rc) return rc;
    if (fold)
      hipLaunchKernelGGL((k_round_split<Gate, true>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
    else if (skip)
      hipLaunchKernelGGL((k_round_split<Gate, false, 2>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
    else
      hipLaunchKernelGGL((k_round_split<Gate, false>), dim3(blocks), dim3(kBlock), 0, st, a, src, dst);
  }
  if ((rc = launch_ok()) != 0) return rc;
  if (after && hipEventRecord(after, st) != hipSuccess) return -3;
  a.nparts = blocks;
  a.tail = (kind == kSplitTail) ? 1u : 0u;
  const size_t lds = a.tail ? tail_lds_bytes<Gate>() : 0;
  if (lds) allow_tail_lds<FinishTag<Gate>>(reinterpret_cast<const void*>(&k_finish<Gate>), lds);
  hipLaunchKernelGGL((k_finish<Gate>), dim3(1), dim3(kBlock), lds, st, a, dst);
  return launch_ok();
}

template <class Gate, bool FIRST>
struct SpecTag {};

template <class Gate>
struct WaitTag {};

// The launches of a fused schedule (see zc_launch.h): speculative for gates
// whose (d+1)^2 evaluations per pair fit a 16-lane group (k_fin_spec,
// k_finish_spec), waiting for the challenge otherwise (k_fin_wait, then a
// plain k_finish with the tail).
template <class Gate>
int launch_spec(ZC_SPEC_ARGS) {
  int rc = 0;
  if (step == kSpecRoundOnly) {
    if (sa.q <= half_q<Gate>() && src.p[0] != dst.p[0]) {
      // two waves per 64 pairs (round_body HALF), never in place (see
      // launch_round); the proof moves its folded tables for it
      const void* kern = reinterpret_cast<const void*>(&k_round<Gate, true, 0, true>);
      const int per_cu = resident_blocks<RoundTag<Gate, true, false, 0, true>>(kern);
      const uint32_t b = round_grid((2 * sa.q + kBlock - 1) / kBlock, per_cu, &rc, sa.share != 0);
      if (rc) return rc;
      hipLaunchKernelGGL((k_round<Gate, true, 0, true>), dim3(b), dim3(kBlock), 0, st, sa, src, dst);
      *blocks = b;
      return launch_ok();
    }
    const void* kern = reinterpret_cast<const void*>(&k_round<Gate, true>);
    const int per_cu = resident_blocks<RoundTag<Gate, true, false>>(kern);
    const uint32_t b = round_grid((sa.q + kBlock - 1) / kBlock, per_cu, &rc, sa.share != 0);
    if (rc) return rc;
    hipLaunchKernelGGL((k_round<Gate, true>), dim3(b), dim3(kBlock), 0, st, sa, src, dst);
    *blocks = b;
    return launch_ok();
  }
  if constexpr (!SpecShape<Gate>::kOk) {
    if (step == kSpecFinishTail) {
      if (!fa.tail) return -1;
      allow_tail_lds<FinishTag<Gate>>(reinterpret_cast<const void*>(&k_finish<Gate>), tail_lds_bytes<Gate>());
      hipLaunchKernelGGL((k_finish<Gate>), dim3(1), dim3(kBlock), tail_lds_bytes<Gate>(), st, fa, fdst);
    } else {
      const void* kern = reinterpret_cast<const void*>(&k_fin_wait<Gate>);
      const int per_cu = resident_blocks<WaitTag<Gate>>(kern);
      // one resident generation including the finisher block
      uint32_t b = round_grid((sa.q + kSplitPairs - 1) / kSplitPairs + 1, per_cu, &rc) - 1;
      if (rc) return rc;
      if (b < 1) b = 1;
      if (b > kSpecBlocks) b = kSpecBlocks;
      // the finisher has no tail here and the round folds in place
      if (fa.tail || src.p[0] != dst.p[0]) return -1;
      RoundArgs f = fa;
      f.signal = 1;
      hipLaunchKernelGGL((k_fin_wait<Gate>), dim3(b + 1), dim3(kBlock), 0, st, f, sa, src);
      *blocks = b;
    }
    return launch_ok();
  } else {
    if (step == kSpecFinishTail) {
      allow_tail_lds<FinishSpecTag<Gate>>(reinterpret_cast<const void*>(&k_finish_spec<Gate>), tail_lds_bytes<Gate>());
      hipLaunchKernelGGL((k_finish_spec<Gate>), dim3(1), dim3(kBlock), tail_lds_bytes<Gate>(), st, fa, fdst);
    } else {
      const bool first = step == kSpecFirst;
      const void* kern = first ? reinterpret_cast<const void*>(&k_fin_spec<Gate, true>)
                               : reinterpret_cast<const void*>(&k_fin_spec<Gate, false>);
      const int per_cu = first ? resident_blocks<SpecTag<Gate, true>>(kern) : resident_blocks<SpecTag<Gate, false>>(kern);
      // one resident generation including the finisher block
      uint32_t b = round_grid((sa.q + kSplitPairs - 1) / kSplitPairs + 1, per_cu, &rc) - 1;
      if (rc) return rc;
      if (b < 1) b = 1;
      if (b > kSpecBlocks) b = kSpecBlocks;
      // the finisher has no tail here and the speculative round folds in place
      if (fa.tail || src.p[0] != dst.p[0]) return -1;
      if (first)
        hipLaunchKernelGGL((k_fin_spec<Gate, true>), dim3(b + 1), dim3(kBlock), 0, st, fa, sa, src);
      else
        hipLaunchKernelGGL((k_fin_spec<Gate, false>), dim3(b + 1), dim3(kBlock), 0, st, fa, sa, src);
      *blocks = b;
    }
    return launch_ok();
  }
}

template <class Gate>
int launch_batch(const BatchStep& bs, uint32_t blocks, bool fold, bool tail, hipStream_t st) {
  if (bs.count == 0) return 0;
  if (fold)
    hipLaunchKernelGGL((k_batch_round<Gate, true>), dim3(blocks), dim3(kBlock), 0, st, bs);
  else
    hipLaunchKernelGGL((k_batch_round<Gate, false>), dim3(blocks), dim3(kBlock), 0, st, bs);
  int rc = launch_ok();
  if (rc != 0) return rc;
  if (tail) allow_tail_lds<BatchFinishTag<Gate>>(reinterpret_cast<const void*>(&k_batch_finish<Gate>), tail_lds_bytes<Gate>());
  hipLaunchKernelGGL((k_batch_finish<Gate>), dim3(bs.count), dim3(kBlock), tail ? tail_lds_bytes<Gate>() : 0, st, bs);
  return launch_ok();
}

template <class Gate>
int launch_serve(const ServeStep& ss, uint32_t blocks, bool fold, bool tail, hipStream_t st) {
  if (ss.count == 0) return 0;
  if (fold)
    hipLaunchKernelGGL((k_serve_round<Gate, true>), dim3(blocks), dim3(kBlock), 0, st, ss);
  else
    hipLaunchKernelGGL((k_serve_round<Gate, false>), dim3(blocks), dim3(kBlock), 0, st, ss);
  int rc = launch_ok();
  if (rc != 0) return rc;
  if (ss.nfin == 0) return 0;
  if (tail) allow_tail_lds<ServeFinishTag<Gate>>(reinterpret_cast<const void*>(&k_serve_finish<Gate>), tail_lds_bytes<Gate>());
  hipLaunchKernelGGL((k_serve_finish<Gate>), dim3(ss.nfin), dim3(kBlock), tail ? tail_lds_bytes<Gate>() : 0, st, ss);
  return launch_ok();
}

}  // namespace

#if defined(ZC_INST_VANILLA)
int launch_round_vanilla(bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src, const TabPtrs& dst,
                         hipStream_t st, hipEvent_t after) {
  return launch_round<GateVanilla>(fold, kind, a, src, dst, st, after);
}
int launch_batch_vanilla(const BatchStep& bs, uint32_t blocks, bool fold, bool tail, hipStream_t st) {
  return launch_batch<GateVanilla>(bs, blocks, fold, tail, st);
}
int launch_serve_vanilla(const ServeStep& ss, uint32_t blocks, bool fold, bool tail, hipStream_t st) {
  return launch_serve<GateVanilla>(ss, blocks, fold, tail, st);
}
int launch_spec_vanilla(ZC_SPEC_ARGS) { return launch_spec<GateVanilla>(step, fa, fdst, sa, src, dst, st, blocks); }
#elif defined(ZC_INST_PROD)
#define ZC_CAT2(a, b) a##b
#define ZC_CAT(a, b) ZC_CAT2(a, b)
int ZC_CAT(launch_round_prod, ZC_INST_PROD)(bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src,
                                            const TabPtrs& dst, hipStream_t st, hipEvent_t after) {
  return launch_round<GateProd<ZC_INST_PROD>>(fold, kind, a, src, dst, st, after);
}
int ZC_CAT(launch_batch_prod, ZC_INST_PROD)(const BatchStep& bs, uint32_t blocks, bool fold, bool tail,
                                            hipStream_t st) {
  return launch_batch<GateProd<ZC_INST_PROD>>(bs, blocks, fold, tail, st);
}
int ZC_CAT(launch_serve_prod, ZC_INST_PROD)(const ServeStep& ss, uint32_t blocks, bool fold, bool tail,
                                            hipStream_t st) {
  return launch_serve<GateProd<ZC_INST_PROD>>(ss, blocks, fold, tail, st);
}
int ZC_CAT(launch_spec_prod, ZC_INST_PROD)(ZC_SPEC_ARGS) {
  return launch_spec<GateProd<ZC_INST_PROD>>(step, fa, fdst, sa, src, dst, st, blocks);
}
#elif defined(ZC_INST_SUM)
// m = P + 16 A of a Table 1 shape
using GateT1 = GateSum<(ZC_INST_SUM & 15), (ZC_INST_SUM >> 4)>;
#define ZC_CAT2(a, b) a##b
#define ZC_CAT(a, b) ZC_CAT2(a, b)
int ZC_CAT(launch_round_sum, ZC_INST_SUM)(bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src,
                                          const TabPtrs& dst, hipStream_t st, hipEvent_t after) {
  return launch_round<GateT1>(fold, kind, a, src, dst, st, after);
}
int ZC_CAT(launch_batch_sum, ZC_INST_SUM)(const BatchStep& bs, uint32_t blocks, bool fold, bool tail,
                                          hipStream_t st) {
  return launch_batch<GateT1>(bs, blocks, fold, tail, st);
}
int ZC_CAT(launch_serve_sum, ZC_INST_SUM)(const ServeStep& ss, uint32_t blocks, bool fold, bool tail,
                                          hipStream_t st) {
  return launch_serve<GateT1>(ss, blocks, fold, tail, st);
}
int ZC_CAT(launch_spec_sum, ZC_INST_SUM)(ZC_SPEC_ARGS) {
  return launch_spec<GateT1>(step, fa, fdst, sa, src, dst, st, blocks);
}
#else
#error "build zc_inst.hip with -DZC_INST_VANILLA, -DZC_INST_PROD=<m> or -DZC_INST_SUM=<P + 16 A>"
#endif

}  // namespace zc
