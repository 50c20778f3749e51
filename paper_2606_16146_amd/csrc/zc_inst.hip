// Round-kernel instantiations for one gate.  Built once per gate with
// -DZC_INST_VANILLA or -DZC_INST_PROD=<m>, so the unrolled kernels compile in
// parallel.
#include <hip/hip_runtime.h>

#include "zc_kernels.h"
#include "zc_launch.h"

namespace zc {
namespace {

inline uint32_t grid_for(uint64_t work, uint32_t cap) {
  uint64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (uint32_t)(b < cap ? b : cap);
}

inline int launch_ok() { return hipGetLastError() == hipSuccess ? 0 : -3; }

template <class Gate>
size_t tail_lds_bytes() {
  return (size_t)(Gate::K + 1) * 4 * kTailQ * NL * sizeof(uint32_t);
}

// Launches the round kernel of round a.round.  The grid has one extra block
// when a.with_t0 is set (it hashes T_0 while the others evaluate).
template <class Gate>
int launch_round(bool fold, RoundKind kind, RoundArgs a, hipStream_t st) {
  const uint32_t t0 = a.with_t0 ? 1u : 0u;
  if (kind == kPerPair) {
    const uint32_t blocks = grid_for(a.q, kMaxBlocks - 1) + t0;
    if (fold)
      hipLaunchKernelGGL((k_round<Gate, true>), dim3(blocks), dim3(kBlock), 0, st, a);
    else
      hipLaunchKernelGGL((k_round<Gate, false>), dim3(blocks), dim3(kBlock), 0, st, a);
  } else {
    const uint64_t nb = (a.q + kSplitPairs - 1) / kSplitPairs;
    const uint32_t blocks = (uint32_t)(nb < (uint64_t)(kMaxBlocks - 1) ? nb : (uint64_t)(kMaxBlocks - 1)) + t0;
    a.tail = (kind == kSplitTail) ? 1u : 0u;
    const size_t lds = a.tail ? tail_lds_bytes<Gate>() : 0;
    if (fold)
      hipLaunchKernelGGL((k_round_split<Gate, true>), dim3(blocks), dim3(kBlock), lds, st, a);
    else
      hipLaunchKernelGGL((k_round_split<Gate, false>), dim3(blocks), dim3(kBlock), lds, st, a);
  }
  return launch_ok();
}

}  // namespace

#if defined(ZC_INST_VANILLA)
int launch_round_vanilla(bool fold, RoundKind kind, const RoundArgs& a, hipStream_t st) {
  return launch_round<GateVanilla>(fold, kind, a, st);
}
#elif defined(ZC_INST_PROD)
#define ZC_CAT2(a, b) a##b
#define ZC_CAT(a, b) ZC_CAT2(a, b)
int ZC_CAT(launch_round_prod, ZC_INST_PROD)(bool fold, RoundKind kind, const RoundArgs& a, hipStream_t st) {
  return launch_round<GateProd<ZC_INST_PROD>>(fold, kind, a, st);
}
#else
#error "build zc_inst.hip with -DZC_INST_VANILLA or -DZC_INST_PROD=<m>"
#endif

}  // namespace zc
