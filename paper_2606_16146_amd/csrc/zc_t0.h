// The opening transcript state T_0 (one block of a setup launch).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sha256.h"
#include "zc_device.h"

namespace zc {

// T_0 = SHA-256("ZCv1" || u32 mu || u32 gate || u32 m || enc(r_1) .. enc(r_mu)),
// one block: lane b expands message block b, lane 0 compresses.
__device__ __forceinline__ void t0_body(const uint32_t* __restrict__ r, uint32_t mu, uint32_t gate, uint32_t m,
                                        Ctrl* ctrl) {
  __shared__ uint32_t m0[4 + kMuMax * 8];
  __shared__ uint32_t kw[((16u + 32u * kMuMax + 9u + 63u) / 64u) * 64u];
  if (threadIdx.x == 0) {
    m0[0] = 0x3176435au;  // bytes 'Z' 'C' 'v' '1'
    m0[1] = mu;
    m0[2] = gate;
    m0[3] = m;
  }
  for (uint32_t i = threadIdx.x; i < mu * 8; i += blockDim.x) m0[4 + i] = r[i];
  __syncthreads();
  const uint32_t nb = sha256_schedule_var(m0, 16u + 32u * mu, kw);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t dg[8];
    sha256_compress_blocks(kw, nb, dg);
#pragma unroll
    for (int k = 0; k < 8; ++k) ctrl->ts[k] = dg[k];
  }
}

}  // namespace zc
