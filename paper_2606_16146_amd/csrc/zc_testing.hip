// Test hooks declared in include/zc_testing.h.
#include <hip/hip_runtime.h>

#include "../../include/zc_testing.h"
#include "zc_device.h"

using namespace zc;

namespace {

__global__ __launch_bounds__(kBlock) void k_test_field(int op, const uint32_t* __restrict__ a,
                                                       const uint32_t* __restrict__ b, uint32_t* __restrict__ out,
                                                       uint64_t n) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const Fe x = load_words_fe(a + j * 8);
  const Fe y = load_words_fe(b + j * 8);
  Fe r = fe_zero();
  switch (op) {
    case ZC_TEST_MUL: r = fe_from_mont(fe_mul(fe_to_mont(x), fe_to_mont(y))); break;
    case ZC_TEST_ADD: r = fe_addmod(x, y); break;
    case ZC_TEST_SUB: r = fe_submod(x, y); break;
    case ZC_TEST_MONT_RAW: r = fe_reduce32(fe_mul(x, y)); break;
    case ZC_TEST_TO_MONT: r = fe_to_mont(x); break;
    case ZC_TEST_FROM_MONT: r = fe_reduce32(fe_mul(x, [] { Fe o = fe_zero(); o.l[0] = 1; return o; }())); break;
    case ZC_TEST_EXT_SQR: {
      Fe e = x;
#pragma unroll
      for (int k = 0; k < 10; ++k) e = fe_add(e, y);  // < 11p
      r = fe_from_mont(fe_reduce2(fe_mul(e, e)));
      break;
    }
    default: break;
  }
  store_words_fe(out + j * 8, r);
}

__global__ void k_test_sha(const uint32_t* __restrict__ msg, uint32_t len, uint32_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t dg[8];
  sha256(msg, len, dg);
#pragma unroll
  for (int k = 0; k < 8; ++k) out[k] = dg[k];
}

}  // namespace

extern "C" {

int zc_test_field(int op, const uint32_t* a, const uint32_t* b, uint32_t* out, uint64_t n, hipStream_t stream) {
  if (!a || !b || !out || n == 0 || op < 0 || op > ZC_TEST_EXT_SQR) return -1;
  hipLaunchKernelGGL(k_test_field, dim3((uint32_t)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, op, a, b,
                     out, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int zc_test_sha256(const uint32_t* msg, uint32_t len, uint32_t* out, hipStream_t stream) {
  if (!msg || !out) return -1;
  hipLaunchKernelGGL(k_test_sha, dim3(1), dim3(64), 0, stream, msg, len, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
