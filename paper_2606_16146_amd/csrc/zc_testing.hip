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

// ---- peak-rate microbenchmarks ------------------------------------------------------

// v_mad_u64_u32 throughput: CH independent 64-bit multiply-add chains per
// thread, 32 steps per iteration.  Each step multiplies the low word of its
// own accumulator, so no step can be folded into another.  The sink store is
// taken only for one improbable value, which keeps every chain live.
template <int CH>
__global__ __launch_bounds__(kBlock) void k_bench_mad(uint32_t iters, uint32_t seed, uint32_t magic,
                                                     uint32_t* __restrict__ sink) {
  uint64_t acc[CH];
  const uint32_t b = seed * 2654435761u + threadIdx.x;
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = ((uint64_t)(threadIdx.x + 1) << 20) + (uint64_t)c * 0x9e3779b9u;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 32; ++u) {
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = (uint64_t)(uint32_t)acc[c] * b + acc[c];
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) x ^= (uint32_t)acc[c] ^ (uint32_t)(acc[c] >> 32);
  if (x == magic) sink[blockIdx.x] = x;
}

// Montgomery product throughput: CH independent chains x <- x * y per thread
// (x < 2p, y < p keeps x < 2p), `iters` products per chain.  The sink
// compares with a run-time value, so the compiler cannot drop a chain.
template <int CH>
__global__ __launch_bounds__(kBlock) void k_bench_fmul(const uint32_t* __restrict__ in, uint32_t iters,
                                                      uint32_t magic, uint32_t* __restrict__ out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const Fe y = load_words_fe(in + (t & 63u) * 8);
  Fe x[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) x[c] = load_words_fe(in + ((t + 1 + c) & 63u) * 8);
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) x[c] = fe_mul(x[c], y);
  }
  uint32_t h = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int i = 0; i < NL; ++i) h ^= x[c].l[i];
  if (h == magic) out[t] = h;
  if (t < 64) store_words_fe(out + t * 8, fe_reduce2(x[0]));
}

// One lane chains n SHA-256 compressions of one block: variant 0 takes
// k_t + w_t from LDS (the round messages' blocks after the first), variant 1
// expands the schedule on the fly (their first block), variant 2 is variant 0
// while the block's other three waves run chains of field products (a
// finisher's side work).  Lane 0 also reads the shader clock (s_memtime) and
// the constant 100 MHz clock (s_memrealtime) around its loop.
__global__ __launch_bounds__(kBlock) void k_bench_sha(uint32_t variant, uint32_t n, const uint32_t* __restrict__ in,
                                                     uint32_t* __restrict__ out) {
  __shared__ uint32_t kw[64];
  __shared__ uint32_t stop;
  if (threadIdx.x < 64) kw[threadIdx.x] = threadIdx.x * 0x9e3779b9u + 0x1234567u;
  if (threadIdx.x == 0) stop = 0;
  __syncthreads();
  if (threadIdx.x >= 64) {
    // side waves: products until lane 0 is done (at most 8 n of them)
    if (variant != 2) return;
    Fe x = load_words_fe(in + (threadIdx.x & 63u) * 8), y = load_words_fe(in + ((threadIdx.x + 7) & 63u) * 8);
    uint32_t k = 0;
    while (k < 8 * n && __atomic_load_n(&stop, __ATOMIC_RELAXED) == 0) {
      x = fe_mul(x, y);
      ++k;
    }
    if (fe_is_zero(x)) out[16 + threadIdx.x] = k;
    return;
  }
  if (variant == 3) {
    // the scalar-unit rounds: the whole of wave 0, uniform operands
    const uint64_t c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    uint32_t h[8];
    sha256_init(h);
    for (uint32_t i = 0; i < n; ++i) sha256_compress_kw_s(h, kw);
    const uint64_t c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) out[k] = h[k];
      out[8] = (uint32_t)(c1 - c0);
      out[9] = (uint32_t)((c1 - c0) >> 32);
      out[10] = (uint32_t)(r1 - r0);
      out[11] = (uint32_t)((r1 - r0) >> 32);
    }
    return;
  }
  if (threadIdx.x != 0) return;
  const uint64_t c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  uint32_t h[8];
  sha256_init(h);
  if (variant != 1) {
    for (uint32_t i = 0; i < n; ++i) sha256_compress_kw(h, kw);
  } else {
    for (uint32_t i = 0; i < n; ++i) {
      uint32_t W[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) W[k] = sha_vreg(h[k & 7] ^ (uint32_t)k);
      sha256_compress(h, W);
    }
  }
  const uint64_t c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
  __atomic_store_n(&stop, 1u, __ATOMIC_RELAXED);
#pragma unroll
  for (int k = 0; k < 8; ++k) out[k] = h[k];
  out[8] = (uint32_t)(c1 - c0);
  out[9] = (uint32_t)((c1 - c0) >> 32);
  out[10] = (uint32_t)(r1 - r0);
  out[11] = (uint32_t)((r1 - r0) >> 32);
}

}  // namespace

extern "C" {

int zc_bench_mad(uint32_t blocks, uint32_t chains, uint32_t iters, uint32_t* sink, hipStream_t stream) {
  if (!sink || blocks == 0 || iters == 0) return -1;
  if (chains == 1)
    hipLaunchKernelGGL(k_bench_mad<1>, dim3(blocks), dim3(kBlock), 0, stream, iters, 7u, iters ^ 0x5ca1ab1eu, sink);
  else if (chains == 8)
    hipLaunchKernelGGL(k_bench_mad<8>, dim3(blocks), dim3(kBlock), 0, stream, iters, 7u, iters ^ 0x5ca1ab1eu, sink);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int zc_bench_fmul(uint32_t blocks, uint32_t chains, uint32_t iters, const uint32_t* in, uint32_t* out,
                  hipStream_t stream) {
  if (!in || !out || blocks == 0 || iters == 0) return -1;
  if (chains == 1)
    hipLaunchKernelGGL(k_bench_fmul<1>, dim3(blocks), dim3(kBlock), 0, stream, in, iters, iters & 0xfffu, out);
  else if (chains == 4)
    hipLaunchKernelGGL(k_bench_fmul<4>, dim3(blocks), dim3(kBlock), 0, stream, in, iters, iters & 0xfffu, out);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int zc_bench_sha(uint32_t variant, uint32_t n, const uint32_t* in, uint32_t* out, hipStream_t stream) {
  if (!in || !out || variant > 3) return -1;
  hipLaunchKernelGGL(k_bench_sha, dim3(1), dim3(kBlock), 0, stream, variant, n, in, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

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
