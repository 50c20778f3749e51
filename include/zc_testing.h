/*
 * zc_testing.h -- test and measurement hooks of libzc (not part of the prover's API).
 *
 * They run single device building blocks of the prover on caller buffers so
 * that tests can compare them with Python integers and hashlib: the field
 * arithmetic (Montgomery product of Sec. 5.1 / Table 2's modular
 * multiplier, modular addition) and the SHA-256 used for the Fiat-Shamir
 * challenges of Fig. 2.  Same conventions as zc.h: device pointers,
 * canonical 8 x uint32 little-endian elements, work enqueued on `stream`.
 */
#ifndef ZC_TESTING_H
#define ZC_TESTING_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "zc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ZC_TEST_MUL = 0,        /* out = a*b mod p (canonical in, canonical out) */
  ZC_TEST_ADD = 1,        /* out = a+b mod p */
  ZC_TEST_SUB = 2,        /* out = a-b mod p */
  ZC_TEST_MONT_RAW = 3,   /* out = A*B*2^-261 mod p for raw 256-bit A, B (any value < 2^256) */
  ZC_TEST_TO_MONT = 4,    /* out = a*2^261 mod p */
  ZC_TEST_FROM_MONT = 5,  /* out = a*2^-261 mod p, a any value < 2^256 */
  ZC_TEST_EXT_SQR = 6     /* E = a + 10*b as plain sum (a, b < p); out = E*E*2^-522 mod p */
} zc_test_op;

/* Element-wise op over n elements: a, b, out are uint32[n][8]. */
int zc_test_field(int op, const uint32_t* a, const uint32_t* b, uint32_t* out, uint64_t n, hipStream_t stream);

/* zc_prove (same launches, same outputs) with a HIP event recorded on
   `stream` right before and right after the round kernel of every round
   (the one-block finisher that follows it is outside the bracket): events is
   a host array of 2*mu hipEvent_t, round i bracketed by events[2(i-1)] and
   events[2(i-1)+1]; rounds run inside the tail get two back-to-back events.
   For measuring the round kernels. */
int zc_prove_profiled(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws,
                      uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, void* events,
                      hipStream_t stream);

/* Which kernel zc_prove uses for round i (1..mu) of a proof of this shape:
   0 one thread per pair, 1 sixteen lanes per pair, 2 sixteen lanes per pair
   whose finisher then runs all later rounds and the openings in one block,
   3 a round run inside such a tail, 4 sixteen lanes per pair evaluated for
   every candidate alpha_{i-1} in 0..d in the launch that finishes round i-1
   (gates of degree <= 3), 5 the same whose finisher then runs the tail.
   Negative zc_status for a bad shape or i. */
int zc_prove_round_kernel(const zc_shape* shape, uint32_t i);

/* ---- peak-rate microbenchmarks (timed by the caller with events on `stream`) ----

   zc_bench_mad: `blocks` blocks of 256 threads; each thread runs `chains`
   (1 or 8) independent chains of iters * 32 dependent v_mad_u64_u32
   (64-bit multiply-add, the instruction of the field product).  Operations:
   blocks * 256 * chains * iters * 32.  sink: device, >= blocks words (written
   only for one improbable value). */
int zc_bench_mad(uint32_t blocks, uint32_t chains, uint32_t iters, uint32_t* sink, hipStream_t stream);

/* zc_bench_fmul: the library's Montgomery product (radix 2^29 product
   scanning), `chains` (1 or 4) independent chains of `iters` products per
   thread over `blocks` blocks of 256 threads.  in: 64 elements (uint32[64][8],
   limbs < 2^29 after conversion, values < p); out: device, >= 64 * 8 words. */
int zc_bench_fmul(uint32_t blocks, uint32_t chains, uint32_t iters, const uint32_t* in, uint32_t* out,
                  hipStream_t stream);

/* zc_bench_sha: one lane chains n SHA-256 compressions of a 64-byte block;
   variant 0 reads k_t + w_t from LDS, variant 1 expands the message schedule
   on the fly, variant 2 is variant 0 while the block's three other waves
   multiply field elements, variant 3 is variant 0 on the scalar unit (the
   whole of one wave, uniform operands).  in: 64 elements (uint32[64][8], values < p).
   out: device uint32[16 + 256]: [0..8) the final chaining value, [8..10) the
   shader clock cycles of lane 0's loop (s_memtime, lo/hi), [10..12) the same
   interval in 100 MHz ticks (s_memrealtime), the rest scratch. */
int zc_bench_sha(uint32_t variant, uint32_t n, const uint32_t* in, uint32_t* out, hipStream_t stream);

/* SHA-256 of len bytes (msg: little-endian packed uint32 words); out: 32 bytes as uint32[8]. */
int zc_test_sha256(const uint32_t* msg, uint32_t len, uint32_t* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* ZC_TESTING_H */
