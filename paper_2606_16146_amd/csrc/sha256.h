// SHA-256 (FIPS 180-4) on the device, for the Fiat-Shamir transcript.
//
// The paper derives each challenge from a hash of the round polynomial
// (Fig. 2, right: alpha_i <- Hash(G_i)); the hash itself is left open.  This
// library uses chained SHA-256 and runs it on the GPU, so a challenge never
// travels to the host between rounds.
//
// One lane hashes; the message is uniform across the wave, which would lead
// the compiler to run the rounds on the scalar unit, where every rotate has
// to cross to the vector unit and back.  The working state is therefore
// pinned to vector registers, and the round constants are immediates.
//
// Messages are passed as little-endian packed bytes in 32-bit words: byte k
// of the message is bits 8(k%4)..8(k%4)+7 of word k/4.  The digest is
// returned the same way, i.e. out[j] holds digest bytes 4j..4j+3, so reading
// out[] as little-endian 32-bit limbs gives the digest as a little-endian
// 256-bit integer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sha256_consts.h"

namespace zc {

__device__ __forceinline__ uint32_t sha_rotr(uint32_t x, uint32_t n) {
  return __builtin_amdgcn_alignbit(x, x, n);
}

__device__ __forceinline__ uint32_t sha_bswap(uint32_t x) { return __builtin_bswap32(x); }

// 3-input XOR and majority in one v_bitop3_b32 (truth tables 0x96, 0xE8; both
// symmetric in their inputs).
__device__ __forceinline__ uint32_t sha_xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t sha_maj(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// Keeps x in a vector register (no instruction is emitted).
__device__ __forceinline__ uint32_t sha_vreg(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// One SHA-256 round on the working variables (a..h as v[0..7]); the roles of
// the eight registers rotate, so 16 unrolled rounds need no moves.
#define ZC_SHA_ROUND(a, b, c, d, e, f, g, h, kw)                                      \
  do {                                                                               \
    const uint32_t S1_ = sha_xor3(sha_rotr(e, 6), sha_rotr(e, 11), sha_rotr(e, 25));  \
    const uint32_t ch_ = (e & f) | (~e & g);                                         \
    const uint32_t t1_ = h + S1_ + ch_ + (kw);                                       \
    const uint32_t S0_ = sha_xor3(sha_rotr(a, 2), sha_rotr(a, 13), sha_rotr(a, 22));  \
    d += t1_;                                                                        \
    h = t1_ + S0_ + sha_maj(a, b, c);                                                \
  } while (0)

// 16 rounds t = 16 it + r, r = 0..15; W[r] holds w_t on entry to round t (the
// message schedule is updated in place when it > 0).
__device__ __forceinline__ void sha256_16(uint32_t v[8], uint32_t W[16], int it) {
  const uint32_t* K = kSha256KDev + 16 * it;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (it > 0) {
      const uint32_t w15 = W[(r + 1) & 15], w2 = W[(r + 14) & 15];
      const uint32_t s0 = sha_xor3(sha_rotr(w15, 7), sha_rotr(w15, 18), w15 >> 3);
      const uint32_t s1 = sha_xor3(sha_rotr(w2, 17), sha_rotr(w2, 19), w2 >> 10);
      W[r] = W[r] + s0 + W[(r + 9) & 15] + s1;
    }
    const uint32_t kw = K[r] + W[r];
    switch (r & 7) {
      case 0: ZC_SHA_ROUND(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], kw); break;
      case 1: ZC_SHA_ROUND(v[7], v[0], v[1], v[2], v[3], v[4], v[5], v[6], kw); break;
      case 2: ZC_SHA_ROUND(v[6], v[7], v[0], v[1], v[2], v[3], v[4], v[5], kw); break;
      case 3: ZC_SHA_ROUND(v[5], v[6], v[7], v[0], v[1], v[2], v[3], v[4], kw); break;
      case 4: ZC_SHA_ROUND(v[4], v[5], v[6], v[7], v[0], v[1], v[2], v[3], kw); break;
      case 5: ZC_SHA_ROUND(v[3], v[4], v[5], v[6], v[7], v[0], v[1], v[2], kw); break;
      case 6: ZC_SHA_ROUND(v[2], v[3], v[4], v[5], v[6], v[7], v[0], v[1], kw); break;
      default: ZC_SHA_ROUND(v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[0], kw); break;
    }
  }
}

// Compression function: rounds 0..15 once, then a rolled loop of three
// 16-round steps.  The loop keeps the code to two copies of 16 rounds, so it
// stays in the instruction cache (a fully unrolled block is ~11 KB of code
// that a single wave would otherwise fetch once and never reuse).
__device__ __forceinline__ void sha256_compress(uint32_t h[8], uint32_t W[16]) {
  uint32_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = h[i];
  sha256_16(v, W, 0);
#pragma unroll 1
  for (int it = 1; it < 4; ++it) sha256_16(v, W, it);
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] += v[i];
}

__device__ __forceinline__ void sha256_init(uint32_t h[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = sha_vreg(kSha256H0[j]);
}

__device__ __forceinline__ void sha256_digest(const uint32_t h[8], uint32_t out[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) out[j] = sha_bswap(h[j]);
}

// SHA-256 of a message of LEN bytes, LEN a multiple of 4 known at compile
// time (the round messages): padding is resolved statically.
template <uint32_t LEN>
__device__ __forceinline__ void sha256_fixed(const uint32_t* msg, uint32_t out[8]) {
  static_assert(LEN % 4 == 0, "word-aligned messages only");
  constexpr uint32_t NB = (LEN + 9u + 63u) / 64u;
  constexpr uint32_t TW = NB * 16u;
  uint32_t h[8];
  sha256_init(h);
#pragma unroll 1
  for (uint32_t blk = 0; blk < NB; ++blk) {
    uint32_t W[16];
#pragma unroll
    for (uint32_t t = 0; t < 16; ++t) {
      const uint32_t w = blk * 16u + t;
      uint32_t x = 0;
      if (w * 4u < LEN) x = sha_bswap(msg[w]);
      if (w * 4u == LEN) x = 0x80000000u;
      if (w == TW - 1) x = LEN << 3;
      W[t] = sha_vreg(x);
    }
    sha256_compress(h, W);
  }
  sha256_digest(h, out);
}

// Big-endian word w of the padded message (FIPS 180-4 Sec. 5.1.1), any length.
__device__ __forceinline__ uint32_t sha_padded_word(const uint32_t* msg, uint32_t len,
                                                    uint32_t total_words, uint32_t w) {
  if (w == total_words - 1) return len << 3;
  if (w == total_words - 2) return len >> 29;
  const uint32_t b0 = 4u * w;
  if (b0 + 4u <= len) return sha_bswap(msg[w]);
  uint32_t x = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t bi = b0 + k;
    uint32_t v = 0;
    if (bi < len)
      v = (msg[bi >> 2] >> (8u * (bi & 3u))) & 0xffu;
    else if (bi == len)
      v = 0x80u;
    x = (x << 8) | v;
  }
  return x;
}

// SHA-256 of len bytes at msg (any length; used for T_0 and in tests).
__device__ inline void sha256(const uint32_t* msg, uint32_t len, uint32_t out[8]) {
  uint32_t h[8];
  sha256_init(h);
  const uint32_t nblocks = (len + 9u + 63u) / 64u;
  const uint32_t total_words = nblocks * 16u;
  for (uint32_t blk = 0; blk < nblocks; ++blk) {
    uint32_t W[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) W[t] = sha_vreg(sha_padded_word(msg, len, total_words, blk * 16u + t));
    sha256_compress(h, W);
  }
  sha256_digest(h, out);
}

// ---- block-parallel form for the round messages ---------------------------------
//
// The message schedule w_16..w_63 of a block depends only on that block's
// message words, so lane b of the calling block expands block b (with the
// round constants added) into LDS while the compression, the serial part,
// runs afterwards in lane 0 and reads k_t + w_t from there.

// 16 rounds from the words k[0..15] = k_t + w_t (the eight working
// variables' roles rotate, so 16 unrolled rounds need no moves).
__device__ __forceinline__ void sha256_16kw(uint32_t v[8], const uint32_t k[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    switch (r & 7) {
      case 0: ZC_SHA_ROUND(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], k[r]); break;
      case 1: ZC_SHA_ROUND(v[7], v[0], v[1], v[2], v[3], v[4], v[5], v[6], k[r]); break;
      case 2: ZC_SHA_ROUND(v[6], v[7], v[0], v[1], v[2], v[3], v[4], v[5], k[r]); break;
      case 3: ZC_SHA_ROUND(v[5], v[6], v[7], v[0], v[1], v[2], v[3], v[4], k[r]); break;
      case 4: ZC_SHA_ROUND(v[4], v[5], v[6], v[7], v[0], v[1], v[2], v[3], k[r]); break;
      case 5: ZC_SHA_ROUND(v[3], v[4], v[5], v[6], v[7], v[0], v[1], v[2], k[r]); break;
      case 6: ZC_SHA_ROUND(v[2], v[3], v[4], v[5], v[6], v[7], v[0], v[1], k[r]); break;
      default: ZC_SHA_ROUND(v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[0], k[r]); break;
    }
  }
}

// Rounds 16 it0 .. 63 on the working variables v, with k_t + w_t read from
// kw[0..63] (LDS).  Each group's 16 words are read during the previous
// group, so the rounds do not wait on LDS.
__device__ __forceinline__ void sha256_rounds_kw(uint32_t v[8], const uint32_t* kw, int it0) {
  uint32_t k[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) k[r] = kw[16 * it0 + r];
#pragma unroll 1
  for (int it = it0; it < 4; ++it) {
    const int nx = it < 3 ? it + 1 : 3;
    uint32_t kn[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) kn[r] = kw[16 * nx + r];
    sha256_16kw(v, k);
#pragma unroll
    for (int r = 0; r < 16; ++r) k[r] = kn[r];
  }
}

// ---- the same rounds on the scalar unit -------------------------------------------
//
// With wave-uniform operands (SGPRs) every lane of one wave runs the code and
// the scalar unit executes it once.  The scalar unit has no rotate: rotr(x, n)
// is the low word of the 64-bit (x:x) >> n, one s_lshr_b64 (pure ALU, no
// memory access).  A round is ~25 scalar instructions against 14 vector ones,
// but scalar instructions issue without the vector pipeline's dependency
// stalls.
template <int N>
__device__ __forceinline__ uint32_t sha_srotr(uint32_t x) {
  x = __builtin_amdgcn_readfirstlane(x);  // no instruction when x is already uniform
  const uint64_t xx = ((uint64_t)x << 32) | x;
  uint64_t r;
  asm("s_lshr_b64 %0, %1, %2" : "=s"(r) : "s"(xx), "n"(N));
  return (uint32_t)r;
}

#define ZC_SHA_ROUND_S(a, b, c, d, e, f, g, h, kw)                                          \
  do {                                                                                       \
    const uint32_t S1_ = sha_srotr<6>(e) ^ sha_srotr<11>(e) ^ sha_srotr<25>(e);               \
    const uint32_t ch_ = g ^ (e & (f ^ g));                                                  \
    const uint32_t t1_ = h + S1_ + ch_ + (kw);                                               \
    const uint32_t S0_ = sha_srotr<2>(a) ^ sha_srotr<13>(a) ^ sha_srotr<22>(a);               \
    d += t1_;                                                                                \
    h = t1_ + S0_ + ((a & b) | (c & (a | b)));                                               \
  } while (0)

__device__ __forceinline__ void sha256_16kw_s(uint32_t v[8], const uint32_t k[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    switch (r & 7) {
      case 0: ZC_SHA_ROUND_S(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], k[r]); break;
      case 1: ZC_SHA_ROUND_S(v[7], v[0], v[1], v[2], v[3], v[4], v[5], v[6], k[r]); break;
      case 2: ZC_SHA_ROUND_S(v[6], v[7], v[0], v[1], v[2], v[3], v[4], v[5], k[r]); break;
      case 3: ZC_SHA_ROUND_S(v[5], v[6], v[7], v[0], v[1], v[2], v[3], v[4], k[r]); break;
      case 4: ZC_SHA_ROUND_S(v[4], v[5], v[6], v[7], v[0], v[1], v[2], v[3], k[r]); break;
      case 5: ZC_SHA_ROUND_S(v[3], v[4], v[5], v[6], v[7], v[0], v[1], v[2], k[r]); break;
      case 6: ZC_SHA_ROUND_S(v[2], v[3], v[4], v[5], v[6], v[7], v[0], v[1], k[r]); break;
      default: ZC_SHA_ROUND_S(v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[0], k[r]); break;
    }
  }
}

// sha256_rounds_kw on the scalar unit: v wave-uniform, kw in LDS read as
// uniform values (the next group's 16 words read during the current group);
// every lane of the wave must run it.
__device__ __forceinline__ void sha256_rounds_kw_s(uint32_t v[8], const uint32_t* kw, int it0) {
  uint32_t k[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) k[r] = __builtin_amdgcn_readfirstlane(kw[16 * it0 + r]);
#pragma unroll 1
  for (int it = it0; it < 4; ++it) {
    const int nx = it < 3 ? it + 1 : 3;
    uint32_t kn[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) kn[r] = kw[16 * nx + r];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = __builtin_amdgcn_readfirstlane(v[i]);
    sha256_16kw_s(v, k);
#pragma unroll
    for (int r = 0; r < 16; ++r) k[r] = __builtin_amdgcn_readfirstlane(kn[r]);
  }
}

__device__ __forceinline__ void sha256_compress_kw_s(uint32_t h[8], const uint32_t* kw) {
  uint32_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = h[i];
  sha256_rounds_kw_s(v, kw, 0);
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] += v[i];
}

// Compression rounds with k_t + w_t precomputed (kw[0..63]).
__device__ __forceinline__ void sha256_compress_kw(uint32_t h[8], const uint32_t* kw) {
  uint32_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = h[i];
  sha256_rounds_kw(v, kw, 0);
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] += v[i];
}

// Rounds 0..15 of the first block of a message whose words are msg[0..15]
// (little-endian packed), the round constants as immediates; v holds the
// chaining value on entry.
__device__ __forceinline__ void sha256_first16(uint32_t v[8], const uint32_t* msg) {
  uint32_t k[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) k[r] = kSha256K[r] + sha_bswap(msg[r]);
  sha256_16kw(v, k);
}

// Message schedule of block b of a LEN-byte message (LEN a multiple of 4,
// compile-time): writes k_t + w_t of block b to kw[64 b + t].  One lane per
// block; a barrier must follow before the compression reads kw.
template <uint32_t LEN>
__device__ __forceinline__ void sha256_expand_block(const uint32_t* msg, uint32_t* kw, uint32_t b) {
  static_assert(LEN % 4 == 0, "word-aligned messages only");
  constexpr uint32_t NB = (LEN + 9u + 63u) / 64u;
  constexpr uint32_t TW = NB * 16u;
  uint32_t W[16];
#pragma unroll
  for (uint32_t t = 0; t < 16; ++t) {
    const uint32_t w = b * 16u + t;
    uint32_t x = 0;
    if (w * 4u < LEN) x = sha_bswap(msg[w]);
    if (w * 4u == LEN) x = 0x80000000u;
    if (w == TW - 1) x = LEN << 3;
    W[t] = x;
    kw[b * 64u + t] = x + kSha256K[t];
  }
#pragma unroll
  for (int t = 16; t < 64; ++t) {
    const uint32_t w15 = W[(t - 15) & 15], w2 = W[(t - 2) & 15];
    const uint32_t s0 = sha_xor3(sha_rotr(w15, 7), sha_rotr(w15, 18), w15 >> 3);
    const uint32_t s1 = sha_xor3(sha_rotr(w2, 17), sha_rotr(w2, 19), w2 >> 10);
    W[t & 15] = W[t & 15] + s0 + W[(t - 7) & 15] + s1;
    kw[b * 64u + t] = W[t & 15] + kSha256K[t];
  }
}

// The same for a message of len bytes known at run time (any length, at most
// kwords/64 blocks): lane b < nblocks expands block b.  Returns the number of
// blocks.
__device__ __forceinline__ uint32_t sha256_schedule_var(const uint32_t* msg, uint32_t len, uint32_t* kw) {
  const uint32_t nb = (len + 9u + 63u) / 64u;
  const uint32_t tw = nb * 16u;
  if (threadIdx.x < nb) {
    const uint32_t b = threadIdx.x;
    uint32_t W[16];
#pragma unroll
    for (uint32_t t = 0; t < 16; ++t) {
      W[t] = sha_padded_word(msg, len, tw, b * 16u + t);
      kw[b * 64u + t] = W[t] + kSha256K[t];
    }
#pragma unroll
    for (int t = 16; t < 64; ++t) {
      const uint32_t w15 = W[(t - 15) & 15], w2 = W[(t - 2) & 15];
      const uint32_t s0 = sha_xor3(sha_rotr(w15, 7), sha_rotr(w15, 18), w15 >> 3);
      const uint32_t s1 = sha_xor3(sha_rotr(w2, 17), sha_rotr(w2, 19), w2 >> 10);
      W[t & 15] = W[t & 15] + s0 + W[(t - 7) & 15] + s1;
      kw[b * 64u + t] = W[t & 15] + kSha256K[t];
    }
  }
  return nb;
}

// The compression of nb blocks whose schedules sha256_schedule_var left in
// kw; one lane.  The digest is in the byte order of sha256().
__device__ __forceinline__ void sha256_compress_blocks(const uint32_t* kw, uint32_t nb, uint32_t out[8]) {
  uint32_t h[8];
  sha256_init(h);
#pragma unroll 1
  for (uint32_t b = 0; b < nb; ++b) sha256_compress_kw(h, kw + b * 64u);
  sha256_digest(h, out);
}

}  // namespace zc
