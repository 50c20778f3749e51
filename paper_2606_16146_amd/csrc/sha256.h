// SHA-256 (FIPS 180-4) on the device, for the Fiat-Shamir transcript.
//
// The paper derives each challenge from a hash of the round polynomial
// (Fig. 2, right: alpha_i <- Hash(G_i)); the hash itself is left open.  This
// library uses chained SHA-256 and runs it on the GPU, so a challenge never
// travels to the host between rounds.
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

// Big-endian word w of the padded message (FIPS 180-4 Sec. 5.1.1).
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

__device__ __forceinline__ void sha256_compress(uint32_t h[8], uint32_t W[16]) {
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll
  for (int t = 0; t < 64; ++t) {
    uint32_t wt;
    if (t < 16) {
      wt = W[t];
    } else {
      const uint32_t w15 = W[(t - 15) & 15], w2 = W[(t - 2) & 15];
      const uint32_t s0 = sha_rotr(w15, 7) ^ sha_rotr(w15, 18) ^ (w15 >> 3);
      const uint32_t s1 = sha_rotr(w2, 17) ^ sha_rotr(w2, 19) ^ (w2 >> 10);
      wt = W[t & 15] + s0 + W[(t - 7) & 15] + s1;
      W[t & 15] = wt;
    }
    const uint32_t S1 = sha_rotr(e, 6) ^ sha_rotr(e, 11) ^ sha_rotr(e, 25);
    const uint32_t ch = (e & f) ^ (~e & g);
    const uint32_t t1 = hh + S1 + ch + kSha256K[t] + wt;
    const uint32_t S0 = sha_rotr(a, 2) ^ sha_rotr(a, 13) ^ sha_rotr(a, 22);
    const uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
    const uint32_t t2 = S0 + maj;
    hh = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + t2;
  }
  h[0] += a;
  h[1] += b;
  h[2] += c;
  h[3] += d;
  h[4] += e;
  h[5] += f;
  h[6] += g;
  h[7] += hh;
}

// SHA-256 of len bytes at msg (little-endian packed words); out as described above.
__device__ inline void sha256(const uint32_t* msg, uint32_t len, uint32_t out[8]) {
  uint32_t h[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = kSha256H0[j];
  const uint32_t nblocks = (len + 9u + 63u) / 64u;
  const uint32_t total_words = nblocks * 16u;
  for (uint32_t blk = 0; blk < nblocks; ++blk) {
    uint32_t W[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) W[t] = sha_padded_word(msg, len, total_words, blk * 16u + t);
    sha256_compress(h, W);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) out[j] = sha_bswap(h[j]);
}

}  // namespace zc
