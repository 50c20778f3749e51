// BN254 scalar field F_p on the gfx950 VALU.
//
// The paper's accelerator multiplies with Montgomery multipliers for its
// 255-bit prime (Sec. 5.1, Table 2).  Here the Montgomery product is laid out
// for the CDNA4 vector ALU instead:
//
// * An element in registers is 9 limbs of 29 bits (radix 2^29, 261 bits),
//   in Montgomery form x*R mod p with R = 2^261.
// * The product is computed by product scanning: every partial product
//   a_i*b_j and m_i*p_j is one v_mad_u64_u32 that adds straight into a
//   64-bit column accumulator.  A column holds at most 18 products of
//   < 2^58 plus a < 2^35 carry, so it never overflows and no carry
//   instruction is needed between the multiplies (with 32-bit limbs every
//   step needs a separate 64-bit addend and carry handling).
// * R/p > 2^7 leaves room for lazy reduction: for inputs a < A*p, b < B*p
//   with A*B <= 128 the product is < p*(1 + A*B/128) <= 2p.
//
// In memory an element is 8 x 32-bit words holding the same integer (< p),
// one limb plane per word (limb-planar tables); fe_load8 / fe_store8 convert.
//
// Only p is written down; every derived constant (-p^-1 mod 2^29, R mod p,
// R^2 mod p, multiples of p) is computed by constexpr evaluation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zc {

constexpr int NL = 9;                    // limbs per element
constexpr uint32_t LM = (1u << 29) - 1;  // limb mask

struct Fe {
  uint32_t l[NL];
};

// p = 0x30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001
struct W8 {
  uint32_t v[8];
};
constexpr W8 kPWords = {{0xf0000001u, 0x43e1f593u, 0x79b97091u, 0x2833e848u, 0x8181585du,
                         0xb85045b6u, 0xe131a029u, 0x30644e72u}};

struct L9 {
  uint32_t v[NL];
};

namespace detail {

constexpr L9 words_to_l9(const W8& w) {
  L9 r{};
  for (int i = 0; i < NL; ++i) {
    const int bit = 29 * i, wi = bit / 32, s = bit % 32;
    uint64_t x = w.v[wi] >> s;
    if (wi + 1 < 8 && s > 0) x |= (uint64_t)w.v[wi + 1] << (32 - s);
    r.v[i] = (uint32_t)x & LM;
  }
  return r;
}

constexpr L9 kP = words_to_l9(kPWords);

constexpr bool geq(const L9& a, const L9& b) {
  for (int i = NL - 1; i >= 0; --i)
    if (a.v[i] != b.v[i]) return a.v[i] > b.v[i];
  return true;
}

constexpr bool same(const L9& a, const L9& b) {
  for (int i = 0; i < NL; ++i)
    if (a.v[i] != b.v[i]) return false;
  return true;
}

constexpr L9 add(const L9& a, const L9& b) {
  L9 r{};
  uint32_t c = 0;
  for (int i = 0; i < NL; ++i) {
    uint32_t s = a.v[i] + b.v[i] + c;
    c = s >> 29;
    r.v[i] = i == NL - 1 ? s : (s & LM);
  }
  return r;
}

constexpr L9 sub(const L9& a, const L9& b) {  // requires a >= b
  L9 r{};
  int32_t br = 0;
  for (int i = 0; i < NL; ++i) {
    int32_t t = (int32_t)a.v[i] - (int32_t)b.v[i] + br;
    br = t < 0 ? -1 : 0;
    r.v[i] = (uint32_t)t & LM;
  }
  return r;
}

constexpr L9 pow2_mod(int e) {
  L9 v{};
  v.v[0] = 1;
  for (int i = 0; i < e; ++i) {
    v = add(v, v);
    if (geq(v, kP)) v = sub(v, kP);
  }
  return v;
}

constexpr L9 mul_small(const L9& a, uint32_t k) {
  L9 r{};
  for (uint32_t i = 0; i < k; ++i) r = add(r, a);
  return r;
}

constexpr uint32_t neg_inv29() {
  uint32_t x = 1;  // Newton: x <- x (2 - p0 x) doubles the correct low bits
  for (int i = 0; i < 6; ++i) x *= 2u - kP.v[0] * x;
  return (0u - x) & LM;
}

// a b R^-1 mod p for a, b < p (the device product's steps, then one
// conditional subtraction), for constants.
constexpr L9 mont_mul(const L9& a, const L9& b) {
  const uint32_t ninv = neg_inv29();
  uint32_t m[NL] = {};
  L9 r{};
  uint64_t acc = 0;
  for (int k = 0; k < 2 * NL - 1; ++k) {
    for (int i = 0; i < NL; ++i) {
      const int j = k - i;
      if (j < 0 || j >= NL) continue;
      acc += (uint64_t)a.v[i] * b.v[j];
      if (i < k && i < NL) acc += (uint64_t)m[i] * kP.v[j];
    }
    if (k < NL) {
      m[k] = ((uint32_t)acc * ninv) & LM;
      acc += (uint64_t)m[k] * kP.v[0];
      acc >>= 29;
    } else {
      r.v[k - NL] = (uint32_t)acc & LM;
      acc >>= 29;
    }
  }
  r.v[NL - 1] = (uint32_t)acc;
  return geq(r, kP) ? sub(r, kP) : r;
}

// 1/n mod p for a small n >= 1: (k p + 1) / n for the k < n that makes the
// division exact (long division by n over the 29-bit limbs).
constexpr L9 inv_small(uint32_t n) {
  for (uint32_t k = 0; k < n; ++k) {
    L9 v{};
    v.v[0] = 1;
    v = add(v, mul_small(kP, k));
    uint64_t rem = 0;
    L9 q{};
    for (int i = NL - 1; i >= 0; --i) {
      const uint64_t cur = (rem << 29) | v.v[i];
      q.v[i] = (uint32_t)(cur / n);
      rem = cur % n;
    }
    if (rem == 0) return q;
  }
  return L9{};
}

}  // namespace detail

constexpr L9 kP = detail::kP;
constexpr uint32_t kNInv = detail::neg_inv29();  // -p^-1 mod 2^29
constexpr L9 kOne = detail::pow2_mod(261);       // R mod p: Montgomery form of 1
constexpr L9 kR2 = detail::pow2_mod(522);        // R^2 mod p
constexpr L9 kP2 = detail::mul_small(kP, 2);
constexpr L9 kP4 = detail::mul_small(kP, 4);
constexpr L9 kP8 = detail::mul_small(kP, 8);
constexpr L9 kP16 = detail::mul_small(kP, 16);
constexpr L9 kP32 = detail::mul_small(kP, 32);
constexpr L9 kP64 = detail::mul_small(kP, 64);

static_assert(((kP.v[0] * kNInv) & LM) == LM, "-p^-1 mod 2^29");

// R^(k+1) mod p, k = 0..15: the Montgomery form of R^k.
struct RPowers {
  L9 v[16];
  constexpr RPowers() : v{} {
    v[0] = kOne;
    for (int k = 1; k < 16; ++k) v[k] = detail::mont_mul(v[k - 1], kR2);
  }
};
constexpr RPowers kRPow{};

// Lagrange weights of the nodes 0..D: w_c = 1 / prod_{k != c} (c - k), in
// Montgomery form (D <= 6).  p(x) = sum_c w_c prod_{k != c} (x - k) p(c)
// for any p of degree <= D.
template <int D>
struct LagrangeW {
  L9 w[D + 1];
  L9 node[D + 1];   // c R mod p: the nodes in Montgomery form
  L9 wsh[D + 1];    // w_c R^(D+1): D Montgomery products with canonical factors leave w_c (...) R
  constexpr LagrangeW() : w{}, node{}, wsh{} {
    for (int c = 0; c <= D; ++c) {
      L9 v{};
      for (int k = 0; k < c; ++k) {
        v = detail::add(v, kOne);
        if (detail::geq(v, kP)) v = detail::sub(v, kP);
      }
      node[c] = v;
    }
    for (int c = 0; c <= D; ++c) {
      uint32_t den = 1;  // c! (D - c)!
      for (int k = 1; k <= c; ++k) den *= (uint32_t)k;
      for (int k = 1; k <= D - c; ++k) den *= (uint32_t)k;
      L9 v = detail::mont_mul(detail::inv_small(den), kR2);
      if ((D - c) % 2 == 1) v = detail::sub(kP, v);  // the sign of prod (c - k)
      w[c] = v;
      wsh[c] = detail::mont_mul(v, RPowers{}.v[D]);  // w R * R^(D+1) / R
    }
  }
};
// Lagrange weights of the nodes 0..N-1 in Montgomery form, for any N <= 12:
// w_k = (-1)^(N-1-k) / (k! (N-1-k)!), from the inverses of the small
// factorials (products of exact inverses of small integers).
template <int N>
struct LagrangeN {
  L9 w[N];     // w_k R
  L9 node[N];  // k R
  constexpr LagrangeN() : w{}, node{} {
    L9 invf[N]{};  // (1 / j!) R
    invf[0] = kOne;
    for (int j = 1; j < N; ++j)
      invf[j] = detail::mont_mul(invf[j - 1], detail::mont_mul(detail::inv_small((uint32_t)j), kR2));
    for (int k = 0; k < N; ++k) {
      L9 v = detail::mont_mul(invf[k], invf[N - 1 - k]);
      if ((N - 1 - k) % 2 == 1 && !detail::same(v, L9{})) v = detail::sub(kP, v);
      w[k] = v;
      L9 c{};
      for (int t = 0; t < k; ++t) {
        c = detail::add(c, kOne);
        if (detail::geq(c, kP)) c = detail::sub(c, kP);
      }
      node[k] = c;
    }
  }
};

static_assert(detail::same(detail::mont_mul(kR2, detail::pow2_mod(0)), kOne), "R^2 R^-1 = R");
static_assert(detail::same(kRPow.v[1], kR2) && detail::same(kRPow.v[2], detail::pow2_mod(783)),
              "powers of R from products equal those from doublings");
static_assert(kP.v[8] < (1u << 22), "p < 2^254");

// Constant limb i of a compile-time L9 (folded after unrolling).
#define ZC_CL(C, i) (C).v[i]

__device__ __forceinline__ Fe fe_zero() {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.l[i] = 0;
  return r;
}

__device__ __forceinline__ Fe fe_const(const L9& c) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.l[i] = c.v[i];
  return r;
}

// ---- conversion between the 8-word memory form and 9 x 29-bit limbs -------

__device__ __forceinline__ Fe fe_from_words(const uint32_t w[8]) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int bit = 29 * i, wi = bit / 32, s = bit % 32;
    uint32_t x;
    if (wi + 1 < 8 && s + 29 > 32)
      x = __builtin_amdgcn_alignbit(w[wi + 1], w[wi], s);
    else
      x = w[wi] >> s;
    r.l[i] = x & LM;
  }
  return r;
}

// 9 words (a value < 2^261) -> 9 x 29-bit limbs.
__device__ __forceinline__ Fe fe_from_words9(const uint32_t w[9]) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int bit = 29 * i, wi = bit / 32, s = bit % 32;
    uint32_t x;
    if (wi + 1 < 9 && s + 29 > 32)
      x = __builtin_amdgcn_alignbit(w[wi + 1], w[wi], s);
    else
      x = w[wi] >> s;
    r.l[i] = x & LM;
  }
  return r;
}

// Requires normalized limbs and a value < 2^256.
__device__ __forceinline__ void fe_to_words(const Fe& a, uint32_t w[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int bit = 32 * j, li = bit / 29, s = bit % 29;
    // word j = bits [32j, 32j+32) = (l_li >> s) | l_{li+1} << (29-s) | l_{li+2} << (58-s)
    uint32_t x = a.l[li] >> s;
    if (li + 1 < NL) x |= a.l[li + 1] << (29 - s);
    if (li + 2 < NL && 58 - s < 32) x |= a.l[li + 2] << (58 - s);
    w[j] = x;
  }
}

// ---- additive operations ----------------------------------------------------

// a + b as integers, limbs normalized (a, b normalized; value < 2^261).
__device__ __forceinline__ Fe fe_add(const Fe& a, const Fe& b) {
  Fe r;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const uint32_t s = a.l[i] + b.l[i] + c;
    c = s >> 29;
    r.l[i] = (i == NL - 1) ? s : (s & LM);
  }
  return r;
}

// a - C if a >= C, else a (a, C normalized; top limbs below 2^31).
__device__ __forceinline__ Fe fe_csub(const Fe& a, const L9& C) {
  Fe d;
  int32_t br = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int32_t t = (int32_t)a.l[i] - (int32_t)C.v[i] + br;
    if (i < NL - 1) {
      br = t >> 29;  // 0 or -1 (-2^30 < t < 2^29)
      d.l[i] = (uint32_t)t & LM;
    } else {
      br = t >> 31;  // the sign of a - C
      d.l[i] = (uint32_t)t;
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) d.l[i] = br ? a.l[i] : d.l[i];
  return d;
}

// a + C*... : a + K - b for a constant K >= b (b normalized, value b <= K).
__device__ __forceinline__ Fe fe_sub_plus(const Fe& a, const Fe& b, const L9& K) {
  Fe r;
  int32_t c = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int32_t t = (int32_t)a.l[i] + (int32_t)K.v[i] - (int32_t)b.l[i] + c;
    c = t >> 29;  // arithmetic shift: signed carry
    r.l[i] = (i == NL - 1) ? (uint32_t)t : ((uint32_t)t & LM);
  }
  return r;
}

// (a + b) mod p for a, b < p; result < p.
__device__ __forceinline__ Fe fe_addmod(const Fe& a, const Fe& b) { return fe_csub(fe_add(a, b), kP); }

// (a - b) mod p for a, b < p; result < p.
__device__ __forceinline__ Fe fe_submod(const Fe& a, const Fe& b) {
  return fe_csub(fe_sub_plus(a, b, kP), kP);
}

// Reduce a value < 2p into [0, p).
__device__ __forceinline__ Fe fe_reduce2(const Fe& a) { return fe_csub(a, kP); }

// Reduce a value < 32p into [0, p).
__device__ __forceinline__ Fe fe_reduce32(const Fe& a) {
  return fe_csub(fe_csub(fe_csub(fe_csub(fe_csub(a, kP16), kP8), kP4), kP2), kP);
}

// Reduce a value < 128p into [0, p).
__device__ __forceinline__ Fe fe_reduce128(const Fe& a) {
  return fe_reduce32(fe_csub(fe_csub(a, kP64), kP32));
}

// ---- Montgomery product -----------------------------------------------------

// a*b*R^-1 mod p up to a multiple of p: for a < A*p, b < B*p with
// A*B <= 128 the result is < 2p.  Limbs of a and b normalized (< 2^29;
// the top limb of a value < 2^258 is < 2^26).  Result limbs normalized.
__device__ __forceinline__ Fe fe_mul(const Fe& a, const Fe& b) {
  uint32_t m[NL];
  Fe r;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
#pragma unroll
    for (int i = 0; i < k; ++i) {
      acc = (uint64_t)a.l[i] * b.l[k - i] + acc;
      acc = (uint64_t)m[i] * ZC_CL(kP, k - i) + acc;
    }
    acc = (uint64_t)a.l[k] * b.l[0] + acc;
    m[k] = ((uint32_t)acc * kNInv) & LM;
    acc = (uint64_t)m[k] * ZC_CL(kP, 0) + acc;  // low 29 bits become 0
    acc >>= 29;
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; ++k) {
#pragma unroll
    for (int i = k - NL + 1; i < NL; ++i) {
      acc = (uint64_t)a.l[i] * b.l[k - i] + acc;
      acc = (uint64_t)m[i] * ZC_CL(kP, k - i) + acc;
    }
    r.l[k - NL] = (uint32_t)acc & LM;
    acc >>= 29;
  }
  r.l[NL - 1] = (uint32_t)acc;
  return r;
}

// Sum of N Montgomery products with one reduction: (sum_n a_n b_n) R^-1 mod p
// up to a multiple of p.  The products share the column accumulators and the
// m_i p_j half is done once, so N products cost 81 (N + 1) v_mad_u64_u32
// instead of 162 N.  For a_n < A_n p, b_n < B_n p with sum_n A_n B_n <= 128 the
// result is < 2p (as in fe_mul, since p / R < 2^-7).  A column holds at most
// 9 (N + 1) terms below 2^58 plus a carry below 2^35, so N <= 6 keeps it below
// 2^64.
template <int N>
__device__ __forceinline__ Fe fe_sop(const Fe (&a)[N], const Fe (&b)[N]) {
  static_assert(N >= 1 && N <= 6, "column sums below 2^64");
  uint32_t m[NL];
  Fe r;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
#pragma unroll
    for (int i = 0; i < k; ++i) {
#pragma unroll
      for (int n = 0; n < N; ++n) acc = (uint64_t)a[n].l[i] * b[n].l[k - i] + acc;
      acc = (uint64_t)m[i] * ZC_CL(kP, k - i) + acc;
    }
#pragma unroll
    for (int n = 0; n < N; ++n) acc = (uint64_t)a[n].l[k] * b[n].l[0] + acc;
    m[k] = ((uint32_t)acc * kNInv) & LM;
    acc = (uint64_t)m[k] * ZC_CL(kP, 0) + acc;  // low 29 bits become 0
    acc >>= 29;
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; ++k) {
#pragma unroll
    for (int i = k - NL + 1; i < NL; ++i) {
#pragma unroll
      for (int n = 0; n < N; ++n) acc = (uint64_t)a[n].l[i] * b[n].l[k - i] + acc;
      acc = (uint64_t)m[i] * ZC_CL(kP, k - i) + acc;
    }
    r.l[k - NL] = (uint32_t)acc & LM;
    acc >>= 29;
  }
  r.l[NL - 1] = (uint32_t)acc;
  return r;
}

// k * a for a small integer k <= 15 and a normalized a < p; result < k p,
// normalized (each limb product is one v_mad_u64_u32 with the running carry).
__device__ __forceinline__ Fe fe_mul_small(const Fe& a, uint32_t k) {
  Fe r;
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    c = (uint64_t)a.l[i] * k + c;
    r.l[i] = (i == NL - 1) ? (uint32_t)c : ((uint32_t)c & LM);
    c >>= 29;
  }
  return r;
}

// canonical x < p  ->  Montgomery form x*R mod p, < p.
__device__ __forceinline__ Fe fe_to_mont(const Fe& x) { return fe_reduce2(fe_mul(x, fe_const(kR2))); }

// Montgomery form (value < 2p)  ->  canonical x < p.
__device__ __forceinline__ Fe fe_from_mont(const Fe& a) {
  Fe one = fe_zero();
  one.l[0] = 1;
  return fe_reduce2(fe_mul(a, one));
}

// a + alpha (b - a) mod p, < p, for a, b < p and alpha < p in Montgomery form
// (the fold of a table pair with a challenge).  b - a is taken as b + p - a
// (< 2p, no reduction); alpha times it is < 2p (1 * 2 <= 128), plus a < 3p.
__device__ __forceinline__ Fe fe_lerp(const Fe& a, const Fe& b, const Fe& alpha) {
  return fe_csub(fe_csub(fe_add(a, fe_mul(alpha, fe_sub_plus(b, a, kP))), kP2), kP);
}

// Reduce a value < 128p below 2p.
__device__ __forceinline__ Fe fe_reduce128_to2(const Fe& a) {
  return fe_csub(fe_csub(fe_csub(fe_csub(fe_csub(fe_csub(a, kP64), kP32), kP16), kP8), kP4), kP2);
}

__device__ __forceinline__ bool fe_is_zero(const Fe& a) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) o |= a.l[i];
  return o == 0;
}

// 256-bit word form w < p ?
__device__ __forceinline__ bool words_lt_p(const uint32_t w[8]) {
  int32_t br = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t t = (int64_t)w[i] - (int64_t)kPWords.v[i] + br;
    br = t < 0 ? -1 : 0;
  }
  return br != 0;
}

}  // namespace zc
