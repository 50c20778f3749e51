// Kernels of the ZeroCheck SumCheck prover (gfx950).
//
// What is computed follows the multilinear ZeroCheck of Fig. 2 (right) of
// "When Proofs Meet Hardware": build eq_r once (Sec. 3.3), then for each
// round i evaluate G_i(X) = sum over the remaining hypercube of
// f_M(ext(X)) * eq(ext(X)) at X = 0..d+1, derive alpha_i from the
// transcript, and fold every table (eq included) with alpha_i (Sec. 4.1:
// update, extend, multiply, accumulate).  Variable x_1 is the most
// significant index bit, so round i pairs entries j and j + 2^(mu-i) and the
// fold of a table can be written in place: the thread that owns pair j reads
// and writes only slots j, j+q, j+2q, j+3q.
//
// Value bounds (the field code's contract is a product of inputs < A*p and
// < B*p with A*B <= 128 lands below 2p):
// * every table entry in memory is fully reduced, < p;
// * Delta = u1 - u0 mod p is < p, so the extension e(X) = u0 + X*Delta built
//   by plain additions is < (X+1) p <= (d+2) p <= 11 p;
// * gate values are kept below 11 p before the product with eq's extension;
// * per-thread sums of products stay below 2p.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zc_device.h"

namespace zc {

// ---- gates ---------------------------------------------------------------------
//
// eval() takes the extensions of the witness tables at one point X
// (each < (D+2) p) and returns f_M at X, below 11 p.

// f = qM*a*b + qL*a + qR*b + qO*c + qC, columns [a b c qM qL qR qO qC], degree 3.
struct GateVanilla {
  static constexpr int K = 8;
  static constexpr int D = 3;
  __device__ static __forceinline__ Fe eval(const Fe* e) {
    // e < 5p.  a*(qM*b + qL) + qR*b + qO*c + qC: four products.
    const Fe t1 = fe_mul(e[3], e[1]);            // < 2p (5*5)
    const Fe t2 = fe_add(t1, e[4]);              // < 7p
    const Fe t3 = fe_mul(e[0], t2);              // < 2p (5*7)
    const Fe t4 = fe_mul(e[5], e[1]);            // < 2p
    const Fe t5 = fe_mul(e[6], e[2]);            // < 2p
    return fe_add(fe_add(fe_add(t3, t4), t5), e[7]);  // < 11p
  }
};

constexpr L9 kP11 = detail::mul_small(kP, 11);

// f = s*w1*...*wm - o, columns [s w1 .. wm o], degree m+1.
template <int M>
struct GateProd {
  static constexpr int K = M + 2;
  static constexpr int D = M + 1;
  __device__ static __forceinline__ Fe eval(const Fe* e) {
    // e < (M+3) p <= 11 p.
    Fe prod = fe_mul(e[0], e[1]);  // < 2p (11*11 <= 121)
#pragma unroll
    for (int k = 2; k <= M; ++k) prod = fe_mul(prod, e[k]);  // < 2p (2*11)
    // prod + 11p - o  in (0, 13p)  ->  < 8p after one conditional subtraction
    return fe_csub(fe_sub_plus(prod, e[M + 1], kP11), kP8);
  }
};

// ---- reductions ---------------------------------------------------------------

__device__ __forceinline__ Fe shfl_xor_fe(const Fe& a, int mask) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.l[i] = __shfl_xor(a.l[i], mask, 64);
  return r;
}

// Sum (mod p) of NV values over the block; values < p on entry.  The block's
// totals are written by thread 0 to out[v*8 .. v*8+7] as words (< p).
template <int NV>
__device__ __forceinline__ void block_reduce_store(Fe (&v)[NV], uint32_t* __restrict__ out) {
  __shared__ uint32_t red[kBlock / 64][NV][NL];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int x = 0; x < NV; ++x) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v[x] = fe_addmod(v[x], shfl_xor_fe(v[x], s));
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < NL; ++i) red[wave][x][i] = v[x].l[i];
    }
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int x = threadIdx.x;
    Fe s;
#pragma unroll
    for (int i = 0; i < NL; ++i) s.l[i] = red[0][x][i];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      Fe t;
#pragma unroll
      for (int i = 0; i < NL; ++i) t.l[i] = red[w][x][i];
      s = fe_addmod(s, t);
    }
    store_words_fe(out + x * 8, s);
  }
}

// ---- round kernel ---------------------------------------------------------------
//
// FOLD = false: evaluate G_i on tables holding 2q live entries (pairs j, j+q).
// FOLD = true : the tables hold 4q entries; fold them with alpha_{i-1}
//               (u[j] = t[j] + alpha (t[j+2q] - t[j]), same for j+q), write
//               u[j], u[j+q] to dst, then evaluate G_i on (u[j], u[j+q]).
// Every block writes its d+2 partial sums (Montgomery, < p) to partials.
template <class Gate, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_round(TabPtrs src, TabPtrs dst, uint64_t src_pitch,
                                                  uint64_t dst_pitch, uint64_t q,
                                                  const uint32_t* __restrict__ alpha_words,
                                                  uint32_t* __restrict__ partials) {
  constexpr int K = Gate::K + 1;  // witness tables + eq (last)
  constexpr int NE = Gate::D + 2;
  Fe acc[NE];
#pragma unroll
  for (int x = 0; x < NE; ++x) acc[x] = fe_zero();
  Fe alpha;
  if (FOLD) alpha = load_words_fe(alpha_words);

  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
    Fe lo[K], dl[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      Fe u0, u1;
      if (FOLD) {
        const Fe a0 = load_el(src.p[t], src_pitch, j);
        const Fe a1 = load_el(src.p[t], src_pitch, j + q);
        const Fe a2 = load_el(src.p[t], src_pitch, j + 2 * q);
        const Fe a3 = load_el(src.p[t], src_pitch, j + 3 * q);
        u0 = fe_addmod(a0, fe_reduce2(fe_mul(alpha, fe_submod(a2, a0))));
        u1 = fe_addmod(a1, fe_reduce2(fe_mul(alpha, fe_submod(a3, a1))));
        store_el(dst.p[t], dst_pitch, j, u0);
        store_el(dst.p[t], dst_pitch, j + q, u1);
      } else {
        u0 = load_el(src.p[t], src_pitch, j);
        u1 = load_el(src.p[t], src_pitch, j + q);
      }
      lo[t] = u0;
      dl[t] = fe_submod(u1, u0);
    }
#pragma unroll
    for (int x = 0; x < NE; ++x) {
      if (x > 0) {
#pragma unroll
        for (int t = 0; t < K; ++t) lo[t] = fe_add(lo[t], dl[t]);  // e(x) < (x+1) p
      }
      const Fe f = Gate::eval(lo);                   // < 11p
      const Fe g = fe_mul(f, lo[K - 1]);              // < 2p
      acc[x] = fe_csub(fe_add(acc[x], g), kP2);       // < 2p
    }
  }
#pragma unroll
  for (int x = 0; x < NE; ++x) acc[x] = fe_reduce2(acc[x]);
  block_reduce_store<NE>(acc, partials + (uint64_t)blockIdx.x * NE * 8);
}

// ---- finish a round: sum partials, emit G_i, absorb it, derive alpha_i --------

template <int NE>
__global__ __launch_bounds__(kBlock) void k_finish(const uint32_t* __restrict__ partials, uint32_t nparts,
                                                   Ctrl* ctrl, uint32_t round,
                                                   uint32_t* __restrict__ evals_out,
                                                   uint32_t* __restrict__ alpha_out) {
  Fe s[NE];
#pragma unroll
  for (int x = 0; x < NE; ++x) s[x] = fe_zero();
  for (uint32_t b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int x = 0; x < NE; ++x) s[x] = fe_addmod(s[x], load_words_fe(partials + ((uint64_t)b * NE + x) * 8));
  }
  __shared__ uint32_t tot[NE * 8];
  block_reduce_store<NE>(s, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    // message = T_{i-1} || enc(G_i(0)) || .. || enc(G_i(d+1)), canonical little-endian
    uint32_t msg[8 + NE * 8];
#pragma unroll
    for (int k = 0; k < 8; ++k) msg[k] = ctrl->ts[k];
#pragma unroll
    for (int x = 0; x < NE; ++x) {
      const Fe c = fe_from_mont(load_words_fe(tot + x * 8));
      store_words_fe(msg + 8 + x * 8, c);
#pragma unroll
      for (int k = 0; k < 8; ++k) evals_out[x * 8 + k] = msg[8 + x * 8 + k];
    }
    uint32_t dg[8];
    sha256(msg, 32u * (1u + NE), dg);
    // alpha_i = digest (little-endian 256-bit integer) mod p; digest < 2^256 < 6p
    Fe a = fe_from_words(dg);
    a = fe_csub(fe_csub(fe_csub(a, kP4), kP2), kP);
#pragma unroll
    for (int k = 0; k < 8; ++k) ctrl->ts[k] = dg[k];
    store_words_fe(alpha_out, a);
    store_words_fe(ctrl->alpha_m[round - 1], fe_to_mont(a));
    ctrl->round_done = round;
  }
}

// ---- setup: r to Montgomery, transcript T_0, eq half tables --------------------

// One block.  T_0 = SHA-256("ZCv1" || u32 mu || u32 gate || u32 m || enc(r_1..r_mu)).
__global__ __launch_bounds__(64) void k_setup(const uint32_t* __restrict__ r, uint32_t mu, uint32_t gate,
                                              uint32_t m, Ctrl* ctrl) {
  __shared__ uint32_t msg[4 + kMuMax * 8];
  if (threadIdx.x == 0) {
    msg[0] = 0x3176435au;  // bytes 'Z' 'C' 'v' '1'
    msg[1] = mu;
    msg[2] = gate;
    msg[3] = m;
    ctrl->err = 0;
    ctrl->round_done = 0;
    ctrl->fold_done = 0;
  }
  __syncthreads();  // the reset above must precede any error flagged below
  for (uint32_t i = threadIdx.x; i < mu; i += blockDim.x) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      w[k] = r[i * 8 + k];
      msg[4 + i * 8 + k] = w[k];
    }
    if (!words_lt_p(w)) set_error(ctrl, -4);
    store_words_fe(ctrl->r_m[i], fe_to_mont(fe_from_words(w)));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t dg[8];
    sha256(msg, 16u + 32u * mu, dg);
#pragma unroll
    for (int k = 0; k < 8; ++k) ctrl->ts[k] = dg[k];
  }
}

// Half tables of eq: hi[y] over x_1..x_hb (y's MSB = x_1), lo[z] over
// x_{hb+1}..x_mu.  Entry = product of (x ? r_i : 1 - r_i).  Stored as 8 words.
__global__ __launch_bounds__(kBlock) void k_eq_half(const Ctrl* __restrict__ ctrl, uint32_t mu, uint32_t hb,
                                                    uint32_t* __restrict__ hi, uint32_t* __restrict__ lo) {
  const uint32_t lb = mu - hb;
  const uint32_t nhi = 1u << hb, nlo = 1u << lb;
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nhi + nlo) return;
  const bool is_hi = e < nhi;
  const uint32_t y = is_hi ? e : e - nhi;
  const uint32_t nb = is_hi ? hb : lb;
  const uint32_t first = is_hi ? 0 : hb;
  const Fe one = fe_const(kOne);
  Fe acc = one;
  for (uint32_t k = 0; k < nb; ++k) {
    const Fe ri = load_words_fe(ctrl->r_m[first + k]);
    const uint32_t bit = (y >> (nb - 1 - k)) & 1u;
    const Fe fac = bit ? ri : fe_submod(one, ri);
    acc = fe_reduce2(fe_mul(acc, fac));
  }
  store_words_fe((is_hi ? hi + (uint64_t)y * 8 : lo + (uint64_t)y * 8), acc);
}

// eq[b] = hi[b >> lb] * lo[b & (2^lb - 1)], limb-planar with pitch n.
__global__ __launch_bounds__(kBlock) void k_build_eq(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo,
                                                     uint32_t lb, uint64_t n, uint32_t* __restrict__ eq) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += stride) {
    const Fe h = load_words_fe(hi + (b >> lb) * 8);
    const Fe l = load_words_fe(lo + (b & ((1ull << lb) - 1)) * 8);
    store_el(eq, n, b, fe_reduce2(fe_mul(h, l)));
  }
}

// ---- folds -----------------------------------------------------------------------

// In-place fold of every table with alpha_round: t[j] <- t[j] + alpha (t[j+h] - t[j]),
// j < h.  blockIdx.y selects the table.  With check_state the fold runs only
// when round `round` has been evaluated and not yet folded.
__global__ __launch_bounds__(kBlock) void k_fold(TabPtrs tabs, uint32_t ntab, uint64_t pitch, uint64_t h,
                                                 Ctrl* ctrl, uint32_t round) {
  if (ctrl->round_done != round || ctrl->fold_done + 1 != round) return;
  const uint32_t t = blockIdx.y;
  if (t >= ntab) return;
  const Fe alpha = load_words_fe(ctrl->alpha_m[round - 1]);
  uint32_t* base = tabs.p[t];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < h; j += stride) {
    const Fe a0 = load_el(base, pitch, j);
    const Fe a1 = load_el(base, pitch, j + h);
    store_el(base, pitch, j, fe_addmod(a0, fe_reduce2(fe_mul(alpha, fe_submod(a1, a0)))));
  }
}

// Marks round `round` folded (launched after k_fold on the same stream).
__global__ void k_mark_folded(Ctrl* ctrl, uint32_t round) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (ctrl->round_done == round && ctrl->fold_done + 1 == round)
      ctrl->fold_done = round;
    else
      set_error(ctrl, -5);
  }
}

// Checks that round `round` may be evaluated now (stepping API).
__global__ void k_check_round(Ctrl* ctrl, uint32_t round) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (!(ctrl->round_done == round - 1 && ctrl->fold_done == round - 1)) set_error(ctrl, -5);
  }
}

// Last fold of a whole proof: every table holds 2 entries; write the folded
// value of each, canonical, to openings[t].
__global__ void k_openings(TabPtrs tabs, uint32_t ntab, uint64_t pitch, const Ctrl* __restrict__ ctrl,
                           uint32_t mu, uint32_t* __restrict__ openings) {
  const uint32_t t = threadIdx.x;
  if (t >= ntab) return;
  const Fe alpha = load_words_fe(ctrl->alpha_m[mu - 1]);
  const Fe a0 = load_el(tabs.p[t], pitch, 0);
  const Fe a1 = load_el(tabs.p[t], pitch, 1);
  const Fe u = fe_addmod(a0, fe_reduce2(fe_mul(alpha, fe_submod(a1, a0))));
  store_words_fe(openings + t * 8, fe_from_mont(u));
}

// ---- layout conversion ----------------------------------------------------------

// canonical u32[n][8] -> Montgomery limb-planar u32[8][pitch]; flags inputs >= p.
__global__ __launch_bounds__(kBlock) void k_pack(const uint32_t* __restrict__ canon, uint32_t* __restrict__ planar,
                                                 uint64_t n, uint64_t pitch, Ctrl* ctrl) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    const uint4* src = reinterpret_cast<const uint4*>(canon + j * 8);
    const uint4 x0 = src[0], x1 = src[1];
    uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    if (!words_lt_p(w)) set_error(ctrl, -4);
    store_el(planar, pitch, j, fe_to_mont(fe_from_words(w)));
  }
}

// Montgomery limb-planar (pitch) -> canonical u32[n][8].
__global__ __launch_bounds__(kBlock) void k_unpack(const uint32_t* __restrict__ planar, uint64_t pitch,
                                                   uint32_t* __restrict__ canon, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    uint32_t w[8];
    fe_to_words(fe_from_mont(load_el(planar, pitch, j)), w);
    uint4* dst = reinterpret_cast<uint4*>(canon + j * 8);
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
}

}  // namespace zc
