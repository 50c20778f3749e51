// Setup, eq, fold, layout-conversion and state-check kernels (launched by
// the host API only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zc_device.h"

namespace zc {

// ---- setup: r to Montgomery, eq half tables ---------------------------------------

// One block: resets the control block, checks r and converts it to Montgomery
// form.  (T_0 is hashed by an extra block of the first round kernel.)
__global__ __launch_bounds__(64) void k_setup(const uint32_t* __restrict__ r, uint32_t mu, Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->err = 0;
    ctrl->round_done = 0;
    ctrl->fold_done = 0;
    ctrl->counter = 0;
  }
  __syncthreads();  // the reset above must precede any error flagged below
  for (uint32_t i = threadIdx.x; i < mu; i += blockDim.x) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = r[i * 8 + k];
    if (!words_lt_p(w)) set_error(ctrl, -4);
    store_words_fe(ctrl->r_m[i], fe_to_mont(fe_from_words(w)));
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
