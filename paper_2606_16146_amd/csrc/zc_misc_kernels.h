// Setup, eq, fold, layout-conversion and state-check kernels (launched by
// the host API only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zc_device.h"
#include "zc_t0.h"

namespace zc {

// ---- setup: r, the factored eq tables, round-1 coefficients -------------------------

// lam_k = (-1)^(d-k) C(d+1, k) in Montgomery form (d <= 10): the weight of
// H(k) in H(d+1) = sum_{k<=d} lam_k H(k), exact for H of degree <= d.
__device__ __forceinline__ Fe lam_mont(uint32_t d, uint32_t k) {
  uint32_t c = 1;  // C(d+1, k) <= 462
  for (uint32_t t = 0; t < k; ++t) c = c * (d + 1 - t) / (t + 1);
  Fe v = fe_zero();
  v.l[0] = c;
  v = fe_to_mont(v);
  if ((d - k) & 1u) v = fe_submod(fe_zero(), v);
  return v;
}

// One block: resets the control block, checks r, fills the eq1 rows of
// every round and leaves the state of round 1: C_1 = 1 and no alpha_0, i.e.
// nu[l] = eq1(x, r_1) (slot l), nv = 0, npr = R, nqr = 0.  (T_0 is hashed
// by t0_body, in another block of the same launch.)
__device__ __forceinline__ void setup_body(const uint32_t* __restrict__ r, uint32_t mu, uint32_t ne, Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->err = 0;
    ctrl->round_done = 0;
    ctrl->fold_done = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) __hip_atomic_store(&ctrl->mbox[k], (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    store_words_fe(ctrl->npr, fe_const(kOne));
    store_words_fe(ctrl->nqr, fe_zero());
  }
  __syncthreads();  // the reset above must precede any error flagged below
  for (uint32_t i = threadIdx.x; i < mu; i += blockDim.x) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = r[i * 8 + k];
    if (!words_lt_p(w)) set_error(ctrl, -4);
  }
  // eq1 rows (see Eq1Row).  The slot-l factor of a challenge r (l < nc) is
  // eq1(x, r) = (1 - r) + x (2 r - 1), x = l < ne, else x = d+1 times
  // lam_{l-ne}.  Row i takes 1 - r and 2 r - 1 from r_{i+1} and the slot
  // factors from r_{i+2}; the slot factors of r_1 are coef_1 (C_1 = 1).
  const uint32_t nc = 2 * ne - 1, d = ne - 2, ns = nc + 2;
  Eq1Row* rows = eq1_rows(ctrl);
  auto rval = [&](uint32_t i) {  // r_{i+1}, canonical (a value >= p, flagged above, as 0)
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = r[i * 8 + k];
    return words_lt_p(w) ? fe_from_words(w) : fe_zero();
  };
  Fe one = fe_zero();
  one.l[0] = 1;
  auto slot = [&](const Fe& rc, uint32_t l) {  // the slot-l factor of rc, canonical
    const Fe omr = fe_submod(one, rc), step = fe_submod(fe_addmod(rc, rc), one);
    const uint32_t x = l < ne ? l : d + 1;
    Fe e = fe_addmod(omr, fe_reduce32(fe_mul_small(step, x)));
    if (l >= ne) e = fe_reduce2(fe_mul(e, lam_mont(d, l - ne)));
    return e;
  };
  for (uint32_t idx = threadIdx.x; idx < mu * ns; idx += blockDim.x) {
    const uint32_t i = idx / ns, l = idx % ns;
    const Fe rc = rval(i);
    const Fe omr_m = fe_to_mont(fe_submod(one, rc)), tr_m = fe_to_mont(fe_submod(fe_addmod(rc, rc), one));
    if (l < nc) {
      Fe u = fe_zero(), v = fe_zero();
      if (i + 1 < mu) {
        const Fe e = slot(rval(i + 1), l);
        u = fe_reduce2(fe_mul(omr_m, e));             // (1 - r) e
        v = fe_reduce2(fe_mul(tr_m, fe_to_mont(e)));  // (2 r - 1) e R
      }
      store_words_fe(rows[i].u[l], u);
      store_words_fe(rows[i].v[l], v);
      if (i == 0) {
        store_words_fe(ctrl->nu[l], slot(rc, l));
        store_words_fe(ctrl->nv[l], fe_zero());
      }
    } else if (l == nc) {
      store_words_fe(rows[i].omr, omr_m);
    } else {
      store_words_fe(rows[i].tr2, fe_to_mont(tr_m));
    }
  }
}


// Rows of the factored eq tables (see EqTabs): LO (2^ml rows), the HI heap
// (2^mh rows, row 0 unused) and the SUF heap (2^(ml+1) rows, row 0 unused),
// concatenated in that order.  A row holding a table of nb variables whose
// last variable is v is prod_k (bit ? r : 1 - r) over variables v-nb+1..v,
// the most significant bit of the row index within the table being the
// first of them.
//
// The factors are read from the caller's canonical r (a value >= p, flagged by
// setup_body, is taken as 0); starting from R^(nb+1) each Montgomery product
// with a canonical factor keeps the row in Montgomery form.
__device__ __forceinline__ void eq_row_body(const uint32_t* __restrict__ r, uint32_t mu, uint32_t ml,
                                            uint32_t* __restrict__ rows, uint32_t e) {
  const uint32_t mh = mu - ml;
  const uint32_t nlo = 1u << ml, nhi = 1u << mh, nsuf = 2u << ml;
  if (e >= nlo + nhi + nsuf) return;
  uint32_t y, nb, last;
  if (e < nlo) {
    y = e;
    nb = ml;
    last = mu;
  } else if (e < nlo + nhi) {
    const uint32_t hrow = e - nlo;
    if (hrow == 0) return;
    nb = 31u - __builtin_clz(hrow);  // table of 2^nb rows at [2^nb, 2^(nb+1))
    y = hrow - (1u << nb);
    last = mh;
  } else {
    const uint32_t srow = e - nlo - nhi;
    if (srow == 0) return;
    nb = 31u - __builtin_clz(srow);
    y = srow - (1u << nb);
    last = mu;
  }
  Fe acc = fe_zero();
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if ((uint32_t)k == nb) acc = fe_const(kRPow.v[k]);  // nb <= 15 (mu <= 30)
  Fe one = fe_zero();
  one.l[0] = 1;
  for (uint32_t k = 0; k < nb; ++k) {
    uint32_t w[8];
    const uint32_t* rw = r + (uint64_t)(last - nb + k) * 8;  // variable last-nb+1+k (1-based)
#pragma unroll
    for (int t = 0; t < 8; ++t) w[t] = rw[t];
    const Fe ri = words_lt_p(w) ? fe_from_words(w) : fe_zero();
    const uint32_t bit = (y >> (nb - 1 - k)) & 1u;
    acc = fe_reduce2(fe_mul(acc, bit ? ri : fe_submod(one, ri)));
  }
  store_words_fe(rows + (uint64_t)e * 8, acc);
}

// The setup of a proof in one launch: block 0 runs setup_body, the last
// block hashes T_0 and the blocks between build the eq rows (each part needs
// r only, so they overlap).
__global__ __launch_bounds__(kBlock) void k_setup_eq(Ctrl* __restrict__ ctrl, const uint32_t* __restrict__ r,
                                                     uint32_t mu, uint32_t gate, uint32_t m, uint32_t ml, uint32_t ne,
                                                     uint32_t* __restrict__ rows) {
  if (blockIdx.x == 0) {
    setup_body(r, mu, ne, ctrl);
  } else if (blockIdx.x == gridDim.x - 1) {
    t0_body(r, mu, gate, m, ctrl);
  } else {
    eq_row_body(r, mu, ml, rows, (blockIdx.x - 1) * blockDim.x + threadIdx.x);
  }
}

// ---- folds -----------------------------------------------------------------------

// In-place fold of every witness table with alpha_round:
// t[j] <- t[j] + alpha (t[j+h] - t[j]), j < h.  blockIdx.y selects the table.
// The fold runs only when round `round` has been evaluated and not yet folded.
__global__ __launch_bounds__(kBlock) void k_fold(TabPtrs tabs, uint32_t ntab, uint64_t pitch, uint64_t h,
                                                 Ctrl* ctrl, uint32_t round) {
  if (ctrl->round_done != round || ctrl->fold_done + 1 != round) return;
  const uint32_t t = blockIdx.y;
  if (t >= ntab) return;
  const Fe alpha = fe_to_mont(load_words_fe(ctrl->alpha[round - 1]));
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
