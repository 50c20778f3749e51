// Kernels of the ZeroCheck SumCheck prover (gfx950).
//
// What is computed follows the multilinear ZeroCheck of Fig. 2 (right) of
// "When Proofs Meet Hardware": for each round i evaluate
// G_i(X) = sum over the remaining hypercube of f_M(ext(X)) * eq_r(ext(X)) at
// X = 0..d+1, derive alpha_i from the transcript, and fold every table with
// alpha_i (Sec. 4.1: update, extend, multiply, accumulate).  Variable x_1 is
// the most significant index bit, so round i pairs entries j and
// j + 2^(mu-i), and the fold of a table can be written in place: the thread
// that owns pair j reads and writes only slots j, j+q, j+2q, j+3q.
//
// eq_r is used in factored form (Sec. 3.3 defines it as a product of one
// factor per variable): G_i(X) = C_i eq1(X, r_i) H_i(X) with
// H_i(X) = sum_j E_i[j] f_M(ext_j(X)), E_i the eq table of the variables
// after x_i and C_i the product of the factors already bound to challenges.
// H_i has degree d, so each pair contributes at X = 0..d only, and the last
// value H_i(d+1) is extrapolated once per round.  E_i[j] is one product of
// two tables of about 2^(mu/2) entries (or a lookup for small rounds), so no
// 2^mu-entry eq table is built, streamed or folded.  The values sent are the
// same field elements as with the materialized table.
//
// Value bounds (the field code's contract is a product of inputs < A*p and
// < B*p with A*B <= 128 lands below 2p):
// * every table entry in memory is fully reduced, < p;
// * Delta = u1 - u0 mod p is < p, so the extension e(X) = u0 + X*Delta built
//   by plain additions is < (X+1) p <= (d+1) p <= 10 p;
// * gate values are kept below 12 p before the product with E (< p);
// * per-thread sums of products stay below 2p.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "zc_device.h"
#include "zc_launch.h"

namespace zc {

// ---- compile-time unrolling ------------------------------------------------------

template <int I, int N>
struct Unroll {
  template <class F>
  __device__ __forceinline__ static void run(F& f) {
    f(std::integral_constant<int, I>{});
    Unroll<I + 1, N>::run(f);
  }
};
template <int N>
struct Unroll<N, N> {
  template <class F>
  __device__ __forceinline__ static void run(F&) {}
};

// lo + N dl by N additions: the extension at the first evaluated point when
// the points below N are skipped (the same additions as stepping up to it).
template <int N>
__device__ __forceinline__ Fe ext_at(Fe lo, const Fe& dl) {
#pragma unroll
  for (int i = 0; i < N; ++i) lo = fe_add(lo, dl);
  return lo;
}

// Converts a loaded pair to (lo, dl) = (t[j], t[j+q] - t[j] mod p).
__device__ __forceinline__ void cvt_pair(const RawPair& r, Fe& lo, Fe& dl) {
  lo = fe_from_words(r.w0);
  dl = fe_submod(fe_from_words(r.w1), lo);
}

// The same with a lazy difference dl = t[j+q] + p - t[j] < 2p (not reduced).
// An extension lo + X dl = (1 - X) t[j] + X t[j+q] + X p is then < p at X = 0
// and < 2X p for X >= 1.
__device__ __forceinline__ void cvt_pair_lazy(const RawPair& r, Fe& lo, Fe& dl) {
  lo = fe_from_words(r.w0);
  dl = fe_sub_plus(fe_from_words(r.w1), lo, kP);
}

constexpr L9 kP11 = detail::mul_small(kP, 11);
constexpr L9 kP18 = detail::mul_small(kP, 18);

// ---- the factored eq table --------------------------------------------------------
//
// mu variables split into mh high and ml = floor(mu/2) low ones.  For round
// i < mh, E_i[j] = HI_i[j >> ml] * LO[j mod 2^ml] with HI_i the eq table of
// variables i+1..mh and LO that of mh+1..mu; for i >= mh, E_i = SUF_i, the
// eq table of variables i+1..mu.  HI_i (2^(mh-i) entries) and SUF_i
// (2^(mu-i) entries) are stored heap-style: a table of s entries at rows
// [s, 2s).  Rows are 8 words, Montgomery form, < p.
struct EqTabs {
  const uint32_t* lo;
  const uint32_t* hi;
  const uint32_t* suf;
  uint32_t ml, mh, mu;
};

__device__ __forceinline__ Fe load_row(const uint32_t* __restrict__ tab, uint32_t row) {
  const uint4* p = reinterpret_cast<const uint4*>(tab + (uint64_t)row * 8);
  const uint4 x0 = p[0], x1 = p[1];
  const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
  return fe_from_words(w);
}

// The rows behind E_i[j], loaded but not yet multiplied, so that their
// latency overlaps the table loads of the pair.
struct EqRows {
  uint4 h0, h1, l0, l1;
  bool split;
};

__device__ __forceinline__ EqRows issue_eq(const EqTabs& E, uint32_t round, uint32_t j) {
  EqRows r;
  r.split = round < E.mh;
  const uint32_t hrow = r.split ? (1u << (E.mh - round)) + (j >> E.ml) : 0u;
  const uint32_t lrow = r.split ? (j & ((1u << E.ml) - 1u)) : (1u << (E.mu - round)) + j;
  const uint4* hp = reinterpret_cast<const uint4*>(E.hi + (uint64_t)hrow * 8);
  const uint4* lp = reinterpret_cast<const uint4*>((r.split ? E.lo : E.suf) + (uint64_t)lrow * 8);
  r.l0 = lp[0];
  r.l1 = lp[1];
  if (r.split) {
    r.h0 = hp[0];
    r.h1 = hp[1];
  }
  return r;
}

__device__ __forceinline__ Fe resolve_eq(const EqRows& r) {
  const uint32_t wl[8] = {r.l0.x, r.l0.y, r.l0.z, r.l0.w, r.l1.x, r.l1.y, r.l1.z, r.l1.w};
  const Fe l = fe_from_words(wl);
  if (!r.split) return l;
  const uint32_t wh[8] = {r.h0.x, r.h0.y, r.h0.z, r.h0.w, r.h1.x, r.h1.y, r.h1.z, r.h1.w};
  return fe_reduce2(fe_mul(fe_from_words(wh), l));
}

// E_i[j] for round i (< p).
__device__ __forceinline__ Fe eq_factor(const EqTabs& E, uint32_t round, uint32_t j) {
  if (round < E.mh) {
    const Fe h = load_row(E.hi, (1u << (E.mh - round)) + (j >> E.ml));
    const Fe l = load_row(E.lo, j & ((1u << E.ml) - 1u));
    return fe_reduce2(fe_mul(h, l));
  }
  return load_row(E.suf, (1u << (E.mu - round)) + j);
}

// ---- where a gate reads its pairs -------------------------------------------------
//
// A gate asks for the pair (t[j], t[j+q]) of table t in two steps: issue(t)
// starts the loads, get() turns them into (lo, dl) = (t[j], t[j+q] - t[j]),
// so that the loads of the next table are in flight meanwhile.  getl() gives
// the lazy difference of cvt_pair_lazy (dl < 2p) instead.

// Tables already holding the round's 2q live entries (NT: read them
// non-temporally, for tables read once in the round).
template <bool NT>
struct PairSrcT {
  const TabPtrs& tp;
  uint64_t pitch;
  uint32_t j, q;
  using Raw = RawPair;
  __device__ __forceinline__ Raw issue(int t) const { return issue_pair<NT>(tp.p[t], pitch, j, q); }
  __device__ __forceinline__ void get(const Raw& r, int, Fe& lo, Fe& dl) const { cvt_pair(r, lo, dl); }
  __device__ __forceinline__ void getl(const Raw& r, int, Fe& lo, Fe& dl) const { cvt_pair_lazy(r, lo, dl); }
};
using PairSrc = PairSrcT<false>;

// Tables holding 4q entries, folded on the way with alpha_{i-1}:
// u[j] = t[j] + alpha (t[j+2q] - t[j]), u[j+q] likewise; u is written to the
// destination tables (the next round reads it) and used from registers.
// Loads and stores are non-temporal.
struct FoldSrc {
  const TabPtrs& src;
  const TabPtrs& dst;
  uint64_t sp, dp;
  uint32_t j, q;
  Fe alpha;
  bool st = true;  // store the folded pair (a second wave folding the same pairs does not)
  struct Raw {
    RawPair lo2, hi2;  // (t[j], t[j+q]), (t[j+2q], t[j+3q])
  };
  __device__ __forceinline__ Raw issue(int t) const {
    return Raw{issue_pair<true>(src.p[t], sp, j, q), issue_pair<true>(src.p[t], sp, j + 2 * q, q)};
  }
  __device__ __forceinline__ void fold(const Raw& r, int t, Fe& u0, Fe& u1) const {
    u0 = fe_lerp(fe_from_words(r.lo2.w0), fe_from_words(r.hi2.w0), alpha);
    u1 = fe_lerp(fe_from_words(r.lo2.w1), fe_from_words(r.hi2.w1), alpha);
    if (st) {
      store_el<true>(dst.p[t], dp, j, u0);
      store_el<true>(dst.p[t], dp, j + q, u1);
    }
  }
  __device__ __forceinline__ void get(const Raw& r, int t, Fe& lo, Fe& dl) const {
    Fe u1;
    fold(r, t, lo, u1);
    dl = fe_submod(u1, lo);
  }
  __device__ __forceinline__ void getl(const Raw& r, int t, Fe& lo, Fe& dl) const {
    Fe u1;
    fold(r, t, lo, u1);
    dl = fe_sub_plus(u1, lo, kP);
  }
};

// ---- gates ---------------------------------------------------------------------
//
// eval() adds E * f_M(ext(X)) for X = 0..NH-1 (NH = d+1) of one pair to
// acc[X]; the addend is < 2p and acc is not reduced (round_body reduces it
// every kLazyPairs pairs).  The extension of a table at X is e(X) = lo + X*dl,
// built by plain additions: e(X) < (X+1) p with strict differences (get),
// e(X) < 2X p (X >= 1) with lazy ones (getl).  The NH products of one step
// are independent of each other, which keeps the multiply pipeline busy, and
// the loads of the next table are issued before the current step's products
// so that their latency is hidden.

// f = qM*a*b + qL*a + qR*b + qO*c + qC, columns [a b c qM qL qR qO qC], degree 3,
// evaluated as a*(qM*b + qL) + qR*b + qO*c + qC: per point one product and one
// sum of three products (fe_sop), then the product with E.
struct GateVanilla {
  static constexpr int K = 8;
  // fold in a loop of its own: inlining the 16 fold products into the
  // unrolled gate makes the round-2 kernel slower (measured)
  static constexpr bool kFoldInGate = false;
  static constexpr int D = 3;
  static constexpr int NH = D + 1;
  static constexpr int NE = D + 2;
  // f_M at one point from the witness extensions e[0..7] (< 5p); result < 11p.
  __device__ static __forceinline__ Fe point(const Fe* e) {
    const Fe t1 = fe_mul(e[3], e[1]);                 // qM*b < 2p
    const Fe t3 = fe_mul(e[0], fe_add(t1, e[4]));     // a*(qM*b + qL) < 2p (5*7)
    const Fe t4 = fe_mul(e[5], e[1]);                 // qR*b < 2p
    const Fe t5 = fe_mul(e[6], e[2]);                 // qO*c < 2p
    return fe_add(fe_add(fe_add(t3, t4), t5), e[7]);  // < 11p
  }
  // X0 = 2: only the points X >= 2 (round 1 under ZC_FLAG_ASSUME_SATISFIED)
  template <class Src, int X0 = 0, int XE = NH>
  __device__ static __forceinline__ void eval(const Src& src, const EqRows& er, Fe (&acc)[NH]) {
    // lazy differences: every extension at X <= 3 is < 6p
    Fe bx[NH], s[NH], lo, dl, e;
    typename Src::Raw rb = src.issue(1);   // b
    typename Src::Raw rm = src.issue(3);   // qM
    typename Src::Raw rl = src.issue(4);   // qL
    src.getl(rb, 1, lo, dl);
    typename Src::Raw ra = src.issue(0);   // a
    typename Src::Raw rr = src.issue(5);   // qR
    auto fb = [&](auto x) __attribute__((always_inline)) {
      bx[x] = (x == X0) ? ext_at<X0>(lo, dl) : fe_add(bx[x > X0 ? x - 1 : X0], dl);
    };
    Unroll<X0, XE>::run(fb);
    src.getl(rm, 3, lo, dl);  // qM
    typename Src::Raw ro = src.issue(6);   // qO
    typename Src::Raw rc = src.issue(2);   // c
    e = ext_at<X0>(lo, dl);
    auto f1 = [&](auto x) __attribute__((always_inline)) {
      s[x] = fe_mul(e, bx[x]);  // < 2p (6*6)
      e = fe_add(e, dl);
    };
    Unroll<X0, XE>::run(f1);
    src.getl(rl, 4, lo, dl);  // qL
    typename Src::Raw rq = src.issue(7);   // qC
    e = ext_at<X0>(lo, dl);
    auto f2 = [&](auto x) __attribute__((always_inline)) {
      s[x] = fe_add(s[x], e);  // < 8p
      e = fe_add(e, dl);
    };
    Unroll<X0, XE>::run(f2);
    Fe ea, da, er5, dr5, eo, dlo, ec, dc;
    src.getl(ra, 0, ea, da);    // a
    src.getl(rr, 5, er5, dr5);  // qR
    src.getl(ro, 6, eo, dlo);   // qO
    src.getl(rc, 2, ec, dc);    // c
    ea = ext_at<X0>(ea, da);
    er5 = ext_at<X0>(er5, dr5);
    eo = ext_at<X0>(eo, dlo);
    ec = ext_at<X0>(ec, dc);
    auto f3 = [&](auto x) __attribute__((always_inline)) {
      const Fe fa[3] = {ea, er5, eo};
      const Fe fb2[3] = {s[x], bx[x], ec};
      s[x] = fe_sop<3>(fa, fb2);  // a s + qR b + qO c < 2p (6*8 + 6*6 + 6*6 = 120)
      ea = fe_add(ea, da);
      er5 = fe_add(er5, dr5);
      eo = fe_add(eo, dlo);
      ec = fe_add(ec, dc);
    };
    Unroll<X0, XE>::run(f3);
    src.getl(rq, 7, lo, dl);  // qC
    const Fe E = resolve_eq(er);
    e = ext_at<X0>(lo, dl);
    auto f6 = [&](auto x) __attribute__((always_inline)) {
      const Fe f = fe_add(s[x], e);           // < 8p
      acc[x] = fe_add(acc[x], fe_mul(f, E));  // product < 2p (8*1)
      e = fe_add(e, dl);
    };
    Unroll<X0, XE>::run(f6);
  }
  // The two waves of a two-wave round (round_body HALF) split the terms of
  // f_M, each at every point: H = 0 adds E a (qM b + qL), H = 1 adds
  // E (qR b + qO c + qC); the two sums of a point add up to the same field
  // element.  Both fold on the way (FoldSrc): H = 0 stores a, b, qM, qL,
  // H = 1 stores c, qR, qO, qC and reads b through `nb`, which does not store.
  template <int H, class Src>
  __device__ static __forceinline__ void eval_terms(const Src& src, const Src& nb, const EqRows& er, Fe (&acc)[NH]) {
    if constexpr (H == 0) {
      Fe bx[NH], s[NH], lo, dl, e;
      typename Src::Raw rb = src.issue(1);  // b
      typename Src::Raw rm = src.issue(3);  // qM
      src.getl(rb, 1, lo, dl);
      typename Src::Raw rl = src.issue(4);  // qL
      auto fb = [&](auto x) __attribute__((always_inline)) { bx[x] = x == 0 ? lo : fe_add(bx[x > 0 ? x - 1 : 0], dl); };
      Unroll<0, NH>::run(fb);
      src.getl(rm, 3, lo, dl);
      typename Src::Raw ra = src.issue(0);  // a
      e = lo;
      auto f1 = [&](auto x) __attribute__((always_inline)) {
        s[x] = fe_mul(e, bx[x]);  // < 2p (6*6)
        e = fe_add(e, dl);
      };
      Unroll<0, NH>::run(f1);
      src.getl(rl, 4, lo, dl);
      e = lo;
      auto f2 = [&](auto x) __attribute__((always_inline)) {
        s[x] = fe_add(s[x], e);  // < 8p
        e = fe_add(e, dl);
      };
      Unroll<0, NH>::run(f2);
      src.getl(ra, 0, lo, dl);
      // E a(X) = E a[lo] + X E a[dl], both products < p: extensions < 4p
      const Fe E = resolve_eq(er);
      Fe ea = fe_reduce2(fe_mul(E, lo));
      const Fe da = fe_reduce2(fe_mul(E, dl));  // (1*2)
      auto f3 = [&](auto x) __attribute__((always_inline)) {
        acc[x] = fe_add(acc[x], fe_mul(ea, s[x]));  // product < 2p (4*8)
        ea = fe_add(ea, da);
      };
      Unroll<0, NH>::run(f3);
    } else {
      Fe lb, db, lr, dr, lo, dO, lc, dc, lq, dq;
      typename Src::Raw rb = nb.issue(1);   // b
      typename Src::Raw rr = src.issue(5);  // qR
      nb.getl(rb, 1, lb, db);
      typename Src::Raw ro = src.issue(6);  // qO
      src.getl(rr, 5, lr, dr);
      typename Src::Raw rc = src.issue(2);  // c
      src.getl(ro, 6, lo, dO);
      typename Src::Raw rq = src.issue(7);  // qC
      src.getl(rc, 2, lc, dc);
      src.getl(rq, 7, lq, dq);
      const Fe E = resolve_eq(er);
      auto f4 = [&](auto x) __attribute__((always_inline)) {
        const Fe fa[2] = {lr, lo};
        const Fe fb2[2] = {lb, lc};
        const Fe u = fe_add(fe_sop<2>(fa, fb2), lq);  // qR b + qO c < 2p (6*6 + 6*6), + qC < 8p
        acc[x] = fe_add(acc[x], fe_mul(u, E));       // product < 2p (8*1)
        lr = fe_add(lr, dr);
        lo = fe_add(lo, dO);
        lb = fe_add(lb, db);
        lc = fe_add(lc, dc);
        lq = fe_add(lq, dq);
      };
      Unroll<0, NH>::run(f4);
    }
  }
};

// f = s*w1*...*wm - o, columns [s w1 .. wm o], degree m+1.
template <int M>
struct GateProd {
  static constexpr int K = M + 2;
  static constexpr bool kFoldInGate = true;  // the gate's table loop is rolled
  static constexpr int D = M + 1;
  static constexpr int NH = D + 1;
  static constexpr int NE = D + 2;
  // f_M at one point from the witness extensions e[0..K-1] (< 11p); result < 8p.
  __device__ static __forceinline__ Fe point(const Fe* e) {
    Fe prod = fe_mul(e[0], e[1]);  // < 2p (11*11)
    auto f = [&](auto k) __attribute__((always_inline)) { prod = fe_mul(prod, e[k]); };  // < 2p (2*11)
    Unroll<2, M + 1>::run(f);
    return fe_csub(fe_sub_plus(prod, e[M + 1], kP11), kP8);
  }
  // From m = 3 on (NH >= 5 points), E multiplies s's pair (2 products)
  // instead of every point's value (NH products), and o's part of the sum,
  // sum_j E_j o_j(X) = sum_j E_j o_j[lo] + X sum_j E_j o_j[dl], is kept as
  // two extra sums (2 products) that finalize() subtracts once per thread.
  // The field elements summed are the same.
  static constexpr bool kEqInS = M >= 3;
  static constexpr int kExtraAcc = kEqInS ? 2 : 0;
  template <int NA, int X0 = 0, int XE = NH>
  __device__ static __forceinline__ void finalize(Fe (&acc)[NA]) {
    if constexpr (kEqInS) {
      // acc[x] -= acc[NH] + x acc[NH+1]  (all < p: the sums were reduced)
      auto f = [&](auto x) __attribute__((always_inline)) {
        const Fe t = fe_reduce32(fe_add(acc[NH], fe_mul_small(acc[NH + 1], (uint32_t)x)));  // < p + 10p
        acc[x] = fe_submod(acc[x], t);
      };
      Unroll<X0, XE>::run(f);
    }
  }
  template <class Src, int NA, int X0 = 0, int XE = NH>
  __device__ static __forceinline__ void eval(const Src& src, const EqRows& er, Fe (&acc)[NA]) {
    // s and w1 with strict differences (extensions at X <= m+1 < (m+2) p <= 10p,
    // so their product fits: 10*10), the other tables lazy (< 2(m+1) p <= 18p)
    Fe pr[NH], lo, dl, e;
    typename Src::Raw cur = src.issue(0);  // s
    typename Src::Raw nxt = src.issue(1);  // w1
    src.get(cur, 0, lo, dl);
    Fe E;
    if constexpr (kEqInS) {
      // E s(X) = E s[lo] + X E s[dl], each product < p (mont), so the
      // extensions keep the strict bound (X + 1) p
      E = resolve_eq(er);
      lo = fe_reduce2(fe_mul(E, lo));
      dl = fe_reduce2(fe_mul(E, dl));
    }
    auto f0 = [&](auto x) __attribute__((always_inline)) {
      pr[x] = (x == X0) ? ext_at<X0>(lo, dl) : fe_add(pr[x > X0 ? x - 1 : X0], dl);
    };
    Unroll<X0, XE>::run(f0);
#pragma unroll 1
    for (int k = 1; k <= M; ++k) {  // pr *= w_k  (< 2p after each product: 10*10, then 2*18)
      cur = nxt;
      nxt = src.issue(k + 1);  // w_{k+1}, or o after the last w
      if (k == 1)
        src.get(cur, k, lo, dl);
      else
        src.getl(cur, k, lo, dl);
      e = ext_at<X0>(lo, dl);
      auto fk = [&](auto x) __attribute__((always_inline)) {
        pr[x] = fe_mul(pr[x], e);
        e = fe_add(e, dl);
      };
      Unroll<X0, XE>::run(fk);
    }
    src.getl(nxt, M + 1, lo, dl);  // o (< 18p): pr + 18p - o < 20p
    if constexpr (kEqInS) {
      auto fe = [&](auto x) __attribute__((always_inline)) { acc[x] = fe_add(acc[x], pr[x]); };  // pr < 2p
      Unroll<X0, XE>::run(fe);
      acc[NH] = fe_add(acc[NH], fe_reduce2(fe_mul(E, lo)));          // < p (o[lo] < p)
      acc[NH + 1] = fe_add(acc[NH + 1], fe_reduce2(fe_mul(E, dl)));  // < p (1*2 <= 128, then reduced)
    } else {
      E = resolve_eq(er);
      e = ext_at<X0>(lo, dl);
      auto fo = [&](auto x) __attribute__((always_inline)) {
        const Fe f = fe_sub_plus(pr[x], e, kP18);
        acc[x] = fe_add(acc[x], fe_mul(f, E));  // product < 2p (20*1)
        e = fe_add(e, dl);
      };
      Unroll<X0, XE>::run(fo);
    }
  }
};

// f = g1*...*gP + gP+1 + ... + gP+A, the polynomials of Table 1 (degree P,
// P + A unique polynomials, A + 1 additive terms), columns [g1 .. gP+A].
template <int P, int A>
struct GateSum {
  static_assert(P >= 2 && P <= 4 && A >= 0 && A <= 3, "Table 1 shapes");
  static constexpr int K = P + A;
  static constexpr bool kFoldInGate = true;
  static constexpr int D = P;
  static constexpr int NH = D + 1;
  static constexpr int NE = D + 2;
  // f_M at one point from the extensions e[0..K-1] (< 5p); result < 17p.
  __device__ static __forceinline__ Fe point(const Fe* e) {
    Fe f = fe_mul(e[0], e[1]);  // < 2p (5*5)
    auto pm = [&](auto k) __attribute__((always_inline)) { f = fe_mul(f, e[k]); };  // < 2p (2*5)
    Unroll<2, P>::run(pm);
    auto ad = [&](auto k) __attribute__((always_inline)) { f = fe_add(f, e[k]); };  // < 2p + 15p
    Unroll<P, K>::run(ad);
    return f;
  }
  template <class Src, int X0 = 0, int XE = NH>
  __device__ static __forceinline__ void eval(const Src& src, const EqRows& er, Fe (&acc)[NH]) {
    // lazy differences: extensions at X <= P are < 2P p <= 8p
    Fe f[NH], lo, dl;
    typename Src::Raw cur = src.issue(0);
    typename Src::Raw nxt = src.issue(1);
    src.getl(cur, 0, lo, dl);
    auto f0 = [&](auto x) __attribute__((always_inline)) {
      f[x] = (x == X0) ? ext_at<X0>(lo, dl) : fe_add(f[x > X0 ? x - 1 : X0], dl);
    };
    Unroll<X0, XE>::run(f0);
    auto step = [&](auto k) __attribute__((always_inline)) {
      cur = nxt;
      if (k + 1 < K) nxt = src.issue(k + 1 < K ? k + 1 : 0);
      src.getl(cur, k, lo, dl);
      Fe e = ext_at<X0>(lo, dl);
      auto px = [&](auto x) __attribute__((always_inline)) {
        if (k < P)
          f[x] = fe_mul(f[x], e);  // < 2p (8*8, then 2*8)
        else
          f[x] = fe_add(f[x], e);  // < 26p after A <= 3 additions
        e = fe_add(e, dl);
      };
      Unroll<X0, XE>::run(px);
    };
    Unroll<1, K>::run(step);
    const Fe E = resolve_eq(er);
    auto fo = [&](auto x) __attribute__((always_inline)) {
      acc[x] = fe_add(acc[x], fe_mul(f[x], E));  // product < 2p (26*1)
    };
    Unroll<X0, XE>::run(fo);
  }
};

// ---- reductions ---------------------------------------------------------------

__device__ __forceinline__ Fe shfl_xor_fe(const Fe& a, int mask) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.l[i] = __shfl_xor(a.l[i], mask, 64);
  return r;
}

__device__ __forceinline__ Fe lds_fe(const uint32_t* p) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.l[i] = p[i];
  return r;
}

__device__ __forceinline__ void lds_put(uint32_t* p, const Fe& a) {
#pragma unroll
  for (int i = 0; i < NL; ++i) p[i] = a.l[i];
}

// Sum (mod p) over the block of NV values per thread (each < p).  Thread x < NV
// returns the block total of value x; other threads return 0.
template <int NV>
__device__ __forceinline__ Fe block_reduce(Fe (&v)[NV]) {
  __shared__ uint32_t red[kBlock / 64][NV][NL];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto f = [&](auto x) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v[x] = fe_addmod(v[x], shfl_xor_fe(v[x], s));
    if (lane == 0) lds_put(red[wave][x], v[x]);
  };
  Unroll<0, NV>::run(f);
  __syncthreads();
  Fe s = fe_zero();
  if (threadIdx.x < NV) {
    const int x = threadIdx.x;
    s = lds_fe(red[0][x]);
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = fe_addmod(s, lds_fe(red[w][x]));
  }
  return s;
}

// ---- the finisher's sum of the round kernel's partial sums -------------------------
//
// A round kernel's block b stores its NV values at partials[b * NVP + x]
// (32-byte elements, NVP = part_stride(NV), the power of two >= NV).  The
// finisher's thread t takes value x = t mod NVP of blocks t / NVP,
// t / NVP + 256 / NVP, ..., so consecutive lanes read consecutive elements,
// each whole (two 16-byte loads), and adds their words into 64-bit
// accumulators (no carries between words until the end).

template <int NV>
struct Gather {
  static constexpr uint32_t NVP = part_stride(NV);
  static constexpr uint32_t BPS = kBlock / NVP;  // blocks per sweep of the block's threads
  uint64_t acc[8];
  // the loads and 64-bit sums of this thread's share
  __device__ __forceinline__ void load(const uint32_t* __restrict__ partials, uint32_t nparts) {
    const uint32_t t = threadIdx.x, x = t % NVP;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0;
    if (x >= (uint32_t)NV) return;
#pragma unroll 4
    for (uint32_t b = t / NVP; b < nparts; b += BPS) {
      const uint4* p = reinterpret_cast<const uint4*>(partials + ((uint64_t)b * NVP + x) * 8);
      const uint4 w0 = p[0], w1 = p[1];
      acc[0] += w0.x;
      acc[1] += w0.y;
      acc[2] += w0.z;
      acc[3] += w0.w;
      acc[4] += w1.x;
      acc[5] += w1.y;
      acc[6] += w1.z;
      acc[7] += w1.w;
    }
  }
  // the block total of value x (< p) into out[x], x < NV; ends with a barrier
  __device__ __forceinline__ void reduce(uint32_t nparts, uint32_t (*out)[NL]) {
    __shared__ uint32_t red[kBlock / 64][NVP][NL];
    const uint32_t t = threadIdx.x, x = t % NVP;
    // the 64-bit word sums -> 9 words -> limbs; the value is below cnt p with
    // cnt = the most terms any thread added (<= 128)
    uint32_t w[9];
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t sk = acc[k] + c;
      w[k] = (uint32_t)sk;
      c = sk >> 32;
    }
    w[8] = (uint32_t)c;
    Fe v = fe_from_words9(w);
    const uint32_t cnt = (nparts + BPS - 1) / BPS;
    if (cnt > 64) v = fe_csub(v, kP64);
    if (cnt > 32) v = fe_csub(v, kP32);
    if (cnt > 16) v = fe_csub(v, kP16);
    if (cnt > 8) v = fe_csub(v, kP8);
    if (cnt > 4) v = fe_csub(v, kP4);
    if (cnt > 2) v = fe_csub(v, kP2);
    if (cnt > 1) v = fe_csub(v, kP);
    // lanes x, x + NVP, ... of the wave, then the block's waves
#pragma unroll
    for (uint32_t msk = NVP; msk < 64; msk <<= 1) v = fe_addmod(v, shfl_xor_fe(v, (int)msk));
    if ((t & 63u) < NVP) lds_put(red[t >> 6][x], v);
    __syncthreads();
    if (t < (uint32_t)NV) {
      Fe s = lds_fe(red[0][t]);
#pragma unroll
      for (int wv = 1; wv < kBlock / 64; ++wv) s = fe_addmod(s, lds_fe(red[wv][t]));
      lds_put(out[t], s);
    }
    __syncthreads();
  }
};

// ---- end of a round ------------------------------------------------------------

// The scalars of one round; the tables travel beside it (TabPtrs), as kernel
// arguments or from a batch descriptor.
struct RoundArgs {
  uint64_t src_pitch, dst_pitch;
  uint64_t q;                  // pairs of the evaluated round
  uint32_t round;              // i (1-based)
  uint32_t mu;
  uint32_t nparts;             // blocks of the round kernel (partial sums to add up)
  uint32_t* partials;          // [nparts][NH][8]
  Ctrl* ctrl;
  uint32_t* evals_out;         // G_i(0..d+1), canonical
  uint32_t* alpha_out;         // alpha_i, canonical
  uint32_t tail;               // 1: the finisher also runs rounds round+1..mu and the openings
  uint32_t* openings;          // tail only: (k+1) x 8 canonical
  EqTabs eq;
  uint32_t check;              // 1: the verifier's claim checks on the device (ZC_FLAG_CHECK_CLAIMS)
  uint32_t share;              // host only: round grids sized for a shared GPU (ZC_FLAG_SHARED_GPU)
  uint32_t signal;             // 1: the finisher also posts alpha_i to the mailbox (k_fin_wait)
  uint32_t skip01;             // host only: round 1 skips X = 0, 1 (ZC_FLAG_ASSUME_SATISFIED)
};

// Montgomery product reduced below p.
__device__ __forceinline__ Fe mont(const Fe& a, const Fe& b) { return fe_reduce2(fe_mul(a, b)); }

// c ? a : b, limb by limb.
__device__ __forceinline__ Fe fe_sel(bool c, const Fe& a, const Fe& b) {
  Fe r;
#pragma unroll
  for (int i = 0; i < NL; ++i) r.l[i] = c ? a.l[i] : b.l[i];
  return r;
}

// The same value, held in vector registers.  A value the compiler can prove
// uniform across the wave (e.g. read from one LDS or control-block address)
// would otherwise be multiplied on the scalar unit, where a 32 x 32 -> 64-bit
// product takes four instructions and the unit is shared by the whole CU.
__device__ __forceinline__ Fe fe_vgpr(Fe a) {
#pragma unroll
  for (int i = 0; i < NL; ++i) asm("" : "+v"(a.l[i]));
  return a;
}

// ---- the verifier's claims, for the optional self-checks ---------------------------

__device__ __forceinline__ bool fe_eq(const Fe& a, const Fe& b) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) o |= a.l[i] ^ b.l[i];
  return o == 0;
}

// sum_k y_k L_k(x) for the polynomial of degree < N whose values at the nodes
// 0..N-1 are y (N canonical elements, 8 words each), at x (canonical): the
// claim G_i(alpha_i) of Sec. 3.4.  One lane; canonical result < p.  L_k(x) =
// w_k prod_{j != k} (x - j) from prefix and suffix products.
template <int N>
__device__ __noinline__ Fe lagrange_at(const uint32_t* y, Fe x) {
  constexpr LagrangeN<N> W{};
  const Fe xm = fe_to_mont(fe_vgpr(x));
  Fe dif[N], pre[N];
#pragma unroll
  for (int k = 0; k < N; ++k) dif[k] = fe_submod(xm, fe_const(W.node[k]));  // (x - k) R
  pre[0] = fe_const(kOne);
#pragma unroll
  for (int k = 1; k < N; ++k) pre[k] = mont(pre[k - 1], dif[k - 1]);
  Fe suf = fe_const(kOne), acc = fe_zero();
#pragma unroll
  for (int k = N - 1; k >= 0; --k) {
    const Fe lk = mont(fe_const(W.w[k]), mont(pre[k], suf));  // L_k(x) R
    acc = fe_addmod(acc, mont(lk, fe_to_mont(load_words_fe(y + 8 * k))));
    suf = mont(suf, dif[k]);
  }
  return fe_from_mont(acc);
}

// ---- the end of a round ---------------------------------------------------------
//
// Round i sends G_i(x) = C_i eq1(x, r_i) H_i(x), x = 0..d+1, where H_i(x)
// (x <= d) are the block sums and H_i(d+1) = sum_k lam_k H_i(k).  The
// coefficients coef_i[x] = C_i eq1(x, r_i) (x <= d+1) and
// coefl_i[k] = coef_i[d+1] lam_k (k <= d) are canonical, so one Montgomery
// product with H (Montgomery form) gives G canonical.
//
// The only work after the hash is alpha_i = T_i mod p and its stores: the
// finisher of round i takes coef_i and C_i from the state the finisher of
// round i-1 left (one product each with alpha_{i-1}, beside its own
// partial-sum loads, see Ctrl), and leaves the state of round i+1 before its
// own hash:
//   nu_l = C_i (1 - r_i) e_l,  nv_l = C_i (2 r_i - 1) e_l R,
//   npr = C_i (1 - r_i) R,     nqr = C_i (2 r_i - 1) R^2,
// each one product of C_i R with a factor of the eq1 row of round i filled
// at setup (e_l = eq1(x, r_{i+1}) or its lam-weighted form).  Consumers of
// alpha_i in Montgomery form (the folds) convert it themselves, beside their
// first loads.  A field product is some 160 64-bit multiply-adds, which one
// wave issues one after another (~0.4 us), so the products of one step are
// spread over the block's waves rather than chained in one.

template <int D>
struct FinLds {
  static constexpr int NH = D + 1, NE = D + 2, NC = NE + NH;
  static constexpr uint32_t LEN = 32u * (1u + NE);  // T_{i-1} || G_i(0..d+1)
  static constexpr uint32_t NB = (LEN + 9u + 63u) / 64u;
  uint32_t h[NH][NL];       // H_i(x), Montgomery, < p
  uint32_t cf[NC][NL];      // coef_i[0..d+1], coefl_i[0..d], canonical
  uint32_t u[NC][NL];       // nu of round i+1 (canonical)
  uint32_t v[NC][NL];       // nv of round i+1
  uint32_t pc[NL], q2[NL];  // npr, nqr of round i+1
  uint32_t cm[NL];          // C_i R
  uint32_t ac[8];           // alpha_i canonical words, after emit_round
  uint32_t msg[LEN / 4];    // T_{i-1} || G_i; T_i in words 0..7 after emit_round
  uint32_t kw[NB * 64];
  uint32_t skip;
};

// coef_i and C_i R of round `round` from the state in the control block and
// alpha_{round-1} (none for round 1: the state of round 1 has nv = nqr = 0):
// lanes l < NC write S.cf[l], lane NC writes S.cm, lanes 64..71 copy
// T_{round-1} into S.msg.  No barrier.
template <int D>
__device__ __forceinline__ void fin_start(const Ctrl* ctrl, uint32_t round, FinLds<D>& S) {
  constexpr int NC = FinLds<D>::NC;
  const uint32_t t = threadIdx.x;
  if (t <= (uint32_t)NC) {
    const Fe ac = round > 1 ? fe_vgpr(load_words_fe(ctrl->alpha[round - 2])) : fe_zero();
    if (t < (uint32_t)NC)
      lds_put(S.cf[t], fe_addmod(load_words_fe(ctrl->nu[t]), mont(ac, load_words_fe(ctrl->nv[t]))));
    else
      lds_put(S.cm, fe_addmod(fe_vgpr(load_words_fe(ctrl->npr)), mont(ac, fe_vgpr(load_words_fe(ctrl->nqr)))));
  }
  if (t >= 64 && t < 72) S.msg[t - 64] = ctrl->ts[t - 64];
}

// Emits G_round, leaves the state of round+1 (S.u, S.v, S.pc, S.q2 and the
// control block) and derives alpha_round.  On entry S.h, S.cf, S.cm and
// S.msg[0..7] hold round `round`'s values; on exit S.ac holds alpha_round
// (canonical) and S.msg[0..7] T_round.  Ends with a barrier.  All threads of
// the block call it.
//
// The hash: lanes 64 + b expand the schedule of every block b (k_t + w_t,
// the constants as immediates) into LDS while lane 0 runs rounds 0..15 of
// block 0 straight from the message; after a barrier lane 0 runs the rest
// from LDS.  Meanwhile lanes 128 on form the state of round+1, whose factors
// they load from the eq1 rows then (the hash hides that latency).
struct NoSideWork {
  __device__ void operator()() const {}
};

// `side` runs on waves 1..3 while lane 0 compresses the message after its
// first 16 rounds (the hash's serial part); it must not use __syncthreads.
//
// With `signal`, lane 0 also posts alpha_i to the control block's mailbox,
// each word tagged with i (see Ctrl::mbox), before its other stores, for the
// blocks of the same launch that wait for alpha_i (k_fin_wait).
template <int D, class Side = NoSideWork>
__device__ __forceinline__ void emit_round(Ctrl* ctrl, uint32_t round, FinLds<D>& S, uint32_t* evals_out,
                                           uint32_t* alpha_out, bool check, Side side = Side{},
                                           bool signal = false) {
  constexpr int NH = D + 1, NE = D + 2, NC = FinLds<D>::NC;
  constexpr uint32_t LEN = FinLds<D>::LEN, NB = FinLds<D>::NB;
  static_assert(NH <= 16, "one 16-lane group");
  const uint32_t t = threadIdx.x;
  // the state lanes (see below) load their eq1-row factor now, so that its
  // latency overlaps the G step; the rows are written at setup only
  const uint32_t sk = t - 128, sl = sk % ((uint32_t)NC + 1);
  const bool st_lane = t >= 128 && t < 128 + 2 * ((uint32_t)NC + 1), sq = sk > (uint32_t)NC;
  Fe sf = fe_zero();
  if (st_lane) {
    const Eq1Row* row = eq1_rows(ctrl) + (round - 1);
    sf = load_words_fe(sl == (uint32_t)NC ? (sq ? row->tr2 : row->omr) : (sq ? row->v[sl] : row->u[sl]));
  }
  if (t < 64) {
    // wave 0, lanes x <= d: G(x) = coef[x] H(x)
    if (t < (uint32_t)NH) {
      const Fe g = mont(lds_fe(S.cf[t]), lds_fe(S.h[t]));
      uint32_t w[8];
      fe_to_words(g, w);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        S.msg[8 + t * 8 + k] = w[k];
        evals_out[t * 8 + k] = w[k];
      }
    }
  } else if (t < 80) {
    // wave 1, lanes 64 + x: the terms coefl[x] H(x) of G(d+1) = sum_x
    // coefl[x] H(x), summed over the 16-lane group by shuffles
    const uint32_t x = t - 64;
    Fe term = fe_zero();
    if (x < (uint32_t)NH) term = mont(lds_fe(S.cf[NE + x]), lds_fe(S.h[x]));
#pragma unroll
    for (int msk = 8; msk >= 1; msk >>= 1) term = fe_add(term, shfl_xor_fe(term, msk));  // < 16p
    if (x == 0) {
      uint32_t w[8];
      fe_to_words(fe_reduce32(term), w);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        S.msg[8 + NH * 8 + k] = w[k];
        evals_out[NH * 8 + k] = w[k];
      }
    }
  }
  __syncthreads();
  static_assert(LEN >= 64 && NB <= 64, "block 0 is all message; one wave expands every block");
  uint32_t hv[8], v[8];
  if (t == 0) {
    sha256_init(hv);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = hv[i];
    sha256_first16(v, S.msg);
  } else if (t >= 64 && t < 64 + NB) {
    sha256_expand_block<LEN>(S.msg, S.kw, t - 64);
  } else if (st_lane) {
    // the state of round+1, one product with C_i R per lane (the eq1 row
    // holds the other factor, sf): lanes 128 + l (l < NC): nu_l, lane
    // 128 + NC: npr, lanes 128 + NC + 1 + l: nv_l, lane 128 + 2 NC + 1: nqr
    const Fe y = mont(fe_vgpr(lds_fe(S.cm)), sf);
    lds_put(sl == (uint32_t)NC ? (sq ? S.q2 : S.pc) : (sq ? S.v[sl] : S.u[sl]), y);
    store_words_fe(sl == (uint32_t)NC ? (sq ? ctrl->nqr : ctrl->npr) : (sq ? ctrl->nv[sl] : ctrl->nu[sl]), y);
  } else if (check && t == kBlock - 1) {
    // self-check (Sec. 3.4): G_i(0) + G_i(1) = G_{i-1}(alpha_{i-1}), the claim
    // of round i-1 (0 before round 1)
    static_assert(128 + 2 * (NC + 1) < kBlock, "the last lane is free");
    Fe claim = fe_zero();
    if (round > 1) claim = lagrange_at<NE>(evals_out - NE * 8, load_words_fe(ctrl->alpha[round - 2]));
    if (!fe_eq(claim, fe_addmod(load_words_fe(S.msg + 8), load_words_fe(S.msg + 16)))) set_error(ctrl, -7);
  }
  __syncthreads();
  if (t == 0) {
    sha256_rounds_kw(v, S.kw, 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) hv[i] += v[i];
#pragma unroll 1
    for (uint32_t b = 1; b < NB; ++b) sha256_compress_kw(hv, S.kw + b * 64u);
    uint32_t dg[8];
    sha256_digest(hv, dg);
    // alpha = digest (little-endian 256-bit integer) mod p; digest < 2^256 < 6p
    Fe al = fe_from_words(dg);
    al = fe_csub(fe_csub(fe_csub(al, kP4), kP2), kP);
    uint32_t w[8];
    fe_to_words(al, w);
    if (signal) {
      // the mailbox first, so that its stores leave ahead of the others
#pragma unroll
      for (int k = 0; k < 8; ++k)
        __hip_atomic_store(&ctrl->mbox[k], (uint64_t)round << 32 | w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      S.msg[k] = dg[k];
      S.ac[k] = w[k];
      ctrl->ts[k] = dg[k];
      ctrl->alpha[round - 1][k] = w[k];
      alpha_out[k] = w[k];
    }
    ctrl->round_done = round;
  } else if (t >= 64) {
    side();
  }
  __syncthreads();
}

// ---- round kernel, one thread per pair ---------------------------------------------
//
// FOLD = false: evaluate H_i on tables holding 2q live entries (pairs j, j+q).
// FOLD = true : the tables hold 4q entries; fold them with alpha_{i-1}
//               (u[j] = t[j] + alpha (t[j+2q] - t[j]), same for j+q), write
//               u[j], u[j+q] to dst, then evaluate on (u[j], u[j+q]).
// The grid is sized to be resident at once (one generation of blocks, each
// striding over the pairs).  Each block stores its d+1 partial sums; k_finish
// adds them up in the next launch, whose start orders it after every block's
// stores, so no block needs a device-wide fence (on this GPU such a fence
// writes back and invalidates the L2 and holds the CU for several
// microseconds).
//
// The body is shared with the batched kernel: block `blk` of the `nblk`
// blocks working on this round.
// Pairs a thread adds to its sums before bringing them back below 2p: each
// pair adds < 2p, so they stay < 2p + 32 * 2p < 128p.
constexpr uint32_t kLazyPairs = 32;

// Accumulators a gate's eval() keeps per thread: the NH point sums, plus
// GateAcc<Gate>::kExtra of its own, which finalize() folds into them.
template <class Gate, class = void>
struct GateAcc {
  static constexpr int kExtra = 0;
  template <int NA, int X0 = 0, int XE = 0>
  __device__ static __forceinline__ void finalize(Fe (&)[NA]) {}
};
template <class Gate>
struct GateAcc<Gate, std::void_t<decltype(Gate::kExtraAcc)>> {
  static constexpr int kExtra = Gate::kExtraAcc;
  template <int NA, int X0 = 0, int XE = Gate::NH>
  __device__ static __forceinline__ void finalize(Fe (&acc)[NA]) {
    Gate::template finalize<NA, X0, XE>(acc);
  }
};

// Evaluation of one pair at the points X0..XE-1 (0..NH-1: all of them).  The
// gates with extra accumulators take their count as a template argument.
template <class Gate, class = void>
struct EvalTakesNA : std::false_type {};
template <class Gate>
struct EvalTakesNA<Gate, std::void_t<decltype(Gate::kExtraAcc)>> : std::true_type {};
template <class Gate, int X0, int XE = Gate::NH, class Src, int NA>
__device__ __forceinline__ void gate_eval(const Src& src, const EqRows& er, Fe (&acc)[NA]) {
  if constexpr (EvalTakesNA<Gate>::value)
    Gate::template eval<Src, NA, X0, XE>(src, er, acc);
  else
    Gate::template eval<Src, X0, XE>(src, er, acc);
}

// X0 = 2 (round 1 only, ZC_FLAG_ASSUME_SATISFIED): the points 0 and 1 are not
// evaluated and their sums stay 0.
//
// HALF (a folding round with fewer pairs than one wave per SIMD holds):
// waves 2v and 2v+1 of a block take the same 64 pairs.  For gates that fold
// inside their evaluation both fold every table, the first evaluates the
// points [0, NH/2) and stores the folded pairs, the second evaluates
// [NH/2, NH); each point's sum comes from the wave that owns it (the other
// holds 0 there).  The vanilla gate splits its terms instead
// (GateVanilla::eval_terms), each wave folding and storing the tables its
// terms use.  Either way the block sums are the same field elements, from
// twice the waves, each with about half the products.
template <class Gate, bool FOLD, int X0 = 0, bool HALF = false>
__device__ __forceinline__ void round_body(const RoundArgs& a, const TabPtrs& src, const TabPtrs& dst, uint32_t blk,
                                           uint32_t nblk) {
  static_assert(X0 == 0 || !FOLD, "only round 1 skips points");
  static_assert(!HALF || (FOLD && X0 == 0), "halves split a folding round");
  constexpr int NH = Gate::NH;
  constexpr int XM = HALF ? NH / 2 : NH;
  const uint32_t half = HALF ? (threadIdx.x >> 6) & 1u : 0u;
  const uint32_t slot = HALF ? ((threadIdx.x >> 7) << 6) | (threadIdx.x & 63u) : threadIdx.x;
  const uint32_t slots = HALF ? blockDim.x / 2 : blockDim.x;  // pairs per block and pass
  constexpr int NA = NH + GateAcc<Gate>::kExtra;
  Fe acc[NA];
  auto z = [&](auto x) __attribute__((always_inline)) { acc[x] = fe_zero(); };
  Unroll<0, NA>::run(z);
  auto lower = [&](auto x) __attribute__((always_inline)) { acc[x] = fe_reduce128_to2(acc[x]); };

  {
    Fe alpha;
    if (FOLD) alpha = fe_to_mont(fe_vgpr(load_words_fe(a.ctrl->alpha[a.round - 2])));
    const uint32_t q = (uint32_t)a.q;
    const uint32_t stride = nblk * slots;
    // chunks of kLazyPairs pairs per thread, the sums lowered after each
    for (uint32_t j0 = blk * slots + slot; j0 < q; j0 += kLazyPairs * stride) {
      const uint32_t jend = (uint32_t)min((uint64_t)q, (uint64_t)j0 + (uint64_t)kLazyPairs * stride);
      for (uint32_t j = j0; j < jend; j += stride) {
        const EqRows er = issue_eq(a.eq, a.round, j);
        if (FOLD && Gate::kFoldInGate) {
          const FoldSrc fs{src, dst, a.src_pitch, a.dst_pitch, j, q, alpha, half == 0};
          if (half == 0)
            gate_eval<Gate, 0, XM>(fs, er, acc);
          else
            gate_eval<Gate, XM, NH>(fs, er, acc);
        } else if (FOLD && HALF) {
          if constexpr (HALF && !Gate::kFoldInGate) {
            const FoldSrc fs{src, dst, a.src_pitch, a.dst_pitch, j, q, alpha, true};
            if (half == 0) {
              Gate::template eval_terms<0>(fs, fs, er, acc);
            } else {
              const FoldSrc nb{src, dst, a.src_pitch, a.dst_pitch, j, q, alpha, false};
              Gate::template eval_terms<1>(fs, nb, er, acc);
            }
          }
        } else if (FOLD) {
          // fold every table first (a rolled loop: one copy of the code), then
          // evaluate on the folded pairs, which the L2 still holds (so the
          // sources are read non-temporally, the folded values stored normally)
          const uint64_t sp = a.src_pitch, dp = a.dst_pitch;
          RawPair n01 = issue_pair<true>(src.p[0], sp, j, q), n23 = issue_pair<true>(src.p[0], sp, j + 2 * q, q);
#pragma unroll 1
          for (int t = 0; t < Gate::K; ++t) {
            const RawPair c01 = n01, c23 = n23;
            if (t + 1 < Gate::K) {
              n01 = issue_pair<true>(src.p[t + 1], sp, j, q);
              n23 = issue_pair<true>(src.p[t + 1], sp, j + 2 * q, q);
            }
            store_el(dst.p[t], dp, j, fe_lerp(fe_from_words(c01.w0), fe_from_words(c23.w0), alpha));
            store_el(dst.p[t], dp, j + q, fe_lerp(fe_from_words(c01.w1), fe_from_words(c23.w1), alpha));
          }
          gate_eval<Gate, 0>(PairSrc{dst, dp, j, q}, er, acc);
        } else {
          gate_eval<Gate, X0>(PairSrcT<true>{src, a.src_pitch, j, q}, er, acc);
        }
      }
      Unroll<0, NA>::run(lower);
    }
  }
  auto red = [&](auto x) __attribute__((always_inline)) { acc[x] = fe_reduce2(acc[x]); };  // < 2p after lower
  Unroll<0, NA>::run(red);
  if (half == 0)
    GateAcc<Gate>::template finalize<NA, X0, XM>(acc);  // every acc[x] < p again
  else
    GateAcc<Gate>::template finalize<NA, XM, NH>(acc);
  Fe pts[NH];
  auto cp = [&](auto x) __attribute__((always_inline)) { pts[x] = acc[x]; };
  Unroll<0, NH>::run(cp);
  const Fe tot = block_reduce<NH>(pts);
  if (threadIdx.x < NH) store_words_fe(a.partials + ((uint64_t)blk * part_stride(NH) + threadIdx.x) * 8, tot);
}

template <class Gate, bool FOLD, int X0 = 0, bool HALF = false>
__global__ __launch_bounds__(kBlock) void k_round(RoundArgs a, TabPtrs src, TabPtrs dst) {
  round_body<Gate, FOLD, X0, HALF>(a, src, dst, blockIdx.x, gridDim.x);
}

// ---- lane-split rounds: 16 lanes per pair -------------------------------------------
//
// For rounds with few pairs one thread per pair leaves the GPU idle and makes
// the round as long as one thread's whole pair (fold of every table plus all
// d+1 points).  Here a group of 16 lanes shares a pair: lane t folds (or
// loads) table t, the pair goes through LDS, and lane x evaluates point X = x.

constexpr int kGroup = 16;                     // lanes per pair
constexpr int kSplitPairs = kBlock / kGroup;   // pairs per block

// f_M(e(X)) of one pair at point X (< 11p), from the pair's tables u0, u1
// (< p).  e(X) = u0 + X (u1 - u0) < (X+1) p.
template <class Gate, class Get>
__device__ __forceinline__ Fe point_f(Get get, uint32_t X) {
  constexpr int K = Gate::K;
  Fe e[K];
  auto f = [&](auto t) __attribute__((always_inline)) {
    Fe u0, u1;
    get(t, u0, u1);
    e[t] = fe_add(u0, fe_mul_small(fe_submod(u1, u0), X));
  };
  Unroll<0, K>::run(f);
  return Gate::point(e);
}

// Block total (mod p) of one value per lane: lane g of every 16-lane group
// holds the contribution for point g (< p).  Thread x < NH returns the total.
template <int NH>
__device__ __forceinline__ Fe group_reduce(Fe c) {
  __shared__ uint32_t red[kBlock / 64][kGroup][NL];
  c = fe_addmod(c, shfl_xor_fe(c, 16));
  c = fe_addmod(c, shfl_xor_fe(c, 32));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < kGroup) lds_put(red[wave][lane], c);
  __syncthreads();
  Fe s = fe_zero();
  if (threadIdx.x < NH) {
    s = lds_fe(red[0][threadIdx.x]);
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = fe_addmod(s, lds_fe(red[w][threadIdx.x]));
  }
  __syncthreads();
  return s;
}

// The last rounds of a proof inside one block, with the tables in LDS.  On
// entry round a.round has been emitted (S holds alpha_{a.round} and the state
// of round a.round+1) and the tables at dst hold 2q live entries,
// q = a.q <= 2 kTailQ.  Runs rounds a.round+1 .. mu (fold with the previous
// challenge, evaluate, emit) and the final fold, whose values are the
// openings; eq's opening is C_{mu+1}.  The coefficients of each round are
// formed beside its fold.
//
// Evaluation: point x of pair j is one thread's work (SL point slots, the
// power of two >= d+1, times PP = kBlock / SL pairs per pass); the PP lanes
// of a point are adjacent, so their sum is a shuffle reduction in one wave.
//
// With prefold the tables at dst hold T_{a.round - 1} (4q entries) instead:
// they are folded with alpha_{a.round - 1} on the way into LDS.
// ---- speculation inside the tail (gates of degree <= 3) ------------------------------
//
// While lane 0 hashes round r, waves 1..3 evaluate round r+1 for every
// candidate alpha_r = c in 0..d (the tables folded with c, like spec_body);
// round r+1 then takes H_{r+1}(X) = sum_c L_c(alpha_r) H_{r+1}(X; c), one
// product per lane, instead of a fold, an evaluation and a reduction on its
// critical path.  H_{r+1}(X) has degree <= d in alpha_r (the folded tables
// are affine in it, f_M has degree d), so the interpolation is exact.
template <class Gate>
struct TailSpec {
  static constexpr bool kOn = Gate::NH * Gate::NH <= 16 && Gate::D >= 2;
};

// LDS words of the tail: K tables and the eq rows (4 kTailQ entries each),
// then with speculation the candidate tables (K x (d+1) x kTailQ entries),
// 16 speculative sums, 3 x 16 per-wave sums and a barrier counter.
template <class Gate>
constexpr uint32_t tail_lds_words() {
  uint32_t w = (uint32_t)(Gate::K + 1) * 4u * kTailQ * NL;
  if (TailSpec<Gate>::kOn) w += (uint32_t)(Gate::K * Gate::NH) * kTailQ * NL + 16u * NL + 3u * 16u * NL + 1u;
  return w;
}

// L_c(x) R for the nodes 0..D (D = 2, 3), x canonical: w_c R^(D+1) times the
// D factors (x - k), k != c, canonical, in D Montgomery products.
template <int D>
__device__ __forceinline__ Fe lagrange_basis(const Fe& x, uint32_t c) {
  static_assert(D == 2 || D == 3, "two or three factors");
  constexpr LagrangeW<D> W{};
  Fe tk[D + 1];
  Fe ws = fe_zero();
  auto terms = [&](auto k) __attribute__((always_inline)) {
    Fe kk = fe_zero();
    kk.l[0] = (uint32_t)k;
    tk[k] = fe_submod(x, kk);
    if (c == (uint32_t)k) ws = fe_const(W.wsh[k]);
  };
  Unroll<0, D + 1>::run(terms);
  const Fe f0 = fe_sel(c == 0, tk[1], tk[0]);
  const Fe f1 = fe_sel(c <= 1, tk[2], tk[1]);
  if constexpr (D == 3) return mont(mont(ws, f0), mont(f1, fe_sel(c <= 2, tk[3], tk[2])));
  else return mont(mont(ws, f0), f1);
}

// A barrier of waves 1..3 (wave 0 is hashing meanwhile): each wave adds 1 to
// the counter and waits for `target` arrivals; targets grow by 3 per use, so
// the counter is never reset.  All three waves reach every use.
__device__ __forceinline__ void waves123_barrier(uint32_t* ctr, uint32_t target) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  if ((threadIdx.x & 63u) == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) __builtin_amdgcn_s_sleep(1);
  __builtin_amdgcn_wave_barrier();
}

// Waves 1..3 during round r's hash: H_{r+1}(x; c) for x, c in 0..d into
// HSP[4 c + x], from the tables of round r (L entries) folded with c.
// Nothing to do after the last round.
template <class Gate, class TF, class UF>
__device__ __forceinline__ void tail_speculate(uint32_t r, uint32_t L, uint32_t mu, TF T, UF U, const uint32_t* eqrow,
                                               uint32_t* HSP, uint32_t* RED3, uint32_t* CTR, uint32_t& bar_target) {
  constexpr int K = Gate::K;
  constexpr int NH = Gate::NH;
  if (r >= mu) return;
  const uint32_t tt = threadIdx.x - 64;  // 0..191
  const uint32_t h2 = L / 2, qs = L / 4;  // T_{r+1}(c) has h2 entries, round r+1 qs pairs
  // the candidate tables: T(k, e) + c (T(k, e + h2) - T(k, e)), e < h2
  for (uint32_t idx = tt; idx < (uint32_t)K * h2; idx += 192) {
    const uint32_t k = idx / h2, e = idx % h2;
    const Fe t0 = lds_fe(T(k, e));
    const Fe dd = fe_submod(lds_fe(T(k, e + h2)), t0);
    Fe u = t0;
#pragma unroll
    for (int c = 0; c < NH; ++c) {
      lds_put(U(k, c, e), u);
      if (c + 1 < NH) u = fe_addmod(u, dd);
    }
  }
  bar_target += 3;
  waves123_barrier(CTR, bar_target);
  // lane slot (x, c) = tt mod 16; the 12 lanes of a slot stride over the pairs
  const uint32_t x = tt & 3u, c = (tt >> 2) & 3u;
  Fe acc = fe_zero();
  if (x < (uint32_t)NH && c < (uint32_t)NH) {
    for (uint32_t e = tt >> 4; e < qs; e += 12) {
      auto get = [&](int t, Fe& u0, Fe& u1) __attribute__((always_inline)) {
        u0 = lds_fe(U(t, c, e));
        u1 = lds_fe(U(t, c, e + qs));
      };
      acc = fe_addmod(acc, mont(point_f<Gate>(get, x), lds_fe(eqrow + (qs + e) * NL)));
    }
  }
  acc = fe_addmod(acc, shfl_xor_fe(acc, 16));
  acc = fe_addmod(acc, shfl_xor_fe(acc, 32));
  if ((tt & 63u) < 16) lds_put(RED3 + ((tt >> 6) * 16 + (tt & 15u)) * NL, acc);
  bar_target += 3;
  waves123_barrier(CTR, bar_target);
  if (tt < 16) {
    Fe sum = lds_fe(RED3 + tt * NL);
    sum = fe_addmod(sum, lds_fe(RED3 + (16 + tt) * NL));
    sum = fe_addmod(sum, lds_fe(RED3 + (32 + tt) * NL));
    lds_put(HSP + tt * NL, sum);
  }
}

template <class Gate>
__device__ __forceinline__ void run_tail(const RoundArgs& a, const TabPtrs& dst, FinLds<Gate::D>& S, bool prefold) {
  constexpr int K = Gate::K;
  constexpr int NH = Gate::NH;
  constexpr int NC = FinLds<Gate::D>::NC;
  constexpr uint32_t SL = NH <= 4 ? 4u : (NH <= 8 ? 8u : 16u);
  constexpr uint32_t PP = kBlock / SL;
  static_assert(PP <= 64 && SL * PP == kBlock, "point groups within a wave");
  extern __shared__ uint32_t tail_lds[];  // tail_lds_words<Gate>(): [K][4 kTailQ][NL] tables, eq rows, ...
  constexpr uint32_t CAP = 4 * kTailQ;
  auto T = [&](int t, uint32_t e) -> uint32_t* { return tail_lds + ((uint32_t)t * CAP + e) * NL; };
  uint32_t* eqrow = tail_lds + (uint32_t)K * CAP * NL;
  constexpr bool SPECT = TailSpec<Gate>::kOn;
  // speculation: candidate tables SU(k, c, e), sums HSP[c 4 + x], per-wave
  // sums RED3[w][c 4 + x], the barrier counter
  uint32_t* SU = eqrow + CAP * NL;
  auto U = [&](int t, uint32_t c, uint32_t e) -> uint32_t* {
    return SU + (((uint32_t)t * (uint32_t)NH + c) * kTailQ + e) * NL;
  };
  uint32_t* HSP = SU + (uint32_t)(K * NH) * kTailQ * NL;
  uint32_t* RED3 = HSP + 16 * NL;
  uint32_t* CTR = RED3 + 3 * 16 * NL;
  const uint32_t tid = threadIdx.x;
  if (SPECT && tid == 0) *CTR = 0;
  uint32_t bar_target = 0;
  uint32_t L = 2 * (uint32_t)a.q;
  const Fe pa = prefold ? fe_to_mont(fe_vgpr(load_words_fe(a.ctrl->alpha[a.round - 2]))) : fe_zero();
  for (uint32_t idx = tid; idx < K * L; idx += blockDim.x) {
    const uint32_t t = idx / L, e = idx % L;
    Fe v = load_el(dst.p[t], a.dst_pitch, e);
    if (prefold) v = fe_lerp(v, load_el(dst.p[t], a.dst_pitch, e + L), pa);
    lds_put(T(t, e), v);
  }
  // E_r[j] of every tail round r, heap-style: row 2^(mu-r) + j, rows [1, q)
  for (uint32_t hrow = tid; hrow < (uint32_t)a.q; hrow += blockDim.x) {
    if (hrow == 0) continue;
    const uint32_t lg = 31u - __builtin_clz(hrow);
    lds_put(eqrow + hrow * NL, eq_factor(a.eq, a.mu - lg, hrow - (1u << lg)));
  }
  __syncthreads();
  const uint32_t x = tid / PP, pp = tid % PP;
  for (uint32_t r = a.round + 1; r <= a.mu + 1; ++r) {
    // fold with alpha_{r-1}: L -> L/2 entries; beside it coef_r and C_r R
    // from alpha_{r-1} and the state emit_round left
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = S.ac[k];
    const Fe ac = fe_vgpr(fe_from_words(w));
    const uint32_t h = L / 2;
    auto fold = [&](uint32_t first, uint32_t step) __attribute__((always_inline)) {
      const Fe alpha = fe_to_mont(ac);
      for (uint32_t idx = first; idx < K * h; idx += step) {
        const uint32_t t = idx / h, e = idx % h;
        const Fe u0 = lds_fe(T(t, e)), u1 = lds_fe(T(t, e + h));
        lds_put(T(t, e), fe_lerp(u0, u1, alpha));
      }
    };
    // round r was evaluated during round r-1's hash (spec_r): its message
    // needs no folded table, so waves 1-3 fold during round r's hash, before
    // they speculate on round r+1
    const bool spec_r = SPECT && r >= a.round + 2 && r <= a.mu;
    if (!spec_r) fold(tid, blockDim.x);
    if (tid < (uint32_t)NC) {
      if (r <= a.mu) lds_put(S.cf[tid], fe_addmod(lds_fe(S.u[tid]), mont(ac, lds_fe(S.v[tid]))));
    } else if (tid == (uint32_t)NC) {
      lds_put(S.cm, fe_addmod(fe_vgpr(lds_fe(S.pc)), mont(ac, fe_vgpr(lds_fe(S.q2)))));
    }
    // spec_r: the weights L_c(alpha_{r-1})
    Fe lcr = fe_zero();
    const uint32_t sx = tid & 3u, sc = (tid >> 2) & 3u;
    if constexpr (SPECT) {
      if (spec_r && tid >= 64 + 16 && tid < 64 + 16 + 16 && sx < (uint32_t)NH && sc < (uint32_t)NH)
        lcr = lagrange_basis<Gate::D>(ac, sc);
    }
    __syncthreads();
    L = h;
    if (r > a.mu) break;  // the final fold: entry 0 of each table is its opening
    const uint32_t q = L / 2;
    if (spec_r) {
      // lanes 80..95 (wave 1): H_r(x) R = sum_c L_c R H_r(x; c) R / R
      if (tid >= 80 && tid < 96) {
        Fe hv = fe_zero();
        if (sx < (uint32_t)NH && sc < (uint32_t)NH) hv = mont(fe_vgpr(lcr), lds_fe(HSP + (tid & 15u) * NL));
        hv = fe_addmod(hv, shfl_xor_fe(hv, 4));
        hv = fe_addmod(hv, shfl_xor_fe(hv, 8));
        if (sc == 0 && sx < (uint32_t)NH) lds_put(S.h[sx], hv);
      }
      __syncthreads();
      auto side = [&]() __attribute__((always_inline)) {
        if constexpr (SPECT) {
          fold(tid - 64, blockDim.x - 64);
          bar_target += 3;
          waves123_barrier(CTR, bar_target);
          tail_speculate<Gate>(r, L, a.mu, T, U, eqrow, HSP, RED3, CTR, bar_target);
        }
      };
      emit_round<Gate::D>(a.ctrl, r, S, a.evals_out + (uint64_t)(r - a.round) * Gate::NE * 8,
                          a.alpha_out + (uint64_t)(r - a.round) * 8, a.check != 0, side);
      continue;
    }
    Fe c = fe_zero();
    if (x < (uint32_t)NH) {
      // uniform trip count; lanes past q evaluate pair e mod q (q is a power
      // of two) and drop it, so the whole wave stays active (a wave with only
      // a few active lanes ran this loop several times slower, measured)
      for (uint32_t e0 = 0; e0 < q; e0 += PP) {
        const uint32_t e = (e0 + pp) & (q - 1);
        auto get = [&](int t, Fe& u0, Fe& u1) __attribute__((always_inline)) {
          u0 = lds_fe(T(t, e));
          u1 = lds_fe(T(t, e + q));
        };
        Fe v = fe_addmod(c, mont(point_f<Gate>(get, x), lds_fe(eqrow + (q + e) * NL)));
#pragma unroll
        for (int i = 0; i < NL; ++i) asm volatile("" : "+v"(v.l[i]));  // computed on every lane
        if (e0 + pp < q) c = v;
      }
    }
    // lanes pp >= q hold 0, so the sum of lanes 0..q-1 needs the levels below q only
#pragma unroll
    for (uint32_t msk = PP / 2; msk >= 1; msk >>= 1)
      if (msk < q) c = fe_addmod(c, shfl_xor_fe(c, (int)msk));
    if (pp == 0 && x < (uint32_t)NH) lds_put(S.h[x], c);
    __syncthreads();
    auto side = [&]() __attribute__((always_inline)) {
      if constexpr (SPECT) tail_speculate<Gate>(r, L, a.mu, T, U, eqrow, HSP, RED3, CTR, bar_target);
    };
    emit_round<Gate::D>(a.ctrl, r, S, a.evals_out + (uint64_t)(r - a.round) * Gate::NE * 8,
                        a.alpha_out + (uint64_t)(r - a.round) * 8, a.check != 0, side);
  }
  if (a.check && tid == 0) {
    // self-check of the final identity (Sec. 3.3, 3.4): G_mu(alpha_mu) =
    // f_M(openings) eq(alpha, r), the openings being entry 0 of each table
    // and eq(alpha, r) = C_{mu+1}
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = S.ac[k];
    const Fe claim = lagrange_at<Gate::NE>(a.evals_out + (uint64_t)(a.mu - a.round) * Gate::NE * 8, fe_from_words(w));
    Fe e[K];
#pragma unroll
    for (int t = 0; t < K; ++t) e[t] = lds_fe(T(t, 0));
    const Fe f = fe_reduce32(Gate::point(e));  // f_M(openings) R
    if (!fe_eq(claim, fe_from_mont(mont(f, fe_vgpr(lds_fe(S.cm)))))) set_error(a.ctrl, -7);
  }
  if (tid < K) store_words_fe(a.openings + tid * 8, fe_from_mont(lds_fe(T(tid, 0))));
  if (tid == K) store_words_fe(a.openings + K * 8, fe_from_mont(fe_vgpr(lds_fe(S.cm))));
}

// alpha_{round} for the blocks of a k_fin_wait launch: lanes 0..7 poll the
// eight mailbox words (one device-coherent 64-bit load each, together one
// request) until every word carries the tag `round`, or a device error is
// set, or ~10 ms have passed (then ZC_ESTATE: the bytes are wrong but every
// block ends); the block then reads alpha from LDS.  The exits are uniform
// over the eight lanes.  All threads of the block call it (it has a barrier).
constexpr uint64_t kWaitTicks = 1000000;  // s_memrealtime runs at 100 MHz
__device__ __forceinline__ Fe wait_alpha(Ctrl* ctrl, uint32_t round, uint32_t* box) {
  if (threadIdx.x < 8) {
    const uint32_t k = threadIdx.x;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    uint64_t m;
    for (;;) {
      m = __hip_atomic_load(&ctrl->mbox[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__all((uint32_t)(m >> 32) == round)) break;
      if (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {
        if (k == 0) set_error(ctrl, -5);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    box[k] = (uint32_t)m;
  }
  __syncthreads();
  uint32_t w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = box[k];
  return fe_to_mont(fe_vgpr(fe_from_words(w)));
}

// Round with 16 lanes per pair: block `blk` of `nblk` strides over the pairs.
// WAIT (FOLD only): alpha_{i-1} comes from the mailbox once block 0 of the
// same launch has posted it; the block's first loads are issued before the
// wait, so their latency overlaps the hash.
template <class Gate, bool FOLD, bool WAIT, int X0 = 0>
__device__ __forceinline__ void split_body(const RoundArgs& a, const TabPtrs& srct, const TabPtrs& dstt, uint32_t blk,
                                           uint32_t nblk) {
  static_assert(FOLD || !WAIT, "only a folding round waits for its challenge");
  static_assert(X0 == 0 || !FOLD, "only round 1 skips points");
  constexpr int K = Gate::K;
  constexpr int NH = Gate::NH;
  __shared__ uint32_t sh[kSplitPairs][K][2][NL];
  __shared__ uint32_t box[WAIT ? 8 : 1];
  const uint32_t g = threadIdx.x % kGroup, pl = threadIdx.x / kGroup;
  Fe c = fe_zero();
  Fe walpha = fe_zero();
  bool have_alpha = !WAIT;
  {
    const uint32_t q = (uint32_t)a.q;
    const uint64_t stride = (uint64_t)nblk * kSplitPairs;
    for (uint64_t base = (uint64_t)blk * kSplitPairs; base < q; base += stride) {
      const uint32_t j = (uint32_t)(base + pl);
      // the eq rows of the pair are loaded now, used after the exchange
      EqRows er{};
      if (j < q && g < (uint32_t)NH) er = issue_eq(a.eq, a.round, j);
      // table g's pointers, selected without indexing the argument array per lane
      const uint32_t* src = srct.p[0];
      uint32_t* dst = dstt.p[0];
      auto sel = [&](auto t) __attribute__((always_inline)) {
        if (g == (uint32_t)t) {
          src = srct.p[t];
          dst = dstt.p[t];
        }
      };
      Unroll<1, K>::run(sel);
      const bool mine = j < q && g < (uint32_t)K;
      Fe u0, u1, a0, a1, a2, a3;
      if (mine) {
        if (FOLD) {
          const uint64_t sp = a.src_pitch;
          a0 = load_el(src, sp, j);
          a2 = load_el(src, sp, j + 2 * q);
          a1 = load_el(src, sp, j + q);
          a3 = load_el(src, sp, j + 3 * q);
        } else {
          u0 = load_el(src, a.src_pitch, j);
          u1 = load_el(src, a.src_pitch, j + q);
        }
      }
      if (WAIT && !have_alpha) {
        walpha = wait_alpha(a.ctrl, a.round - 1, box);
        have_alpha = true;
      }
      if (mine) {
        if (FOLD) {
          const Fe alpha = WAIT ? walpha : fe_to_mont(fe_vgpr(load_words_fe(a.ctrl->alpha[a.round - 2])));
          u0 = fe_lerp(a0, a2, alpha);
          u1 = fe_lerp(a1, a3, alpha);
          store_el(dst, a.dst_pitch, j, u0);
          store_el(dst, a.dst_pitch, j + q, u1);
        }
        lds_put(sh[pl][g][0], u0);
        lds_put(sh[pl][g][1], u1);
      }
      __syncthreads();
      if (j < q && g < (uint32_t)NH && g >= (uint32_t)X0) {
        auto get = [&](int t, Fe& v0, Fe& v1) __attribute__((always_inline)) {
          v0 = lds_fe(sh[pl][t][0]);
          v1 = lds_fe(sh[pl][t][1]);
        };
        const Fe E = resolve_eq(er);
        c = fe_addmod(c, fe_reduce2(fe_mul(point_f<Gate>(get, g), E)));
      }
      __syncthreads();
    }
  }
  const Fe tot = group_reduce<NH>(c);
  if (threadIdx.x < NH) store_words_fe(a.partials + ((uint64_t)blk * part_stride(NH) + threadIdx.x) * 8, tot);
}

// Round with 16 lanes per pair; the grid strides over the pairs and is sized
// like k_round's.
template <class Gate, bool FOLD, int X0 = 0>
__global__ __launch_bounds__(kBlock) void k_round_split(RoundArgs a, TabPtrs srct, TabPtrs dstt) {
  split_body<Gate, FOLD, false, X0>(a, srct, dstt, blockIdx.x, gridDim.x);
}

// ---- speculative rounds (gates of degree <= 3) -----------------------------------------
//
// Round r needs alpha_{r-1}, which the finisher of round r-1 is still
// deriving.  The fold is linear in alpha, so H_r(X) is a polynomial of degree
// <= d in alpha_{r-1}: spec_body evaluates round r for alpha_{r-1} = c,
// c = 0..d, beside that finisher (blocks 1.. of k_fin_spec), and the next
// finisher interpolates the sums at the true alpha_{r-1} (exact in F_p, so
// the round message is the same field element).  The (d+1)^2 pairs (c, X)
// fill the 16 lanes of a pair.
//
// FIRST: the tables hold T_{r-1} (4q live entries, q the pairs of round r).
// Otherwise they hold T_{r-2} (8q entries); alpha_{r-2} is known, so the
// kernel folds T_{r-1} = T_{r-2} + alpha_{r-2} (T_{r-2}[+4q] - T_{r-2}) for the
// entries j, j+q, j+2q, j+3q of each pair j and writes it to dst (in place:
// each thread writes only entries it read).  The lane of table t also folds
// its pair with every candidate c (a small integer: additions only) into
// LDS; lane (c, X) then evaluates point X.  Block partials hold the (d+1)^2
// sums, slot c (d+1) + X.
template <class Gate>
struct SpecShape {
  static constexpr int NS = Gate::NH * Gate::NH;
  static constexpr bool kOk = NS <= kGroup;
};

template <class Gate, bool FIRST>
__device__ __forceinline__ void spec_body(const RoundArgs& a, const TabPtrs& srct, const TabPtrs& dstt, uint32_t blk,
                                          uint32_t nblk) {
  constexpr int K = Gate::K;
  constexpr int NH = Gate::NH;
  constexpr int NS = SpecShape<Gate>::NS;
  static_assert(SpecShape<Gate>::kOk, "(d+1)^2 lanes per pair");
  __shared__ uint32_t sh[kSplitPairs][K][NH][2][NL];  // T_r[j], T_r[j+q] for alpha_{r-1} = c
  const uint32_t g = threadIdx.x % kGroup, pl = threadIdx.x / kGroup;
  const uint32_t cc = g / NH, X = g % NH;  // candidate alpha_{r-1} = cc and point X of lane g < NS
  Fe acc = fe_zero();
  const uint32_t q = (uint32_t)a.q;
  const uint64_t stride = (uint64_t)nblk * kSplitPairs;
  for (uint64_t base = (uint64_t)blk * kSplitPairs; base < q; base += stride) {
    const uint32_t j = (uint32_t)(base + pl);
    EqRows er{};
    if (j < q && g < (uint32_t)NS) er = issue_eq(a.eq, a.round, j);
    if (j < q && g < (uint32_t)K) {
      const uint32_t* src = srct.p[0];
      uint32_t* dst = dstt.p[0];
      auto sel = [&](auto t) __attribute__((always_inline)) {
        if (g == (uint32_t)t) {
          src = srct.p[t];
          dst = dstt.p[t];
        }
      };
      Unroll<1, K>::run(sel);
      const uint64_t sp = a.src_pitch;
      Fe A[4];  // T_{r-1} at j, j+q, j+2q, j+3q
      if (FIRST) {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) A[k] = load_el(src, sp, j + k * q);
      } else {
        const Fe alpha = fe_to_mont(fe_vgpr(load_words_fe(a.ctrl->alpha[a.round - 3])));  // alpha_{r-2}
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
          A[k] = fe_lerp(load_el(src, sp, j + k * q), load_el(src, sp, j + k * q + 4 * q), alpha);
          store_el(dst, a.dst_pitch, j + k * q, A[k]);
        }
      }
      // T_r for alpha_{r-1} = c: A0 + c (A2 - A0), A1 + c (A3 - A1), c = 0..d
      const Fe d0 = fe_submod(A[2], A[0]), d1 = fe_submod(A[3], A[1]);
      Fe u0 = A[0], u1 = A[1];
#pragma unroll
      for (int c = 0; c < NH; ++c) {
        lds_put(sh[pl][g][c][0], u0);
        lds_put(sh[pl][g][c][1], u1);
        if (c + 1 < NH) {
          u0 = fe_addmod(u0, d0);
          u1 = fe_addmod(u1, d1);
        }
      }
    }
    __syncthreads();
    if (j < q && g < (uint32_t)NS) {
      auto get = [&](int t, Fe& u0, Fe& u1) __attribute__((always_inline)) {
        u0 = lds_fe(sh[pl][t][cc][0]);
        u1 = lds_fe(sh[pl][t][cc][1]);
      };
      const Fe E = resolve_eq(er);
      acc = fe_addmod(acc, fe_reduce2(fe_mul(point_f<Gate>(get, X), E)));
    }
    __syncthreads();
  }
  const Fe tot = group_reduce<NS>(acc);
  if (threadIdx.x < (uint32_t)NS) store_words_fe(a.partials + ((uint64_t)blk * part_stride(NS) + threadIdx.x) * 8, tot);
}

// ---- end of a round: one block -------------------------------------------------------
//
// Adds up the round kernel's a.nparts partial sums, emits G_i, derives
// alpha_i and, with a.tail, runs the rest of the proof in LDS (run_tail).
// The challenge never leaves the device.  Runs only when round i-1 has been
// emitted (ZC_ESTATE otherwise).
// (Body shared with the batched finisher; `dst` holds the tables the tail
// starts from.)
//
// SPEC: the partials are spec_body's (d+1)^2 sums per block, H_i(X) for
// alpha_{i-1} = c; the finisher interpolates them at alpha_{i-1}:
// H_i(X) = sum_c L_c(alpha_{i-1}) H_i(X; c), L_c the Lagrange basis of the
// nodes 0..d, formed beside the partial-sum loads.  A tail then starts from
// T_{i-1} (prefold).
template <class Gate, bool SPEC = false>
__device__ __forceinline__ void finish_body(const RoundArgs& a, const TabPtrs& dst) {
  constexpr int NH = Gate::NH;
  constexpr int NC = FinLds<Gate::D>::NC;
  constexpr int NV = SPEC ? NH * NH : NH;  // partial sums per block
  __shared__ FinLds<Gate::D> S;
  __shared__ uint32_t hs[SPEC ? NV : 1][NL];  // SPEC: H_i(X; c), slot c NH + X
  __shared__ uint32_t lc[SPEC ? NH : 1][NL];  // SPEC: L_c(alpha_{i-1}) R (its first factor until the barrier)
  __shared__ uint32_t lb[SPEC ? NH : 1][NL];  // SPEC: the second factor of L_c(alpha_{i-1}) R
  const uint32_t t = threadIdx.x;
  // every global load first, so that their latencies overlap: the
  // control-block values of lanes <= NC (coef_i, C_i), alpha_{i-1} for the
  // Lagrange lanes, T_{i-1}, then the partial sums
  const bool coef_lane = t <= (uint32_t)NC;
  const bool lag_lane = SPEC && ((t >= 128 && t < 128 + (uint32_t)NH) || (t >= 192 && t < 192 + (uint32_t)NH));
  Fe ca = fe_zero(), cu = fe_zero(), cv = fe_zero();
  if ((coef_lane || lag_lane) && a.round > 1) ca = fe_vgpr(load_words_fe(a.ctrl->alpha[a.round - 2]));
  if (coef_lane) {
    cu = fe_vgpr(load_words_fe(t < (uint32_t)NC ? a.ctrl->nu[t] : a.ctrl->npr));
    cv = fe_vgpr(load_words_fe(t < (uint32_t)NC ? a.ctrl->nv[t] : a.ctrl->nqr));
  }
  uint32_t tsw = 0;
  if (t >= 64 && t < 72) tsw = a.ctrl->ts[t - 64];
  if (t == 0) {
    const bool ok = a.ctrl->round_done + 1 == a.round;
    S.skip = ok ? 0u : 1u;
    if (!ok) set_error(a.ctrl, -5);
  }
  Gather<NV> gat;
  gat.load(a.partials, a.nparts);
  // coef_i[l] = nu_l + alpha_{i-1} nv_l (lanes l < NC), C_i R (lane NC), see Ctrl
  if (coef_lane) lds_put(t < (uint32_t)NC ? S.cf[t] : S.cm, fe_addmod(cu, mont(ca, cv)));
  if (t >= 64 && t < 72) S.msg[t - 64] = tsw;
  if constexpr (SPEC) {
    // L_c(alpha) R = w_c prod_{k != c} (alpha - k) R, from the d factors
    // (alpha - k) canonical multiplied pairwise onto w_c R^(d+1): lane 128 + c
    // forms (w_c R^(d+1)) x, lane 192 + c the rest (y z, or y when d = 2),
    // lane 128 + c their product after the barrier below
    static_assert(Gate::D == 2 || Gate::D == 3, "two or three factors");
    if (lag_lane) {
      constexpr LagrangeW<Gate::D> W{};
      const uint32_t c = t & 63u;
      Fe tk[NH];  // alpha - k, canonical
      Fe ws = fe_zero();
      auto terms = [&](auto k) __attribute__((always_inline)) {
        Fe kk = fe_zero();
        kk.l[0] = (uint32_t)k;
        tk[k] = fe_submod(ca, kk);
        if (c == (uint32_t)k) ws = fe_const(W.wsh[k]);
      };
      Unroll<0, NH>::run(terms);
      // the factors k != c in order: x, y (, z)
      if (t < 192) {
        lds_put(lc[c], mont(ws, fe_sel(c == 0, tk[1], tk[0])));
      } else {
        const Fe y = fe_sel(c <= 1, tk[2], tk[1]);
        if constexpr (Gate::D == 3)
          lds_put(lb[c], mont(y, fe_sel(c <= 2, tk[3], tk[2])));
        else
          lds_put(lb[c], y);
      }
    }
  }
  gat.reduce(a.nparts, SPEC ? hs : S.h);
  if (S.skip) return;
  if constexpr (SPEC) {
    if (t >= 128 && t < 128 + (uint32_t)NH) lds_put(lc[t - 128], mont(lds_fe(lc[t - 128]), lds_fe(lb[t - 128])));
    __syncthreads();
    // H_i(X) = sum_c L_c H_i(X; c): lane c NP + X of wave 0 forms one product
    // (NP = NH rounded up to a power of two), and shuffles across the lanes NP
    // apart sum over c (every term < p, so the sum is the same in any order)
    constexpr uint32_t NP = NH <= 2 ? 2u : 4u;
    static_assert(NH <= 4, "degree <= 3");
    if (t < 64) {
      const uint32_t c = t / NP, X = t % NP;
      Fe h = fe_zero();
      if (c < (uint32_t)NH && X < (uint32_t)NH) h = mont(fe_vgpr(lds_fe(lc[c])), lds_fe(hs[c * NH + X]));
#pragma unroll
      for (uint32_t msk = NP; msk < NP * NP; msk <<= 1) h = fe_addmod(h, shfl_xor_fe(h, (int)msk));
      if (t < (uint32_t)NH) lds_put(S.h[t], h);
    }
    __syncthreads();
  }
  emit_round<Gate::D>(a.ctrl, a.round, S, a.evals_out, a.alpha_out, a.check != 0, NoSideWork{}, a.signal != 0);
  if (a.tail) run_tail<Gate>(a, dst, S, SPEC);
}

template <class Gate>
__global__ __launch_bounds__(kBlock) void k_finish(RoundArgs a, TabPtrs dst) {
  finish_body<Gate>(a, dst);
}

// The finisher of round r-1 (block 0, no tail) beside the speculative
// evaluation of round r (the other blocks), on the folded copies `tabs`.
// FIRST: round r-1 was evaluated normally, and the tables hold T_{r-1}.
template <class Gate, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_fin_spec(RoundArgs fa, RoundArgs sa, TabPtrs tabs) {
  if (blockIdx.x == 0)
    finish_body<Gate, !FIRST>(fa, tabs);
  else
    spec_body<Gate, FIRST>(sa, tabs, tabs, blockIdx.x - 1, gridDim.x - 1);
}

// The finisher of the last speculative round, which then runs the tail.
template <class Gate>
__global__ __launch_bounds__(kBlock) void k_finish_spec(RoundArgs a, TabPtrs dst) {
  finish_body<Gate, true>(a, dst);
}

// Gates without speculation (degree > 3): the finisher of round i-1 (block 0,
// no tail, fa.signal set) beside the lane-split evaluation of round i (the
// other blocks), which folds the tables in place with alpha_{i-1} as soon as
// block 0 posts it.  Blocks are dispatched in order, so block 0 runs before
// any block waits for it.
template <class Gate>
__global__ __launch_bounds__(kBlock) void k_fin_wait(RoundArgs fa, RoundArgs sa, TabPtrs tabs) {
  if (blockIdx.x == 0)
    finish_body<Gate, false>(fa, tabs);
  else
    split_body<Gate, true, true>(sa, tabs, tabs, blockIdx.x - 1, gridDim.x - 1);
}

// ---- batches: many instances, round by round in lockstep ------------------------------
//
// Instance n of a batch is described once (InstDesc) and proves exactly as a
// single zc_prove would, with its own workspace, so its bytes are the same.
// At step s every instance with a round-kernel round left runs its round
// s+1; the blocks of one launch are shared out by a prefix sum over the
// instances of one gate, and one finisher block per instance then emits the
// round (and, at the instance's last launched round, runs its tail).  The
// per-round serial work of the instances (reduction, SHA-256, challenge)
// thereby overlaps instead of adding up.

struct InstDesc {
  TabPtrs orig;      // caller tables (read only), pitch 2^mu
  TabPtrs fold;      // folded copies in the instance workspace, pitch 2^(mu-1)
  EqTabs eq;
  Ctrl* ctrl;
  uint32_t* partials;
  uint32_t* evals;     // mu x (d+2) x 8
  uint32_t* alphas;    // mu x 8
  uint32_t* openings;  // (k+1) x 8
  const uint32_t* r;
  uint32_t mu, gate, m, ne;
  uint32_t last;       // last round with a round kernel; its finisher runs the tail
  uint32_t flags;      // zc_shape.flags
  uint64_t pitch;      // plane pitch of the caller tables (elements, >= 2^mu)
};

// One gate's share of a step: instances inst[0..count) (indices into descs)
// with block ranges [prefix[i], prefix[i+1]), all running round step + 1.
struct BatchStep {
  const InstDesc* descs;
  const uint32_t* inst;
  const uint32_t* prefix;
  uint32_t count;
  uint32_t step;
  __device__ __forceinline__ uint32_t n() const { return count; }
  __device__ __forceinline__ uint32_t pre(uint32_t i) const { return prefix[i]; }
  __device__ __forceinline__ const InstDesc& desc(uint32_t i) const { return descs[inst[i]]; }
  __device__ __forceinline__ uint32_t round(uint32_t) const { return step + 1; }
  __device__ __forceinline__ uint32_t part(uint32_t) const { return 0; }
  __device__ __forceinline__ uint32_t parts(uint32_t) const { return 1; }
};

// One gate's share of a serving step: up to kServeMax instances, each at its
// own round, carried whole in the kernel arguments (no copy per step).
constexpr int kServeMax = 256;
// An instance's round may also be split into `parts` launches of equal
// block counts (part p runs blocks [p nb, (p + 1) nb) of the nb * parts
// blocks of the round); only the last part's launch has a finisher.
// nfin: entries 0..nfin-1 get a finisher block.
struct ServeStep {
  const InstDesc* pool;
  uint32_t count;
  uint32_t nfin;
  uint32_t prefix[kServeMax + 1];
  uint16_t slot[kServeMax];
  uint8_t rnd[kServeMax];
  uint8_t prt[kServeMax];
  uint8_t nprt[kServeMax];
  __device__ __forceinline__ uint32_t n() const { return count; }
  __device__ __forceinline__ uint32_t pre(uint32_t i) const { return prefix[i]; }
  __device__ __forceinline__ const InstDesc& desc(uint32_t i) const { return pool[slot[i]]; }
  __device__ __forceinline__ uint32_t round(uint32_t i) const { return rnd[i]; }
  __device__ __forceinline__ uint32_t part(uint32_t i) const { return prt[i]; }
  __device__ __forceinline__ uint32_t parts(uint32_t i) const { return nprt[i]; }
};
static_assert(sizeof(ServeStep) <= 4096 - 64, "kernel argument size");

__device__ __forceinline__ RoundArgs batch_round_args(const InstDesc& d, uint32_t round, uint32_t nparts) {
  RoundArgs a{};  // every field set: signal, share and skip01 stay 0 here
  const uint64_t n = 1ull << d.mu;
  a.src_pitch = round <= 2 ? d.pitch : n / 2;
  a.dst_pitch = round == 1 ? d.pitch : n / 2;
  a.q = 1ull << (d.mu - round);
  a.round = round;
  a.mu = d.mu;
  a.nparts = nparts;
  a.partials = d.partials;
  a.ctrl = d.ctrl;
  a.evals_out = d.evals + (uint64_t)(round - 1) * d.ne * 8;
  a.alpha_out = d.alphas + (uint64_t)(round - 1) * 8;
  a.tail = round == d.last ? 1u : 0u;
  a.openings = d.openings;
  a.eq = d.eq;
  a.check = d.flags & 1u;
  return a;
}

// Index i with pre(i) <= b < pre(i+1) (pre(0) = 0, n() >= 1).
template <class Step>
__device__ __forceinline__ uint32_t batch_find(const Step& st, uint32_t b) {
  uint32_t lo = 0, hi = st.n();
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (st.pre(mid) <= b) lo = mid; else hi = mid;
  }
  return lo;
}

template <class Gate, bool FOLD, class Step>
__device__ __forceinline__ void batch_round_body(const Step& st) {
  const uint32_t i = batch_find(st, blockIdx.x);
  const InstDesc& d = st.desc(i);
  const uint32_t round = st.round(i);
  const uint32_t p0 = st.pre(i), nb = st.pre(i + 1) - p0;  // this launch's blocks of the round
  const uint32_t nblk = nb * st.parts(i);                   // all the round's blocks
  const RoundArgs a = batch_round_args(d, round, nblk);
  round_body<Gate, FOLD>(a, round <= 2 ? d.orig : d.fold, round == 1 ? d.orig : d.fold,
                         blockIdx.x - p0 + st.part(i) * nb, nblk);
}

template <class Gate, class Step>
__device__ __forceinline__ void batch_finish_body(const Step& st) {
  const InstDesc& d = st.desc(blockIdx.x);
  const uint32_t round = st.round(blockIdx.x);
  const RoundArgs a =
      batch_round_args(d, round, (st.pre(blockIdx.x + 1) - st.pre(blockIdx.x)) * st.parts(blockIdx.x));
  finish_body<Gate>(a, round == 1 ? d.orig : d.fold);
}

template <class Gate, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_batch_round(BatchStep bs) {
  batch_round_body<Gate, FOLD>(bs);
}

template <class Gate>
__global__ __launch_bounds__(kBlock) void k_batch_finish(BatchStep bs) {
  batch_finish_body<Gate>(bs);
}

template <class Gate, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_serve_round(ServeStep ss) {
  batch_round_body<Gate, FOLD>(ss);
}

template <class Gate>
__global__ __launch_bounds__(kBlock) void k_serve_finish(ServeStep ss) {
  batch_finish_body<Gate>(ss);
}

}  // namespace zc
