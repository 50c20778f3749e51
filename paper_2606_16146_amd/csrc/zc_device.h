// Device-side building blocks shared by the prover kernels and the test
// hooks: constants, the workspace control block, element access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr.h"
#include "sha256.h"

namespace zc {

constexpr int kMaxTables = 12;  // witness tables of a gate
constexpr int kMaxEvals = 12;   // d + 2 for d <= 10
constexpr int kMuMax = 30;
constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

// Elements between the partial sums of consecutive blocks of a round kernel
// that stores nv values per block: the power of two >= nv (at most 16).
constexpr uint32_t part_stride(int nv) { return nv <= 1 ? 1u : nv <= 2 ? 2u : nv <= 4 ? 4u : nv <= 8 ? 8u : 16u; }
constexpr uint32_t kPartStrideMax = 16;

// Control block at the start of the workspace.
//
// eq_r is never materialized: it factors as
//   eq_r(a_1..a_{i-1}, X, x_{>i}) = C_i * eq1(X, r_i) * E_i[x_{>i}],
// C_i = prod_{k<i} eq1(alpha_k, r_k), E_i = eq over r_{i+1..mu}, so the
// round kernels accumulate H_i(X) = sum_j E_i[j] f(ext_j(X)) and the round's
// finisher multiplies by coef_i[X] = C_i * eq1(X, r_i).  H_i has degree d, so
// G_i(d+1) comes from H_i(0..d) through lam_k = (-1)^(d-k) C(d+1, k).
//
// coef_{i+1} and C_{i+1} depend on alpha_i only through
// C_{i+1} = C_i eq1(alpha_i, r_i) = C_i (1 - r_i) + alpha_i C_i (2 r_i - 1), so
// the finisher of round i leaves, before its hash, the alpha-free parts
// (nu, nv, npr, nqr below), and the finisher of round i+1 applies alpha_i
// with one product per value at its start, beside its partial-sum loads:
//   coef_{i+1}[l] = nu[l] + mont(alpha_i, nv[l]),  C_{i+1} R = npr + mont(alpha_i, nqr)
// with alpha_i canonical (mont(a, b R) = a b).  Setup leaves the state of
// round 1 (C_1 = 1, no alpha_0: nv = nqr = 0).
constexpr int kMaxCoef = 2 * kMaxEvals - 1;  // slots l: x = l < d+2, then lam_{l-d-2} weights
struct Ctrl {
  uint32_t err;         // first device-detected error (negative status), 0 if none
  uint32_t round_done;  // last round whose challenge has been derived
  uint32_t fold_done;   // last round whose fold has been applied
  uint32_t reserved;
  uint32_t ts[8];                   // transcript digest T_i (little-endian bytes)
  uint32_t alpha[kMuMax][8];        // alpha_i, canonical
  uint32_t nu[kMaxCoef][8];         // C_i (1 - r_i) e_l, canonical (e_l: slot l of r_{i+1}), i = round_done
  uint32_t nv[kMaxCoef][8];         // C_i (2 r_i - 1) e_l R
  uint32_t npr[8];                  // C_i (1 - r_i) R
  uint32_t nqr[8];                  // C_i (2 r_i - 1) R^2
  // Mailbox of a launch whose block 0 finishes round i-1 while its other
  // blocks wait to evaluate round i: word k is (i-1) << 32 | word k of
  // alpha_{i-1}, each written and read as one 64-bit device-coherent
  // (agent-scope) access, so a reader that finds the tag i-1 in all eight
  // words holds the whole challenge, whatever order the words landed in.
  uint64_t mbox[8];
};

constexpr uint32_t kCtrlBytes = 4096;
static_assert(sizeof(Ctrl) <= kCtrlBytes, "control block size");

// The eq1 factors of every round, computed once from r at setup; the
// workspace holds kMuMax of these rows right after the control block.  Row i
// serves the emission of round i+1, which turns C_{i+1} into C_{i+2} and the
// coefficients of round i+2.  With NE = d + 2 and NC = 2d + 3 slots, e_l the
// slot-l factor of r_{i+2} (eq1(x, r_{i+2}) for x = l < NE, else
// eq1(d+1, r_{i+2}) lam_{l-NE}):
constexpr int kEq1Slots = 2 * kMaxEvals - 1;
struct Eq1Row {
  uint32_t u[kEq1Slots][8];  // (1 - r_{i+1}) e_l, canonical (zero in the last row)
  uint32_t v[kEq1Slots][8];  // (2 r_{i+1} - 1) e_l R (zero in the last row)
  uint32_t omr[8];           // (1 - r_{i+1}) R
  uint32_t tr2[8];           // (2 r_{i+1} - 1) R^2
};
constexpr size_t kEq1Bytes = sizeof(Eq1Row) * kMuMax;

__device__ __forceinline__ Eq1Row* eq1_rows(Ctrl* c) {
  return reinterpret_cast<Eq1Row*>(reinterpret_cast<char*>(c) + kCtrlBytes);
}
__device__ __forceinline__ const Eq1Row* eq1_rows(const Ctrl* c) {
  return reinterpret_cast<const Eq1Row*>(reinterpret_cast<const char*>(c) + kCtrlBytes);
}

struct TabPtrs {
  uint32_t* p[kMaxTables];
};

__device__ __forceinline__ void set_error(Ctrl* c, int32_t code) {
  atomicCAS(&c->err, 0u, (uint32_t)code);
}

// ---- limb-planar element access ----------------------------------------------
//
// Limb l of element j lives at base[l * pitch + j].  The plane address
// base + l * pitch is uniform across the wave (scalar registers) and the
// per-lane part is the 32-bit byte offset 4j, so each limb is one
// global_load_dword with a scalar base and a 32-bit vector offset.  Element
// indices are below 2^30 (tables of at most 2^30 entries).

__device__ __forceinline__ const uint32_t* plane_ptr(const uint32_t* base, uint64_t pitch, int l) {
  return base + (uint64_t)l * pitch;
}

// NT: non-temporal access (the line is kept in the caches with low
// priority).  Table data read or written once per round goes this way, so
// that a round's streams do not push out what the next launches use again:
// the finisher's code and control block, the eq tables (measured faster).
template <bool NT = false>
__device__ __forceinline__ void load_words(const uint32_t* __restrict__ base, uint64_t pitch, uint32_t j,
                                           uint32_t w[8]) {
  const uint32_t off = j << 2;
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    const uint32_t* p = reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(plane_ptr(base, pitch, l)) + off);
    if constexpr (NT)
      w[l] = __builtin_nontemporal_load(p);
    else
      w[l] = *p;
  }
}

__device__ __forceinline__ Fe load_el(const uint32_t* __restrict__ base, uint64_t pitch, uint32_t j) {
  uint32_t w[8];
  load_words(base, pitch, j, w);
  return fe_from_words(w);
}

template <bool NT = false>
__device__ __forceinline__ void store_el(uint32_t* __restrict__ base, uint64_t pitch, uint32_t j, const Fe& a) {
  uint32_t w[8];
  fe_to_words(a, w);
  const uint32_t off = j << 2;
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    uint32_t* p = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base + (uint64_t)l * pitch) + off);
    if constexpr (NT)
      __builtin_nontemporal_store(w[l], p);
    else
      *p = w[l];
  }
}

// The two entries (j, j + q) of a table, loaded but not yet converted, so that
// the loads of the next table can be in flight during the current step.
struct RawPair {
  uint32_t w0[8], w1[8];
};

template <bool NT = false>
__device__ __forceinline__ RawPair issue_pair(const uint32_t* __restrict__ base, uint64_t pitch, uint32_t j,
                                              uint32_t q) {
  RawPair r;
  load_words<NT>(base, pitch, j, r.w0);
  load_words<NT>(base, pitch, j + q, r.w1);
  return r;
}

__device__ __forceinline__ Fe load_words_fe(const uint32_t* p) {
  uint32_t w[8];
#pragma unroll
  for (int l = 0; l < 8; ++l) w[l] = p[l];
  return fe_from_words(w);
}

__device__ __forceinline__ void store_words_fe(uint32_t* p, const Fe& a) {
  uint32_t w[8];
  fe_to_words(a, w);
#pragma unroll
  for (int l = 0; l < 8; ++l) p[l] = w[l];
}

}  // namespace zc
