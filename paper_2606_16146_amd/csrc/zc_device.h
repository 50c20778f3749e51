// Device-side building blocks shared by the prover kernels and the test
// hooks: constants, the workspace control block, element access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr.h"
#include "sha256.h"

namespace zc {

constexpr int kMaxTables = 12;  // witness tables + eq
constexpr int kMaxEvals = 12;   // d + 2 for d <= 10
constexpr int kMuMax = 30;
constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

// Control block at the start of the workspace.
struct Ctrl {
  uint32_t err;         // first device-detected error (negative status), 0 if none
  uint32_t round_done;  // last round whose challenge has been derived
  uint32_t fold_done;   // last round whose fold has been applied
  uint32_t pad0;
  uint32_t ts[8];                 // transcript digest T_i (little-endian bytes)
  uint32_t alpha_m[kMuMax][8];    // alpha_i, Montgomery form, < p
  uint32_t r_m[kMuMax][8];        // r_i, Montgomery form, < p
  uint32_t pad1[8];
};

constexpr uint32_t kCtrlBytes = 4096;
static_assert(sizeof(Ctrl) <= kCtrlBytes, "control block size");

struct TabPtrs {
  uint32_t* p[kMaxTables];
};

__device__ __forceinline__ void set_error(Ctrl* c, int32_t code) {
  atomicCAS(&c->err, 0u, (uint32_t)code);
}

// ---- limb-planar element access ----------------------------------------------

__device__ __forceinline__ Fe load_el(const uint32_t* __restrict__ base, uint64_t pitch, uint64_t j) {
  uint32_t w[8];
#pragma unroll
  for (int l = 0; l < 8; ++l) w[l] = base[(uint64_t)l * pitch + j];
  return fe_from_words(w);
}

__device__ __forceinline__ void store_el(uint32_t* __restrict__ base, uint64_t pitch, uint64_t j, const Fe& a) {
  uint32_t w[8];
  fe_to_words(a, w);
#pragma unroll
  for (int l = 0; l < 8; ++l) base[(uint64_t)l * pitch + j] = w[l];
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
