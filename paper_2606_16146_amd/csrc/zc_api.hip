// Host side of the C ABI declared in include/zc.h: argument checks,
// workspace layout and the launch sequence of a proof.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/zc.h"
#include "../../include/zc_testing.h"
#include "zc_kernels.h"
#include "zc_launch.h"
#include "zc_misc_kernels.h"

using namespace zc;

// Workspace of zc_prove_static (see static_scratch below): one copy per
// device, held for the life of the process.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t zc_static_scratch[kStaticScratchBytes];

namespace {

struct Layout {
  uint32_t k;       // witness tables
  uint32_t d;       // gate degree
  uint32_t ml, mh;  // split of the variables for the factored eq tables
  size_t eqrows, partials, specparts, scratch, total;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Table 1 shapes g1..gP + gP+1..gP+A, m = P + 16 A; index in the gate keys.
constexpr uint32_t kSumCodes[6] = {2, 18, 34, 50, 3, 4};

int sum_index(uint32_t m) {
  for (int i = 0; i < 6; ++i)
    if (kSumCodes[i] == m) return i;
  return -1;
}

int shape_k(const zc_shape* s) {
  if (!s) return ZC_EINVAL;
  if (s->gate == ZC_GATE_VANILLA) return 8;
  if (s->gate == ZC_GATE_PROD) return (s->m >= 1 && s->m <= 8) ? (int)s->m + 2 : ZC_EUNSUPPORTED;
  if (s->gate == ZC_GATE_SUMPROD) return sum_index(s->m) >= 0 ? (int)((s->m & 15) + (s->m >> 4)) : ZC_EUNSUPPORTED;
  return ZC_EUNSUPPORTED;
}

int shape_d(const zc_shape* s) {
  const int k = shape_k(s);
  if (k < 0) return k;
  if (s->gate == ZC_GATE_VANILLA) return 3;
  if (s->gate == ZC_GATE_SUMPROD) return (int)(s->m & 15);
  return (int)s->m + 1;
}

int make_layout(const zc_shape* s, Layout* L) {
  const int k = shape_k(s);
  if (k < 0) return k;
  if (s->mu < 1 || s->mu > (uint32_t)kMuMax ||
      (s->flags & ~(uint32_t)(ZC_FLAG_CHECK_CLAIMS | ZC_FLAG_SHARED_GPU | ZC_FLAG_ASSUME_SATISFIED)))
    return ZC_EINVAL;
  L->k = (uint32_t)k;
  L->d = (uint32_t)shape_d(s);
  L->ml = s->mu / 2;
  L->mh = s->mu - L->ml;
  const size_t n = (size_t)1 << s->mu;
  size_t off = align256(kCtrlBytes + kEq1Bytes);  // control block, then the eq1 rows
  L->eqrows = off;  // LO (2^ml rows) + HI heap (2^mh) + SUF heap (2^(ml+1)), 32 bytes each
  off = align256(off + (((size_t)1 << L->ml) + ((size_t)1 << L->mh) + ((size_t)2 << L->ml)) * 32);
  L->partials = off;
  off = align256(off + (size_t)kMaxBlocks * kPartStrideMax * 32);
  L->specparts = off;  // two buffers of speculative partial sums (kSpecBlocks x kGroup values)
  off = align256(off + 2 * (size_t)kSpecBlocks * 16 * 32);
  L->scratch = off;  // folded copies of the k witness tables, 2^(mu-1) entries each
  off = align256(off + (size_t)k * (n / 2 > 0 ? n / 2 : 1) * 32);
  L->total = off;
  return ZC_OK;
}

// Largest table (mu = kMuMax): element indices stay below 2^30, so the
// kernels' 32-bit byte offsets (4 j) cannot wrap.
constexpr uint64_t kMaxElems = 1ull << kMuMax;
static_assert(kMuMax <= 30, "element byte offsets are 32-bit");

inline uint32_t grid_for(uint64_t work, uint32_t cap) {
  uint64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (uint32_t)(b < cap ? b : cap);
}

inline int launch_ok() { return hipGetLastError() == hipSuccess ? ZC_OK : ZC_EHIP; }

inline Ctrl* ctrl_of(void* ws) { return reinterpret_cast<Ctrl*>(ws); }
inline uint8_t* bytes(void* ws) { return reinterpret_cast<uint8_t*>(ws); }

int dispatch_round(const zc_shape* s, bool fold, RoundKind kind, const RoundArgs& a, const TabPtrs& src,
                   const TabPtrs& dst, hipStream_t st, hipEvent_t after = nullptr) {
  if (s->gate == ZC_GATE_VANILLA) return launch_round_vanilla(fold, kind, a, src, dst, st, after);
  if (s->gate == ZC_GATE_SUMPROD) {
    switch (s->m) {
      case 2: return launch_round_sum2(fold, kind, a, src, dst, st, after);
      case 18: return launch_round_sum18(fold, kind, a, src, dst, st, after);
      case 34: return launch_round_sum34(fold, kind, a, src, dst, st, after);
      case 50: return launch_round_sum50(fold, kind, a, src, dst, st, after);
      case 3: return launch_round_sum3(fold, kind, a, src, dst, st, after);
      case 4: return launch_round_sum4(fold, kind, a, src, dst, st, after);
      default: return ZC_EUNSUPPORTED;
    }
  }
  switch (s->m) {
    case 1: return launch_round_prod1(fold, kind, a, src, dst, st, after);
    case 2: return launch_round_prod2(fold, kind, a, src, dst, st, after);
    case 3: return launch_round_prod3(fold, kind, a, src, dst, st, after);
    case 4: return launch_round_prod4(fold, kind, a, src, dst, st, after);
    case 5: return launch_round_prod5(fold, kind, a, src, dst, st, after);
    case 6: return launch_round_prod6(fold, kind, a, src, dst, st, after);
    case 7: return launch_round_prod7(fold, kind, a, src, dst, st, after);
    case 8: return launch_round_prod8(fold, kind, a, src, dst, st, after);
    default: return ZC_EUNSUPPORTED;
  }
}

int dispatch_spec(const zc_shape* s, SpecStep step, const RoundArgs& fa, const TabPtrs& fdst, const RoundArgs& sa,
                  const TabPtrs& src, const TabPtrs& dst, hipStream_t st, uint32_t* blocks) {
  if (s->gate == ZC_GATE_VANILLA) return launch_spec_vanilla(step, fa, fdst, sa, src, dst, st, blocks);
  if (s->gate == ZC_GATE_SUMPROD) {
    switch (s->m) {
      case 2: return launch_spec_sum2(step, fa, fdst, sa, src, dst, st, blocks);
      case 18: return launch_spec_sum18(step, fa, fdst, sa, src, dst, st, blocks);
      case 34: return launch_spec_sum34(step, fa, fdst, sa, src, dst, st, blocks);
      case 50: return launch_spec_sum50(step, fa, fdst, sa, src, dst, st, blocks);
      case 3: return launch_spec_sum3(step, fa, fdst, sa, src, dst, st, blocks);
      case 4: return launch_spec_sum4(step, fa, fdst, sa, src, dst, st, blocks);
      default: return ZC_EUNSUPPORTED;
    }
  }
  switch (s->m) {
    case 1: return launch_spec_prod1(step, fa, fdst, sa, src, dst, st, blocks);
    case 2: return launch_spec_prod2(step, fa, fdst, sa, src, dst, st, blocks);
    case 3: return launch_spec_prod3(step, fa, fdst, sa, src, dst, st, blocks);
    case 4: return launch_spec_prod4(step, fa, fdst, sa, src, dst, st, blocks);
    case 5: return launch_spec_prod5(step, fa, fdst, sa, src, dst, st, blocks);
    case 6: return launch_spec_prod6(step, fa, fdst, sa, src, dst, st, blocks);
    case 7: return launch_spec_prod7(step, fa, fdst, sa, src, dst, st, blocks);
    case 8: return launch_spec_prod8(step, fa, fdst, sa, src, dst, st, blocks);
    default: return ZC_EUNSUPPORTED;
  }
}

RoundArgs round_args(const zc_shape* s, const Layout& L, void* ws, uint32_t i,
                     uint32_t* round_evals, uint32_t* challenges) {
  RoundArgs a{};
  a.q = 1ull << (s->mu - i);
  a.round = i;
  a.mu = s->mu;
  a.partials = reinterpret_cast<uint32_t*>(bytes(ws) + L.partials);
  a.ctrl = ctrl_of(ws);
  a.evals_out = round_evals + (uint64_t)(i - 1) * (L.d + 2) * 8;
  a.alpha_out = challenges + (uint64_t)(i - 1) * 8;
  const uint32_t* rows = reinterpret_cast<const uint32_t*>(bytes(ws) + L.eqrows);
  a.eq.lo = rows;
  a.eq.hi = rows + ((size_t)1 << L.ml) * 8;
  a.eq.suf = rows + (((size_t)1 << L.ml) + ((size_t)1 << L.mh)) * 8;
  a.eq.ml = L.ml;
  a.eq.mh = L.mh;
  a.eq.mu = s->mu;
  a.check = (s->flags & ZC_FLAG_CHECK_CLAIMS) ? 1u : 0u;
  a.share = (s->flags & ZC_FLAG_SHARED_GPU) ? 1u : 0u;
  a.skip01 = (i == 1 && (s->flags & ZC_FLAG_ASSUME_SATISFIED)) ? 1u : 0u;
  return a;
}

// One launch: r -> canonical and Montgomery copies, C_1, coef_1 and the eq1
// rows, the factored eq tables, and T_0.
int launch_setup(const zc_shape* s, const Layout& L, const uint32_t* r, void* ws, hipStream_t st) {
  Ctrl* ctrl = ctrl_of(ws);
  const uint32_t nrows = (1u << L.ml) + (1u << L.mh) + (2u << L.ml);
  uint32_t* rows = reinterpret_cast<uint32_t*>(bytes(ws) + L.eqrows);
  const uint32_t grid = 1 + (nrows + kBlock - 1) / kBlock + 1;
  hipLaunchKernelGGL(k_setup_eq, dim3(grid), dim3(kBlock), 0, st, ctrl, r, s->mu, s->gate, s->m, L.ml, L.d + 2, rows);
  return launch_ok();
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int check_tables(const Layout& L, const uint32_t* const* tables) {
  if (!tables) return ZC_EINVAL;
  for (uint32_t t = 0; t < L.k; ++t)
    if (!tables[t] || !aligned(tables[t], 4)) return ZC_EINVAL;
  return ZC_OK;
}

// Whole proof.  With `ev` (2*mu events) the round kernel of round i (not its
// finisher) is bracketed by ev[2(i-1)] and ev[2(i-1)+1] on the same stream.
int prove_impl(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws,
               uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, hipStream_t stream,
               hipEvent_t* ev, uint64_t pitch = 0) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!r || !ws || !round_evals || !challenges || !openings || !aligned(ws, 256)) return ZC_EINVAL;
  const uint32_t mu = shape->mu;
  const uint64_t n = 1ull << mu;
  if (pitch != 0 && (pitch < n || pitch > kMaxElems)) return ZC_EINVAL;
  const uint64_t tp = pitch ? pitch : n;  // plane pitch of the caller's tables
  uint32_t* scratch = reinterpret_cast<uint32_t*>(bytes(ws) + L.scratch);
  const uint64_t half = n / 2;

  TabPtrs orig{}, fold{};
  for (uint32_t t = 0; t < L.k; ++t) {
    orig.p[t] = const_cast<uint32_t*>(tables[t]);
    fold.p[t] = scratch + (uint64_t)t * half * 8;
  }

  if ((rc = launch_setup(shape, L, r, ws, stream)) != ZC_OK) return rc;
  const SpecPlan sp = spec_plan(mu, L.d);
  uint32_t* spec_buf[2] = {reinterpret_cast<uint32_t*>(bytes(ws) + L.specparts),
                           reinterpret_cast<uint32_t*>(bytes(ws) + L.specparts) + (size_t)kSpecBlocks * 16 * 8};
  uint32_t prev_blocks = 0;      // partial-sum blocks of the previous launch (speculative schedule)
  uint32_t* prev_parts = nullptr;
  // The folded tables the next round reads.  A thread-per-pair round from
  // round 3 on folds in place, except in its two-wave form (small enough,
  // kHalfQ), which runs out of place: it reads entries [0, 4q) of each folded
  // table and writes [4q, 6q), and the later rounds continue from there
  // (coff: that offset from the start of the folded tables).
  TabPtrs cur = fold;
  uint64_t coff = 0;
  const uint64_t hq = shape->gate == ZC_GATE_VANILLA ? kHalfQVanilla : kHalfQ;
  auto moved = [&](uint64_t q) {
    TabPtrs d = cur;
    if (coff + 6 * q <= half) {
      for (uint32_t t = 0; t < L.k; ++t) d.p[t] = cur.p[t] + 4 * q;
      coff += 4 * q;
    }
    return d;
  };
  for (uint32_t i = 1; i <= mu; ++i) {
    const RoundKind kind = prove_round_kind(mu, i, L.d);
    if (sp.on && (i + 1 == sp.s0 || kind == kSpec || kind == kSpecTail)) {
      // round s0-1 without its finisher, then for i = s0..r the finisher of
      // round i-1 beside the speculative round i, then round r's finisher
      // with the tail (tables: the folded copies, T_{i-1} or T_{i-2})
      RoundArgs sa = round_args(shape, L, ws, i, round_evals, challenges);
      sa.src_pitch = i <= 2 ? tp : half;
      sa.dst_pitch = half;
      if (ev && hipEventRecord(ev[2 * (i - 1)], stream) != hipSuccess) return ZC_EHIP;
      uint32_t blocks = 0;
      if (i + 1 == sp.s0) {
        const TabPtrs src = i <= 2 ? orig : cur;
        if (i >= 3 && sa.q <= hq) cur = moved(sa.q);
        rc = dispatch_spec(shape, kSpecRoundOnly, sa, cur, sa, src, cur, stream, &blocks);
        prev_parts = sa.partials;
      } else {
        RoundArgs fa = round_args(shape, L, ws, i - 1, round_evals, challenges);
        fa.nparts = prev_blocks;
        fa.partials = prev_parts;
        sa.partials = spec_buf[i & 1];
        sa.src_pitch = sa.dst_pitch = half;
        rc = dispatch_spec(shape, i == sp.s0 ? kSpecFirst : kSpecNext, fa, cur, sa, cur, cur, stream, &blocks);
        prev_parts = sa.partials;
      }
      if (rc != ZC_OK) return rc;
      if (ev && hipEventRecord(ev[2 * (i - 1) + 1], stream) != hipSuccess) return ZC_EHIP;
      prev_blocks = blocks;
      if (kind == kSpecTail) {
        RoundArgs fa = round_args(shape, L, ws, i, round_evals, challenges);
        fa.nparts = prev_blocks;
        fa.partials = prev_parts;
        fa.tail = 1;
        fa.openings = openings;
        fa.src_pitch = fa.dst_pitch = half;
        if ((rc = dispatch_spec(shape, kSpecFinishTail, fa, cur, fa, cur, cur, stream, &blocks)) != ZC_OK) return rc;
      }
      continue;
    }
    if (kind == kInTail) {  // evaluated inside the tail of an earlier launch
      if (ev && (hipEventRecord(ev[2 * (i - 1)], stream) != hipSuccess ||
                 hipEventRecord(ev[2 * (i - 1) + 1], stream) != hipSuccess))
        return ZC_EHIP;
      continue;
    }
    RoundArgs a = round_args(shape, L, ws, i, round_evals, challenges);
    a.openings = openings;
    a.src_pitch = i <= 2 ? tp : half;
    a.dst_pitch = i == 1 ? tp : half;
    const TabPtrs src = i <= 2 ? orig : cur;
    if (i >= 3 && kind == kPerPair && a.q <= hq) cur = moved(a.q);
    const TabPtrs dst = i == 1 ? orig : cur;
    if (ev && hipEventRecord(ev[2 * (i - 1)], stream) != hipSuccess) return ZC_EHIP;
    if ((rc = dispatch_round(shape, i > 1, kind, a, src, dst, stream, ev ? ev[2 * (i - 1) + 1] : nullptr)) != ZC_OK)
      return rc;
  }
  return ZC_OK;
}

// ---- batches -----------------------------------------------------------------

// setup of instance blockIdx.y: setup_body in x block 0, T_0 in the last x
// block, its eq rows in between
__global__ __launch_bounds__(kBlock) void k_batch_setup_eq(const InstDesc* __restrict__ descs) {
  const InstDesc& d = descs[blockIdx.y];
  if (blockIdx.x == 0)
    setup_body(d.r, d.mu, d.ne, d.ctrl);
  else if (blockIdx.x == gridDim.x - 1)
    t0_body(d.r, d.mu, d.gate, d.m, d.ctrl);
  else
    eq_row_body(d.r, d.mu, d.eq.ml, const_cast<uint32_t*>(d.eq.lo), (blockIdx.x - 1) * blockDim.x + threadIdx.x);
}

constexpr uint32_t kBatchMax = 65536;
constexpr uint32_t kGateKeys = 15;  // 0 vanilla, 1..8 product gate m, 9..14 the Table 1 shapes

// Host-side schedule of a batch, recomputed identically by upload and launch.
struct BatchSeg {
  uint32_t key, step, count, blocks;
  bool tail;
  size_t inst_off, prefix_off;  // in u32 words within the schedule array
};

struct BatchPlan {
  std::vector<Layout> L;
  std::vector<uint32_t> last;
  std::vector<BatchSeg> segs;
  std::vector<uint32_t> words;  // the schedule array (instance lists, block prefixes)
  uint32_t max_eq_rows = 0;
};

size_t desc_bytes(uint32_t n) { return align256((size_t)n * sizeof(InstDesc)); }

size_t sched_words_max(uint32_t n) { return (size_t)kMuMax * (2 * (size_t)n + kGateKeys); }

uint32_t gate_key(const zc_shape& s) {
  if (s.gate == ZC_GATE_VANILLA) return 0u;
  if (s.gate == ZC_GATE_SUMPROD) return 9u + (uint32_t)sum_index(s.m);
  return s.m;
}

int check_instance(const zc_instance& in, Layout* L) {
  int rc = make_layout(&in.shape, L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(*L, in.tables)) != ZC_OK) return rc;
  if (!in.r || !in.ws || !in.round_evals || !in.challenges || !in.openings || !aligned(in.ws, 256))
    return ZC_EINVAL;
  if (in.pitch != 0 && (in.pitch < (1ull << in.shape.mu) || in.pitch > kMaxElems)) return ZC_EINVAL;
  return ZC_OK;
}

int make_plan(uint32_t n, const zc_instance* inst, BatchPlan* P) {
  if (!inst || n < 1 || n > kBatchMax) return ZC_EINVAL;
  P->L.resize(n);
  P->last.resize(n);
  uint32_t steps = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const int rc = check_instance(inst[i], &P->L[i]);
    if (rc != ZC_OK) return rc;
    const uint32_t mu = inst[i].shape.mu;
    // the first round with at most 2 kTailQ pairs launches the tail
    P->last[i] = mu <= 6 ? 1u : mu - 6;
    steps = std::max(steps, P->last[i]);
    const Layout& L = P->L[i];
    P->max_eq_rows = std::max(P->max_eq_rows, (1u << L.ml) + (1u << L.mh) + (2u << L.ml));
  }
  for (uint32_t s = 0; s < steps; ++s) {
    for (uint32_t key = 0; key < kGateKeys; ++key) {
      BatchSeg g{key, s, 0, 0, false, P->words.size(), 0};
      std::vector<uint32_t> prefix{0};
      for (uint32_t i = 0; i < n; ++i) {
        if (gate_key(inst[i].shape) != key || s + 1 > P->last[i]) continue;
        const uint64_t q = 1ull << (inst[i].shape.mu - (s + 1));
        const uint64_t tile = inst[i].tile ? inst[i].tile : 4;
        uint64_t b = (q + kBlock * tile - 1) / (kBlock * tile);
        b = std::min<uint64_t>(std::max<uint64_t>(b, 1), kMaxBlocks);
        P->words.push_back(i);
        prefix.push_back(prefix.back() + (uint32_t)b);
        if (s + 1 == P->last[i]) g.tail = true;
        ++g.count;
      }
      if (g.count == 0) {
        P->words.resize(g.inst_off);
        continue;
      }
      g.blocks = prefix.back();
      g.prefix_off = P->words.size();
      P->words.insert(P->words.end(), prefix.begin(), prefix.end());
      P->segs.push_back(g);
    }
  }
  return P->words.size() <= sched_words_max(n) ? ZC_OK : ZC_EINVAL;
}

InstDesc make_desc(const zc_instance& in, const Layout& L, uint32_t last) {
  InstDesc d{};
  const uint64_t n = 1ull << in.shape.mu, half = n / 2;
  uint8_t* w = bytes(in.ws);
  for (uint32_t t = 0; t < L.k; ++t) {
    d.orig.p[t] = const_cast<uint32_t*>(in.tables[t]);
    d.fold.p[t] = reinterpret_cast<uint32_t*>(w + L.scratch) + (uint64_t)t * half * 8;
  }
  const uint32_t* rows = reinterpret_cast<const uint32_t*>(w + L.eqrows);
  d.eq.lo = rows;
  d.eq.hi = rows + ((size_t)1 << L.ml) * 8;
  d.eq.suf = rows + (((size_t)1 << L.ml) + ((size_t)1 << L.mh)) * 8;
  d.eq.ml = L.ml;
  d.eq.mh = L.mh;
  d.eq.mu = in.shape.mu;
  d.ctrl = ctrl_of(in.ws);
  d.partials = reinterpret_cast<uint32_t*>(w + L.partials);
  d.evals = in.round_evals;
  d.alphas = in.challenges;
  d.openings = in.openings;
  d.r = in.r;
  d.mu = in.shape.mu;
  d.gate = in.shape.gate;
  d.m = in.shape.m;
  d.ne = L.d + 2;
  d.last = last;
  d.pitch = in.pitch ? in.pitch : n;
  d.flags = in.shape.flags;
  return d;
}

int launch_batch_key(uint32_t key, const BatchStep& bs, uint32_t blocks, bool fold, bool tail, hipStream_t st) {
  switch (key) {
    case 0: return launch_batch_vanilla(bs, blocks, fold, tail, st);
    case 1: return launch_batch_prod1(bs, blocks, fold, tail, st);
    case 2: return launch_batch_prod2(bs, blocks, fold, tail, st);
    case 3: return launch_batch_prod3(bs, blocks, fold, tail, st);
    case 4: return launch_batch_prod4(bs, blocks, fold, tail, st);
    case 5: return launch_batch_prod5(bs, blocks, fold, tail, st);
    case 6: return launch_batch_prod6(bs, blocks, fold, tail, st);
    case 7: return launch_batch_prod7(bs, blocks, fold, tail, st);
    case 8: return launch_batch_prod8(bs, blocks, fold, tail, st);
    case 9: return launch_batch_sum2(bs, blocks, fold, tail, st);
    case 10: return launch_batch_sum18(bs, blocks, fold, tail, st);
    case 11: return launch_batch_sum34(bs, blocks, fold, tail, st);
    case 12: return launch_batch_sum50(bs, blocks, fold, tail, st);
    case 13: return launch_batch_sum3(bs, blocks, fold, tail, st);
    case 14: return launch_batch_sum4(bs, blocks, fold, tail, st);
    default: return ZC_EUNSUPPORTED;
  }
}

// ---- serving -------------------------------------------------------------------

constexpr uint32_t kServeSlots = 65535;  // slot ids travel as u16
constexpr uint32_t kServeMaxParts = 64;   // launches one round of zc_serve_step_part may be split into

// admission of one instance: its descriptor into the pool and setup_body in
// block 0, T_0 in the last block, the eq rows in between
__global__ __launch_bounds__(kBlock) void k_serve_setup_eq(InstDesc* __restrict__ pool, uint32_t slot, InstDesc d) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) pool[slot] = d;
    setup_body(d.r, d.mu, d.ne, d.ctrl);
  } else if (blockIdx.x == gridDim.x - 1) {
    t0_body(d.r, d.mu, d.gate, d.m, d.ctrl);
  } else {
    eq_row_body(d.r, d.mu, d.eq.ml, const_cast<uint32_t*>(d.eq.lo), (blockIdx.x - 1) * blockDim.x + threadIdx.x);
  }
}

// ---- the proof that allocates nothing ----------------------------------------
//
// zc_prove_static runs zc_prove with the workspace in this file-scope device
// array instead of a caller buffer.  Each device the library runs on holds
// its own copy (kStaticScratchBytes) for the life of the process.  The name
// is only a host-side stand-in for the array: its device address is asked
// once per device with hipGetSymbolAddress and that address is what the
// kernels receive.

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices];

// Device address of zc_static_scratch on the stream's device (the current
// device for the null stream).
int static_scratch(hipStream_t stream, void** out) {
  int dev = 0;
  if (stream) {
    if (hipStreamGetDevice(stream, &dev) != hipSuccess) return ZC_EHIP;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return ZC_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return ZC_EHIP;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return ZC_EHIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return ZC_EHIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(zc_static_scratch));
    if (cur != dev && hipSetDevice(cur) != hipSuccess) return ZC_EHIP;
    if (e != hipSuccess || !p) return ZC_EHIP;
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return ZC_OK;
}

// Copies the device-detected status of a proof out of its control block.
__global__ void k_status_out(const Ctrl* ctrl, int32_t* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *status = (int32_t)ctrl->err;
}

uint32_t last_round(uint32_t mu) { return mu <= 6 ? 1u : mu - 6; }

uint32_t tile_blocks(uint32_t mu, uint32_t round, uint32_t tile) {
  const uint64_t q = 1ull << (mu - round);
  const uint64_t t = tile ? tile : 4;
  const uint64_t b = (q + kBlock * t - 1) / (kBlock * t);
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(b, 1), kMaxBlocks);
}

int launch_serve_key(uint32_t key, const ServeStep& ss, uint32_t blocks, bool fold, bool tail, hipStream_t st) {
  switch (key) {
    case 0: return launch_serve_vanilla(ss, blocks, fold, tail, st);
    case 1: return launch_serve_prod1(ss, blocks, fold, tail, st);
    case 2: return launch_serve_prod2(ss, blocks, fold, tail, st);
    case 3: return launch_serve_prod3(ss, blocks, fold, tail, st);
    case 4: return launch_serve_prod4(ss, blocks, fold, tail, st);
    case 5: return launch_serve_prod5(ss, blocks, fold, tail, st);
    case 6: return launch_serve_prod6(ss, blocks, fold, tail, st);
    case 7: return launch_serve_prod7(ss, blocks, fold, tail, st);
    case 8: return launch_serve_prod8(ss, blocks, fold, tail, st);
    case 9: return launch_serve_sum2(ss, blocks, fold, tail, st);
    case 10: return launch_serve_sum18(ss, blocks, fold, tail, st);
    case 11: return launch_serve_sum34(ss, blocks, fold, tail, st);
    case 12: return launch_serve_sum50(ss, blocks, fold, tail, st);
    case 13: return launch_serve_sum3(ss, blocks, fold, tail, st);
    case 14: return launch_serve_sum4(ss, blocks, fold, tail, st);
    default: return ZC_EUNSUPPORTED;
  }
}

}  // namespace

extern "C" {

int zc_table_count(const zc_shape* shape) { return shape_k(shape); }

int zc_degree(const zc_shape* shape) { return shape_d(shape); }

size_t zc_workspace_bytes(const zc_shape* shape) {
  Layout L;
  return make_layout(shape, &L) == ZC_OK ? L.total : 0;
}

int zc_pack(const uint32_t* canon, uint32_t* mont_planar, uint64_t n, void* ws, hipStream_t stream) {
  if (!canon || !mont_planar || !ws || n == 0 || n > kMaxElems || !aligned(canon, 16) || !aligned(ws, 256))
    return ZC_EINVAL;
  hipLaunchKernelGGL(k_pack, dim3(grid_for(n, 8192)), dim3(kBlock), 0, stream, canon, mont_planar, n, n,
                     ctrl_of(ws));
  return launch_ok();
}

int zc_unpack(const uint32_t* mont_planar, uint64_t pitch, uint32_t* canon, uint64_t n, hipStream_t stream) {
  if (!canon || !mont_planar || n == 0 || n > kMaxElems || pitch < n || !aligned(canon, 16)) return ZC_EINVAL;
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(n, 8192)), dim3(kBlock), 0, stream, mont_planar, pitch, canon, n);
  return launch_ok();
}

int zc_prove(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws,
             uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, hipStream_t stream) {
  return prove_impl(shape, tables, r, ws, round_evals, challenges, openings, stream, nullptr);
}

int zc_prove_pitch(const zc_shape* shape, const uint32_t* const* tables, uint64_t pitch, const uint32_t* r, void* ws,
                   uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, hipStream_t stream) {
  return prove_impl(shape, tables, r, ws, round_evals, challenges, openings, stream, nullptr, pitch);
}

int zc_prove_static(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, uint32_t* round_evals,
                    uint32_t* challenges, uint32_t* openings, int32_t* status, hipStream_t stream) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if (L.total > kStaticScratchBytes) return ZC_ETOOBIG;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!r || !round_evals || !challenges || !openings) return ZC_EINVAL;
  void* ws = nullptr;
  if ((rc = static_scratch(stream, &ws)) != ZC_OK) return rc;
  if ((rc = prove_impl(shape, tables, r, ws, round_evals, challenges, openings, stream, nullptr)) != ZC_OK)
    return rc;
  if (status) {
    hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, stream, ctrl_of(ws), status);
    return launch_ok();
  }
  return ZC_OK;
}

int zc_prove_profiled(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws,
                      uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, void* events,
                      hipStream_t stream) {
  if (!events) return ZC_EINVAL;
  return prove_impl(shape, tables, r, ws, round_evals, challenges, openings, stream,
                    reinterpret_cast<hipEvent_t*>(events));
}

int zc_round(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws, uint32_t i,
             uint32_t* round_evals, uint32_t* challenges, hipStream_t stream) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!ws || !round_evals || !challenges || !aligned(ws, 256) || i < 1 || i > shape->mu) return ZC_EINVAL;
  if (i == 1 && !r) return ZC_EINVAL;
  const uint64_t n = 1ull << shape->mu;
  Ctrl* ctrl = ctrl_of(ws);
  TabPtrs cur{};
  for (uint32_t t = 0; t < L.k; ++t) cur.p[t] = const_cast<uint32_t*>(tables[t]);
  if (i == 1) {
    if ((rc = launch_setup(shape, L, r, ws, stream)) != ZC_OK) return rc;
  } else {
    hipLaunchKernelGGL(k_check_round, dim3(1), dim3(1), 0, stream, ctrl, i);
    if ((rc = launch_ok()) != ZC_OK) return rc;
  }
  RoundArgs a = round_args(shape, L, ws, i, round_evals, challenges);
  a.src_pitch = a.dst_pitch = n;
  return dispatch_round(shape, false, a.q > split_q(L.d) ? kPerPair : kSplit, a, cur, cur, stream);
}

int zc_fold(const zc_shape* shape, uint32_t* const* tables, void* ws, uint32_t i, hipStream_t stream) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!ws || !aligned(ws, 256) || i < 1 || i > shape->mu) return ZC_EINVAL;
  const uint32_t mu = shape->mu;
  const uint64_t n = 1ull << mu, h = 1ull << (mu - i);
  TabPtrs cur{};
  for (uint32_t t = 0; t < L.k; ++t) cur.p[t] = tables[t];
  Ctrl* ctrl = ctrl_of(ws);
  hipLaunchKernelGGL(k_fold, dim3(grid_for(h, 1024), L.k), dim3(kBlock), 0, stream, cur, L.k, n, h, ctrl, i);
  if ((rc = launch_ok()) != ZC_OK) return rc;
  hipLaunchKernelGGL(k_mark_folded, dim3(1), dim3(1), 0, stream, ctrl, i);
  return launch_ok();
}

size_t zc_batch_workspace_bytes(uint32_t n) {
  if (n < 1 || n > kBatchMax) return 0;
  return desc_bytes(n) + align256(sched_words_max(n) * sizeof(uint32_t));
}

int zc_batch_upload(uint32_t n, const zc_instance* inst, void* batch_ws, hipStream_t stream) {
  if (!batch_ws || !aligned(batch_ws, 256)) return ZC_EINVAL;
  BatchPlan P;
  const int rc = make_plan(n, inst, &P);
  if (rc != ZC_OK) return rc;
  std::vector<uint8_t> host(desc_bytes(n) + P.words.size() * sizeof(uint32_t), 0);
  InstDesc* d = reinterpret_cast<InstDesc*>(host.data());
  for (uint32_t i = 0; i < n; ++i) d[i] = make_desc(inst[i], P.L[i], P.last[i]);
  std::copy(P.words.begin(), P.words.end(), reinterpret_cast<uint32_t*>(host.data() + desc_bytes(n)));
  if (hipMemcpyAsync(batch_ws, host.data(), host.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return ZC_EHIP;
  return ZC_OK;
}

int zc_batch_launch(uint32_t n, const zc_instance* inst, void* batch_ws, hipStream_t stream) {
  if (!batch_ws || !aligned(batch_ws, 256)) return ZC_EINVAL;
  BatchPlan P;
  int rc = make_plan(n, inst, &P);
  if (rc != ZC_OK) return rc;
  const InstDesc* descs = reinterpret_cast<const InstDesc*>(batch_ws);
  const uint32_t* words = reinterpret_cast<const uint32_t*>(bytes(batch_ws) + desc_bytes(n));
  hipLaunchKernelGGL(k_batch_setup_eq, dim3((P.max_eq_rows + kBlock - 1) / kBlock + 2, n), dim3(kBlock), 0, stream,
                     descs);
  if ((rc = launch_ok()) != ZC_OK) return rc;
  for (const BatchSeg& g : P.segs) {
    BatchStep bs{descs, words + g.inst_off, words + g.prefix_off, g.count, g.step};
    if ((rc = launch_batch_key(g.key, bs, g.blocks, g.step > 0, g.tail, stream)) != ZC_OK) return rc;
  }
  return ZC_OK;
}

int zc_batch_prove(uint32_t n, const zc_instance* inst, void* batch_ws, hipStream_t stream) {
  const int rc = zc_batch_upload(n, inst, batch_ws, stream);
  return rc != ZC_OK ? rc : zc_batch_launch(n, inst, batch_ws, stream);
}

size_t zc_serve_pool_bytes(uint32_t slots) {
  if (slots < 1 || slots > kServeSlots) return 0;
  return align256((size_t)slots * sizeof(InstDesc));
}

int zc_serve_rounds(const zc_shape* shape) {
  Layout L;
  const int rc = make_layout(shape, &L);
  return rc != ZC_OK ? rc : (int)last_round(shape->mu);
}

int zc_serve_admit(void* pool, uint32_t slots, uint32_t slot, const zc_instance* inst, hipStream_t stream) {
  if (!pool || !inst || !aligned(pool, 256) || slots < 1 || slots > kServeSlots || slot >= slots) return ZC_EINVAL;
  Layout L;
  int rc = check_instance(*inst, &L);
  if (rc != ZC_OK) return rc;
  const InstDesc d = make_desc(*inst, L, last_round(inst->shape.mu));
  const uint32_t nrows = (1u << L.ml) + (1u << L.mh) + (2u << L.ml);
  hipLaunchKernelGGL(k_serve_setup_eq, dim3((nrows + kBlock - 1) / kBlock + 2), dim3(kBlock), 0, stream,
                     reinterpret_cast<InstDesc*>(pool), slot, d);
  return launch_ok();
}

int zc_serve_step(void* pool, uint32_t slots, uint32_t n, const uint32_t* slot_ids, const uint32_t* rounds,
                  const zc_instance* inst, hipStream_t stream) {
  if (!pool || !aligned(pool, 256) || slots < 1 || slots > kServeSlots) return ZC_EINVAL;
  if (n == 0) return ZC_OK;
  if (!slot_ids || !rounds || !inst) return ZC_EINVAL;
  for (uint32_t i = 0; i < n; ++i) {
    Layout L;
    const int rc = make_layout(&inst[i].shape, &L);
    if (rc != ZC_OK) return rc;
    if (slot_ids[i] >= slots || rounds[i] < 1 || rounds[i] > last_round(inst[i].shape.mu)) return ZC_EINVAL;
  }
  // one launch pair per (gate, fold) group and per kServeMax instances
  for (uint32_t key = 0; key < kGateKeys; ++key) {
    for (int fold = 0; fold < 2; ++fold) {
      ServeStep ss{};
      ss.pool = reinterpret_cast<const InstDesc*>(pool);
      bool tail = false;
      auto flush = [&]() -> int {
        if (ss.count == 0) return ZC_OK;
        ss.nfin = ss.count;
        const int rc = launch_serve_key(key, ss, ss.prefix[ss.count], fold != 0, tail, stream);
        ss.count = 0;
        tail = false;
        return rc;
      };
      for (uint32_t i = 0; i < n; ++i) {
        if (gate_key(inst[i].shape) != key || (rounds[i] > 1) != (fold != 0)) continue;
        const uint32_t c = ss.count;
        ss.slot[c] = (uint16_t)slot_ids[i];
        ss.rnd[c] = (uint8_t)rounds[i];
        ss.prt[c] = 0;
        ss.nprt[c] = 1;
        ss.prefix[c + 1] = ss.prefix[c] + tile_blocks(inst[i].shape.mu, rounds[i], inst[i].tile);
        if (rounds[i] == last_round(inst[i].shape.mu)) tail = true;
        if (++ss.count == (uint32_t)kServeMax) {
          const int rc = flush();
          if (rc != ZC_OK) return rc;
        }
      }
      const int rc = flush();
      if (rc != ZC_OK) return rc;
    }
  }
  return ZC_OK;
}

int zc_serve_step_part(void* pool, uint32_t slots, uint32_t slot, uint32_t round, uint32_t part, uint32_t parts,
                       const zc_instance* inst, hipStream_t stream) {
  if (!pool || !aligned(pool, 256) || slots < 1 || slots > kServeSlots || !inst || slot >= slots) return ZC_EINVAL;
  Layout L;
  const int rc = make_layout(&inst->shape, &L);
  if (rc != ZC_OK) return rc;
  const uint32_t last = last_round(inst->shape.mu);
  if (round < 1 || round > last || parts < 1 || parts > kServeMaxParts || part >= parts) return ZC_EINVAL;
  if (round == last && parts != 1) return ZC_EINVAL;  // the round that runs the tail is not split
  const uint32_t b = tile_blocks(inst->shape.mu, round, inst->tile);
  const uint32_t nb = (b + parts - 1) / parts;
  if ((uint64_t)nb * parts > (uint64_t)kMaxBlocks) return ZC_EINVAL;
  ServeStep ss{};
  ss.pool = reinterpret_cast<const InstDesc*>(pool);
  ss.count = 1;
  ss.nfin = part + 1 == parts ? 1u : 0u;
  ss.prefix[0] = 0;
  ss.prefix[1] = nb;
  ss.slot[0] = (uint16_t)slot;
  ss.rnd[0] = (uint8_t)round;
  ss.prt[0] = (uint8_t)part;
  ss.nprt[0] = (uint8_t)parts;
  return launch_serve_key(gate_key(inst->shape), ss, nb, round > 1, round == last, stream);
}

int zc_read_error(void* ws, hipStream_t stream) {
  if (!ws) return ZC_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return ZC_EHIP;
  uint32_t err = 0;
  if (hipMemcpy(&err, &ctrl_of(ws)->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return ZC_EHIP;
  return (int)(int32_t)err;
}

int zc_prove_round_kernel(const zc_shape* shape, uint32_t i) {
  Layout L;
  const int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if (i < 1 || i > shape->mu) return ZC_EINVAL;
  return (int)prove_round_kind(shape->mu, i, L.d);
}

const char* zc_strerror(int status) {
  switch (status) {
    case ZC_OK: return "ok";
    case ZC_EINVAL: return "invalid argument";
    case ZC_EUNSUPPORTED: return "unsupported gate or parameter";
    case ZC_EHIP: return "HIP call or kernel launch failed";
    case ZC_ERANGE: return "input element not below p";
    case ZC_ESTATE: return "zc_round / zc_fold called out of order";
    case ZC_ETOOBIG: return "shape needs more workspace than zc_prove_static holds (32 MiB)";
    case ZC_ECLAIM: return "a round polynomial failed the verifier's claim check (ZC_FLAG_CHECK_CLAIMS)";
    default: return "unknown status";
  }
}

}  // extern "C"
