// Host side of the C ABI declared in include/zc.h: argument checks,
// workspace layout and the launch sequence of a proof.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/zc.h"
#include "zc_kernels.h"

using namespace zc;

namespace {

struct Layout {
  uint32_t k;       // witness tables
  uint32_t d;       // gate degree
  uint32_t hb, lb;  // bit split of the eq half tables
  size_t hi, lo, partials, eq, scratch, total;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int shape_k(const zc_shape* s) {
  if (!s) return ZC_EINVAL;
  if (s->gate == ZC_GATE_VANILLA) return 8;
  if (s->gate == ZC_GATE_PROD) return (s->m >= 1 && s->m <= 8) ? (int)s->m + 2 : ZC_EUNSUPPORTED;
  return ZC_EUNSUPPORTED;
}

int shape_d(const zc_shape* s) {
  const int k = shape_k(s);
  if (k < 0) return k;
  return s->gate == ZC_GATE_VANILLA ? 3 : (int)s->m + 1;
}

int make_layout(const zc_shape* s, Layout* L) {
  const int k = shape_k(s);
  if (k < 0) return k;
  if (s->mu < 1 || s->mu > (uint32_t)kMuMax) return ZC_EINVAL;
  L->k = (uint32_t)k;
  L->d = (uint32_t)shape_d(s);
  L->lb = s->mu / 2;
  L->hb = s->mu - L->lb;
  const size_t n = (size_t)1 << s->mu;
  size_t off = kCtrlBytes;
  L->hi = off;
  off = align256(off + ((size_t)32 << L->hb));
  L->lo = off;
  off = align256(off + ((size_t)32 << L->lb));
  L->partials = off;
  off = align256(off + (size_t)kMaxBlocks * kMaxEvals * 32);
  L->eq = off;
  off = align256(off + n * 32);
  L->scratch = off;
  off = align256(off + (size_t)(k + 1) * (n / 2 > 0 ? n / 2 : 1) * 32);
  L->total = off;
  return ZC_OK;
}

inline uint32_t grid_for(uint64_t work, uint32_t cap) {
  uint64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (uint32_t)(b < cap ? b : cap);
}

inline int launch_ok() { return hipGetLastError() == hipSuccess ? ZC_OK : ZC_EHIP; }

inline Ctrl* ctrl_of(void* ws) { return reinterpret_cast<Ctrl*>(ws); }
inline uint8_t* bytes(void* ws) { return reinterpret_cast<uint8_t*>(ws); }

template <class Gate>
int launch_round(bool fold, const TabPtrs& src, const TabPtrs& dst, uint64_t src_pitch, uint64_t dst_pitch,
                 uint64_t q, const uint32_t* alpha, uint32_t* partials, uint32_t* nblocks, hipStream_t st) {
  const uint32_t blocks = grid_for(q, kMaxBlocks);
  *nblocks = blocks;
  if (fold)
    hipLaunchKernelGGL((k_round<Gate, true>), dim3(blocks), dim3(kBlock), 0, st, src, dst, src_pitch, dst_pitch,
                       q, alpha, partials);
  else
    hipLaunchKernelGGL((k_round<Gate, false>), dim3(blocks), dim3(kBlock), 0, st, src, dst, src_pitch,
                       dst_pitch, q, alpha, partials);
  return launch_ok();
}

int dispatch_round(const zc_shape* s, bool fold, const TabPtrs& src, const TabPtrs& dst, uint64_t src_pitch,
                   uint64_t dst_pitch, uint64_t q, const uint32_t* alpha, uint32_t* partials, uint32_t* nblocks,
                   hipStream_t st) {
#define ZC_R(G) launch_round<G>(fold, src, dst, src_pitch, dst_pitch, q, alpha, partials, nblocks, st)
  if (s->gate == ZC_GATE_VANILLA) return ZC_R(GateVanilla);
  switch (s->m) {
    case 1: return ZC_R(GateProd<1>);
    case 2: return ZC_R(GateProd<2>);
    case 3: return ZC_R(GateProd<3>);
    case 4: return ZC_R(GateProd<4>);
    case 5: return ZC_R(GateProd<5>);
    case 6: return ZC_R(GateProd<6>);
    case 7: return ZC_R(GateProd<7>);
    case 8: return ZC_R(GateProd<8>);
    default: return ZC_EUNSUPPORTED;
  }
#undef ZC_R
}

int launch_finish(uint32_t ne, const uint32_t* partials, uint32_t nparts, Ctrl* ctrl, uint32_t round,
                  uint32_t* evals_out, uint32_t* alpha_out, hipStream_t st) {
#define ZC_F(NE)                                                                                              \
  case NE:                                                                                                    \
    hipLaunchKernelGGL(k_finish<NE>, dim3(1), dim3(kBlock), 0, st, partials, nparts, ctrl, round, evals_out, \
                       alpha_out);                                                                            \
    break;
  switch (ne) {
    ZC_F(4) ZC_F(5) ZC_F(6) ZC_F(7) ZC_F(8) ZC_F(9) ZC_F(10) ZC_F(11)
    default: return ZC_EUNSUPPORTED;
  }
#undef ZC_F
  return launch_ok();
}

// r -> Montgomery, T_0, eq half tables, eq table (pitch 2^mu) in ws.
int launch_setup(const zc_shape* s, const Layout& L, const uint32_t* r, void* ws, hipStream_t st) {
  Ctrl* ctrl = ctrl_of(ws);
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, r, s->mu, s->gate, s->m, ctrl);
  if (launch_ok() != ZC_OK) return ZC_EHIP;
  uint32_t* hi = reinterpret_cast<uint32_t*>(bytes(ws) + L.hi);
  uint32_t* lo = reinterpret_cast<uint32_t*>(bytes(ws) + L.lo);
  const uint32_t nhalf = (1u << L.hb) + (1u << L.lb);
  hipLaunchKernelGGL(k_eq_half, dim3((nhalf + kBlock - 1) / kBlock), dim3(kBlock), 0, st, ctrl, s->mu, L.hb, hi,
                     lo);
  if (launch_ok() != ZC_OK) return ZC_EHIP;
  const uint64_t n = 1ull << s->mu;
  uint32_t* eq = reinterpret_cast<uint32_t*>(bytes(ws) + L.eq);
  hipLaunchKernelGGL(k_build_eq, dim3(grid_for(n, 8192)), dim3(kBlock), 0, st, hi, lo, L.lb, n, eq);
  return launch_ok();
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int check_tables(const Layout& L, const uint32_t* const* tables) {
  if (!tables) return ZC_EINVAL;
  for (uint32_t t = 0; t < L.k; ++t)
    if (!tables[t] || !aligned(tables[t], 4)) return ZC_EINVAL;
  return ZC_OK;
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
  if (!canon || !mont_planar || !ws || n == 0 || !aligned(canon, 16) || !aligned(ws, 256)) return ZC_EINVAL;
  hipLaunchKernelGGL(k_pack, dim3(grid_for(n, 8192)), dim3(kBlock), 0, stream, canon, mont_planar, n, n,
                     ctrl_of(ws));
  return launch_ok();
}

int zc_unpack(const uint32_t* mont_planar, uint64_t pitch, uint32_t* canon, uint64_t n, hipStream_t stream) {
  if (!canon || !mont_planar || n == 0 || pitch < n || !aligned(canon, 16)) return ZC_EINVAL;
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(n, 8192)), dim3(kBlock), 0, stream, mont_planar, pitch, canon, n);
  return launch_ok();
}

int zc_prove(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws,
             uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, hipStream_t stream) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!r || !ws || !round_evals || !challenges || !openings || !aligned(ws, 256)) return ZC_EINVAL;
  const uint32_t mu = shape->mu, ne = L.d + 2, K = L.k + 1;
  const uint64_t n = 1ull << mu;
  Ctrl* ctrl = ctrl_of(ws);
  uint32_t* eq = reinterpret_cast<uint32_t*>(bytes(ws) + L.eq);
  uint32_t* partials = reinterpret_cast<uint32_t*>(bytes(ws) + L.partials);
  uint32_t* scratch = reinterpret_cast<uint32_t*>(bytes(ws) + L.scratch);
  const uint64_t half = n / 2;

  TabPtrs orig{}, fold{};
  for (uint32_t t = 0; t < L.k; ++t) orig.p[t] = const_cast<uint32_t*>(tables[t]);
  orig.p[L.k] = eq;
  for (uint32_t t = 0; t < K; ++t) fold.p[t] = scratch + (uint64_t)t * half * 8;

  if ((rc = launch_setup(shape, L, r, ws, stream)) != ZC_OK) return rc;
  for (uint32_t i = 1; i <= mu; ++i) {
    const uint64_t q = 1ull << (mu - i);
    uint32_t nb = 0;
    if (i == 1)
      rc = dispatch_round(shape, false, orig, orig, n, n, q, nullptr, partials, &nb, stream);
    else
      rc = dispatch_round(shape, true, i == 2 ? orig : fold, fold, i == 2 ? n : half, half, q,
                          ctrl->alpha_m[i - 2], partials, &nb, stream);
    if (rc != ZC_OK) return rc;
    rc = launch_finish(ne, partials, nb, ctrl, i, round_evals + (uint64_t)(i - 1) * ne * 8,
                       challenges + (uint64_t)(i - 1) * 8, stream);
    if (rc != ZC_OK) return rc;
  }
  hipLaunchKernelGGL(k_openings, dim3(1), dim3(64), 0, stream, mu == 1 ? orig : fold, K, mu == 1 ? n : half, ctrl,
                     mu, openings);
  return launch_ok();
}

int zc_round(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws, uint32_t i,
             uint32_t* round_evals, uint32_t* challenges, hipStream_t stream) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!ws || !round_evals || !challenges || !aligned(ws, 256) || i < 1 || i > shape->mu) return ZC_EINVAL;
  if (i == 1 && !r) return ZC_EINVAL;
  const uint32_t mu = shape->mu, ne = L.d + 2;
  const uint64_t n = 1ull << mu;
  Ctrl* ctrl = ctrl_of(ws);
  uint32_t* partials = reinterpret_cast<uint32_t*>(bytes(ws) + L.partials);
  TabPtrs cur{};
  for (uint32_t t = 0; t < L.k; ++t) cur.p[t] = const_cast<uint32_t*>(tables[t]);
  cur.p[L.k] = reinterpret_cast<uint32_t*>(bytes(ws) + L.eq);
  if (i == 1) {
    if ((rc = launch_setup(shape, L, r, ws, stream)) != ZC_OK) return rc;
  } else {
    hipLaunchKernelGGL(k_check_round, dim3(1), dim3(1), 0, stream, ctrl, i);
    if ((rc = launch_ok()) != ZC_OK) return rc;
  }
  uint32_t nb = 0;
  rc = dispatch_round(shape, false, cur, cur, n, n, 1ull << (mu - i), nullptr, partials, &nb, stream);
  if (rc != ZC_OK) return rc;
  return launch_finish(ne, partials, nb, ctrl, i, round_evals + (uint64_t)(i - 1) * ne * 8,
                       challenges + (uint64_t)(i - 1) * 8, stream);
}

int zc_fold(const zc_shape* shape, uint32_t* const* tables, void* ws, uint32_t i, hipStream_t stream) {
  Layout L;
  int rc = make_layout(shape, &L);
  if (rc != ZC_OK) return rc;
  if ((rc = check_tables(L, tables)) != ZC_OK) return rc;
  if (!ws || !aligned(ws, 256) || i < 1 || i > shape->mu) return ZC_EINVAL;
  const uint32_t mu = shape->mu, K = L.k + 1;
  const uint64_t n = 1ull << mu, h = 1ull << (mu - i);
  TabPtrs cur{};
  for (uint32_t t = 0; t < L.k; ++t) cur.p[t] = tables[t];
  cur.p[L.k] = reinterpret_cast<uint32_t*>(bytes(ws) + L.eq);
  Ctrl* ctrl = ctrl_of(ws);
  hipLaunchKernelGGL(k_fold, dim3(grid_for(h, 1024), K), dim3(kBlock), 0, stream, cur, K, n, h, ctrl, i);
  if ((rc = launch_ok()) != ZC_OK) return rc;
  hipLaunchKernelGGL(k_mark_folded, dim3(1), dim3(1), 0, stream, ctrl, i);
  return launch_ok();
}

int zc_read_error(void* ws, hipStream_t stream) {
  if (!ws) return ZC_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return ZC_EHIP;
  uint32_t err = 0;
  if (hipMemcpy(&err, &ctrl_of(ws)->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return ZC_EHIP;
  return (int)(int32_t)err;
}

const char* zc_strerror(int status) {
  switch (status) {
    case ZC_OK: return "ok";
    case ZC_EINVAL: return "invalid argument";
    case ZC_EUNSUPPORTED: return "unsupported gate or parameter";
    case ZC_EHIP: return "HIP call or kernel launch failed";
    case ZC_ERANGE: return "input element not below p";
    case ZC_ESTATE: return "zc_round / zc_fold called out of order";
    default: return "unknown status";
  }
}

}  // extern "C"
