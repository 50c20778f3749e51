"""Python binding of libzc (include/zc.h): argument marshalling only.

Every step of a proof runs in the library's HIP kernels; torch provides the
device buffers and the stream.  Tensors are uint32 on the current CUDA
(HIP) device; element arrays are uint32[..][8] canonical little-endian
limbs, packed tables are uint32[8][pitch] limb-planar.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# ZC_LIB may name another build of the library (e.g. to compare two builds).
LIB_PATH = os.environ.get("ZC_LIB") or os.path.join(HERE, "libzc.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ZC_OK, ZC_EINVAL, ZC_EUNSUPPORTED, ZC_EHIP, ZC_ERANGE, ZC_ESTATE, ZC_ETOOBIG, ZC_ECLAIM = 0, -1, -2, -3, -4, -5, -6, -7
ZC_FLAG_CHECK_CLAIMS = 1
ZC_FLAG_SHARED_GPU = 2
ZC_FLAG_ASSUME_SATISFIED = 4
GATE_VANILLA, GATE_PROD, GATE_SUMPROD = 0, 1, 2


class Shape(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_uint32), ("gate", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class Instance(ctypes.Structure):
    """zc_instance: one proof of a batch."""
    _fields_ = [("shape", Shape), ("tables", ctypes.c_void_p), ("r", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("round_evals", ctypes.c_void_p), ("challenges", ctypes.c_void_p),
                ("openings", ctypes.c_void_p), ("tile", ctypes.c_uint32), ("pitch", ctypes.c_uint64)]


class ZcError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status} ({strerror(status)})")
        self.status = status


_lib = None
_VP = ctypes.c_void_p
_SIGS = {
    "zc_table_count": (ctypes.c_int, [ctypes.POINTER(Shape)]),
    "zc_degree": (ctypes.c_int, [ctypes.POINTER(Shape)]),
    "zc_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Shape)]),
    "zc_pack": (ctypes.c_int, [_VP, _VP, ctypes.c_uint64, _VP, _VP]),
    "zc_unpack": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, ctypes.c_uint64, _VP]),
    "zc_prove": (ctypes.c_int, [ctypes.POINTER(Shape), _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "zc_prove_pitch": (ctypes.c_int, [ctypes.POINTER(Shape), _VP, ctypes.c_uint64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "zc_prove_static": (ctypes.c_int, [ctypes.POINTER(Shape), _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "zc_round": (ctypes.c_int, [ctypes.POINTER(Shape), _VP, _VP, _VP, ctypes.c_uint32, _VP, _VP, _VP]),
    "zc_fold": (ctypes.c_int, [ctypes.POINTER(Shape), _VP, _VP, ctypes.c_uint32, _VP]),
    "zc_read_error": (ctypes.c_int, [_VP, _VP]),
    "zc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "zc_test_field": (ctypes.c_int, [ctypes.c_int, _VP, _VP, _VP, ctypes.c_uint64, _VP]),
    "zc_test_sha256": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP, _VP]),
    "zc_bench_mad": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP]),
    "zc_bench_fmul": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP]),
    "zc_bench_sha": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP]),
    "zc_prove_round_kernel": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.c_uint32]),
    "zc_prove_profiled": (ctypes.c_int, [ctypes.POINTER(Shape), _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                         _VP]),
    "zc_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32]),
    "zc_batch_upload": (ctypes.c_int, [ctypes.c_uint32, _VP, _VP, _VP]),
    "zc_batch_launch": (ctypes.c_int, [ctypes.c_uint32, _VP, _VP, _VP]),
    "zc_batch_prove": (ctypes.c_int, [ctypes.c_uint32, _VP, _VP, _VP]),
    "zc_serve_pool_bytes": (ctypes.c_size_t, [ctypes.c_uint32]),
    "zc_serve_rounds": (ctypes.c_int, [ctypes.POINTER(Shape)]),
    "zc_serve_admit": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP]),
    "zc_serve_step": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP, _VP, _VP]),
    "zc_serve_step_part": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, _VP, _VP]),
}


def lib():
    """Load libzc.so (built in-tree by __graft_entry__.build()); fail loudly if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def declared_symbols() -> list[str]:
    """Every function name declared in include/*.h."""
    names = []
    for fn in sorted(os.listdir(INCLUDE)):
        if fn.endswith(".h"):
            text = open(os.path.join(INCLUDE, fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(zc_[a-z_0-9]+)\s*\(", text, re.M)
    return names


def strerror(status: int) -> str:
    return lib().zc_strerror(status).decode()


def _check(rc: int, what: str) -> None:
    if rc != ZC_OK:
        raise ZcError(rc, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def shape(mu: int, gate: int, m: int = 0, flags: int = 0) -> Shape:
    return Shape(mu, gate, m, flags)


def table_count(s: Shape) -> int:
    return lib().zc_table_count(ctypes.byref(s))


def degree(s: Shape) -> int:
    return lib().zc_degree(ctypes.byref(s))


def workspace_bytes(s: Shape) -> int:
    return lib().zc_workspace_bytes(ctypes.byref(s))


def new_workspace(s: Shape, device="cuda") -> torch.Tensor:
    nb = workspace_bytes(s)
    if nb == 0:
        raise ZcError(ZC_EINVAL, "workspace size")
    return torch.zeros(nb, dtype=torch.uint8, device=device)  # error word starts clear


def pack(canon: torch.Tensor, ws: torch.Tensor, stream=None) -> torch.Tensor:
    """uint32[n][8] canonical (device) -> uint32[8][n] packed table."""
    n = canon.shape[0]
    out = torch.empty((8, n), dtype=torch.uint32, device=canon.device)
    _check(lib().zc_pack(_ptr(canon), _ptr(out), n, _ptr(ws), _stream(stream)), "zc_pack")
    return out


def unpack(planar: torch.Tensor, n: int | None = None, stream=None) -> torch.Tensor:
    """Packed table uint32[8][pitch] -> first n elements as uint32[n][8] canonical."""
    pitch = planar.shape[1]
    n = pitch if n is None else n
    out = torch.empty((n, 8), dtype=torch.uint32, device=planar.device)
    _check(lib().zc_unpack(_ptr(planar), pitch, _ptr(out), n, _stream(stream)), "zc_unpack")
    return out


def _table_array(tables):
    arr = (ctypes.c_void_p * len(tables))(*[t.data_ptr() for t in tables])
    return arr


def new_outputs(s: Shape, device="cuda"):
    d, k = degree(s), table_count(s)
    evals = torch.empty((s.mu, d + 2, 8), dtype=torch.uint32, device=device)
    alphas = torch.empty((s.mu, 8), dtype=torch.uint32, device=device)
    openings = torch.empty((k + 1, 8), dtype=torch.uint32, device=device)
    return evals, alphas, openings


def prove(s: Shape, tables, r: torch.Tensor, ws: torch.Tensor, outputs=None, stream=None, pitch: int = 0):
    """Whole proof; returns (round_evals, challenges, openings) device tensors.
    pitch != 0: the tables' limb planes are `pitch` elements apart
    (zc_prove_pitch), e.g. 2^mu-row windows of larger packed tables."""
    evals, alphas, openings = outputs if outputs is not None else new_outputs(s, r.device)
    arr = _table_array(tables)
    if pitch:
        rc = lib().zc_prove_pitch(ctypes.byref(s), arr, pitch, _ptr(r), _ptr(ws), _ptr(evals), _ptr(alphas),
                                  _ptr(openings), _stream(stream))
        _check(rc, "zc_prove_pitch")
    else:
        rc = lib().zc_prove(ctypes.byref(s), arr, _ptr(r), _ptr(ws), _ptr(evals), _ptr(alphas),
                            _ptr(openings), _stream(stream))
        _check(rc, "zc_prove")
    return evals, alphas, openings


def prove_static(s: Shape, tables, r: torch.Tensor, outputs=None, status: torch.Tensor | None = None,
                 stream=None):
    """zc_prove_static: the whole proof in the library's own per-device
    workspace (no workspace argument).  Returns (round_evals, challenges,
    openings); `status` (int32[1] device tensor), if given, receives the
    device-detected status."""
    evals, alphas, openings = outputs if outputs is not None else new_outputs(s, r.device)
    arr = _table_array(tables)
    rc = lib().zc_prove_static(ctypes.byref(s), arr, _ptr(r), _ptr(evals), _ptr(alphas), _ptr(openings),
                               _ptr(status) if status is not None else None, _stream(stream))
    _check(rc, "zc_prove_static")
    return evals, alphas, openings


def round_(s: Shape, tables, r: torch.Tensor, ws: torch.Tensor, i: int, evals, alphas, stream=None):
    arr = _table_array(tables)
    rc = lib().zc_round(ctypes.byref(s), arr, _ptr(r) if r is not None else None, _ptr(ws), i,
                        _ptr(evals), _ptr(alphas), _stream(stream))
    _check(rc, "zc_round")


def fold(s: Shape, tables, ws: torch.Tensor, i: int, stream=None):
    arr = _table_array(tables)
    _check(lib().zc_fold(ctypes.byref(s), arr, _ptr(ws), i, _stream(stream)), "zc_fold")


def read_error(ws: torch.Tensor, stream=None) -> int:
    return lib().zc_read_error(_ptr(ws), _stream(stream))


def prove_profiled(s: Shape, tables, r: torch.Tensor, ws: torch.Tensor, events: "HipEvents",
                   outputs=None, first_event: int = 0, stream=None):
    """zc_prove with events[first_event .. first_event + 2*mu) around the round kernels."""
    evals, alphas, openings = outputs if outputs is not None else new_outputs(s, r.device)
    if first_event + 2 * s.mu > events.n:
        raise ValueError("not enough events")
    arr = _table_array(tables)
    base = ctypes.addressof(events.arr) + first_event * ctypes.sizeof(ctypes.c_void_p)
    rc = lib().zc_prove_profiled(ctypes.byref(s), arr, _ptr(r), _ptr(ws), _ptr(evals), _ptr(alphas),
                                 _ptr(openings), ctypes.c_void_p(base), _stream(stream))
    _check(rc, "zc_prove_profiled")
    return evals, alphas, openings


class Batch:
    """Instances proved together (zc_batch_*).

    items: sequence of (shape, tables, r, ws, outputs, tile), each as for
    prove(); outputs from new_outputs(shape).  Keeps the ctypes arrays the
    library reads alive and owns the batch workspace.
    """

    def __init__(self, items, device="cuda"):
        self.items = list(items)
        self.n = len(self.items)
        self._tabs = [_table_array(it[1]) for it in self.items]
        self.arr = (Instance * self.n)()
        for i, (s, tables, r, ws, outs, tile) in enumerate(self.items):
            ev, al, op = outs
            self.arr[i] = Instance(s, ctypes.cast(self._tabs[i], ctypes.c_void_p), r.data_ptr(), ws.data_ptr(),
                                   ev.data_ptr(), al.data_ptr(), op.data_ptr(), tile)
        nb = lib().zc_batch_workspace_bytes(self.n)
        if nb == 0:
            raise ZcError(ZC_EINVAL, "batch workspace size")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)

    def upload(self, stream=None):
        _check(lib().zc_batch_upload(self.n, self.arr, _ptr(self.ws), _stream(stream)), "zc_batch_upload")

    def launch(self, stream=None):
        _check(lib().zc_batch_launch(self.n, self.arr, _ptr(self.ws), _stream(stream)), "zc_batch_launch")

    def prove(self, stream=None):
        _check(lib().zc_batch_prove(self.n, self.arr, _ptr(self.ws), _stream(stream)), "zc_batch_prove")


def serve_rounds(s: Shape) -> int:
    n = lib().zc_serve_rounds(ctypes.byref(s))
    _check(min(n, 0), "zc_serve_rounds")
    return n


class ServePool:
    """zc_serve_*: a device pool of instance slots advanced one round per step."""

    def __init__(self, slots: int, device="cuda"):
        nb = lib().zc_serve_pool_bytes(slots)
        if nb == 0:
            raise ZcError(ZC_EINVAL, "serve pool size")
        self.slots = slots
        self.mem = torch.empty(nb, dtype=torch.uint8, device=device)

    def admit(self, slot: int, inst: Instance, stream=None):
        _check(lib().zc_serve_admit(_ptr(self.mem), self.slots, slot, ctypes.byref(inst), _stream(stream)),
               "zc_serve_admit")

    def step(self, slot_ids, rounds, insts, stream=None):
        n = len(slot_ids)
        sl = (ctypes.c_uint32 * n)(*slot_ids)
        rd = (ctypes.c_uint32 * n)(*rounds)
        arr = (Instance * n)(*insts)
        _check(lib().zc_serve_step(_ptr(self.mem), self.slots, n, sl, rd, arr, _stream(stream)), "zc_serve_step")

    def step_part(self, slot: int, rnd: int, part: int, parts: int, inst: "Instance", stream=None):
        """zc_serve_step_part: part `part` of `parts` of round `rnd` of one instance."""
        _check(lib().zc_serve_step_part(_ptr(self.mem), self.slots, slot, rnd, part, parts, ctypes.byref(inst),
                                        _stream(stream)), "zc_serve_step_part")


class HipEvents:
    """A host array of hipEvent_t created through the HIP runtime (for zc_prove_profiled)."""

    def __init__(self, n: int):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), _VP, _VP]
        self.hip.hipEventSynchronize.argtypes = [_VP]
        self.hip.hipEventDestroy.argtypes = [_VP]
        self.n = n
        self.arr = (ctypes.c_void_p * n)()
        base = ctypes.addressof(self.arr)
        for i in range(n):
            rc = self.hip.hipEventCreate(ctypes.c_void_p(base + i * ctypes.sizeof(ctypes.c_void_p)))
            if rc != 0:
                raise ZcError(ZC_EHIP, "hipEventCreate")

    def record(self, i: int, stream=None):
        """hipEventRecord of event i on the stream (torch's current one by default)."""
        self.hip.hipEventRecord.argtypes = [_VP, _VP]
        rc = self.hip.hipEventRecord(ctypes.c_void_p(self.arr[i]), _stream(stream))
        if rc != 0:
            raise ZcError(ZC_EHIP, "hipEventRecord")

    def elapsed_ms(self, a: int, b: int) -> float:
        self.hip.hipEventSynchronize(self.arr[b])
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), self.arr[a], self.arr[b])
        if rc != 0:
            raise ZcError(ZC_EHIP, "hipEventElapsedTime")
        return ms.value

    def __del__(self):
        try:
            for i in range(self.n):
                self.hip.hipEventDestroy(self.arr[i])
        except Exception:
            pass


def test_field(op: int, a: torch.Tensor, b: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty_like(a)
    _check(lib().zc_test_field(op, _ptr(a), _ptr(b), _ptr(out), a.shape[0], _stream(stream)),
           "zc_test_field")
    return out


def test_sha256(msg_words: torch.Tensor, length: int, stream=None) -> torch.Tensor:
    out = torch.empty(8, dtype=torch.uint32, device=msg_words.device)
    _check(lib().zc_test_sha256(_ptr(msg_words), length, _ptr(out), _stream(stream)),
           "zc_test_sha256")
    return out


def bench_mad(blocks: int, chains: int, iters: int, sink: torch.Tensor, stream=None):
    _check(lib().zc_bench_mad(blocks, chains, iters, _ptr(sink), _stream(stream)), "zc_bench_mad")


def bench_fmul(blocks: int, chains: int, iters: int, inp: torch.Tensor, out: torch.Tensor, stream=None):
    _check(lib().zc_bench_fmul(blocks, chains, iters, _ptr(inp), _ptr(out), _stream(stream)), "zc_bench_fmul")


def bench_sha(variant: int, n: int, inp: torch.Tensor, out: torch.Tensor, stream=None):
    _check(lib().zc_bench_sha(variant, n, _ptr(inp), _ptr(out), _stream(stream)), "zc_bench_sha")
