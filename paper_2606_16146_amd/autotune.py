"""Launch-shape autotuner for batched proofs.

The one free launch parameter of a batch is each instance's tile, the pairs
per thread of its round kernels: a small tile gives more blocks (parallelism
for a sparse step), a large one fewer blocks and fewer partial sums to add.
The best choice depends on the gate (work per pair) and on mu (how many
pairs a round has), and on how full the GPU is with the rest of the batch,
so it is measured, not modelled: instances are grouped into buckets
(gate, mu <= 13 or mu >= 14), and each bucket's tile is chosen in turn
(coordinate descent, other buckets fixed) by timing the whole batch.

The tile changes launch shapes only; the proof bytes are the same for any
tile (tested).
"""
from __future__ import annotations

import time

import torch

from . import zc

CANDIDATES = (1, 2, 4, 8, 16)
DEFAULT_TILE = 4


def bucket_of(shape: "zc.Shape") -> tuple[int, int, int]:
    return (shape.gate, shape.m, 0 if shape.mu <= 13 else 1)


def _time_batch(b: "zc.Batch", reps: int) -> float:
    b.upload()
    b.launch()  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(b: "zc.Batch", candidates=CANDIDATES, reps: int = 3, rounds: int = 1, log=None) -> dict:
    """Chooses a tile per bucket for batch b (sets b.arr[i].tile) and returns
    {bucket: tile}.  Leaves b uploaded with the chosen tiles."""
    buckets: dict = {}
    for i in range(b.n):
        buckets.setdefault(bucket_of(b.arr[i].shape), []).append(i)
    choice = {k: DEFAULT_TILE for k in buckets}

    def apply():
        for k, idx in buckets.items():
            for i in idx:
                b.arr[i].tile = choice[k]

    apply()
    best_t = _time_batch(b, reps)
    for _ in range(rounds):
        for k in sorted(buckets):
            keep = choice[k]
            for t in candidates:
                if t == keep:
                    continue
                choice[k] = t
                apply()
                dt = _time_batch(b, reps)
                if dt < best_t:
                    best_t, keep = dt, t
            choice[k] = keep
            apply()
            if log:
                log(f"[autotune] bucket gate={k[0]} m={k[1]} {'mu>=14' if k[2] else 'mu<=13'} "
                    f"({len(buckets[k])} instances): tile {keep}, batch {best_t * 1e3:.2f} ms")
    b.upload()
    return choice
