"""Launch-shape autotuner for batched proofs.

The free launch parameter of a batch is each instance's tile, the pairs per
thread of its round kernels: a small tile gives more blocks (parallelism for
a sparse step), a large one fewer blocks and fewer partial sums to add.  The
best choice could depend on the gate (work per pair), on mu (how many pairs a
round has) and on how full the GPU is with the rest of the batch, so it is
measured, not modelled: instances are grouped into buckets (gate, mu <= 13 or
mu >= 14), and each bucket's tile is chosen in turn (coordinate descent,
other buckets fixed) by timing the whole batch.

Every candidate is timed `reps` times with HIP events around one replay of
the batch launch sequence.  A candidate replaces the current choice only if
its median beats the current choice's median by more than the current
choice's spread (max - min over its reps): differences inside the run-to-run
noise are not taken as improvements, so a bucket keeps the default unless a
tile is measurably better.

The tile changes launch shapes only; the proof bytes are the same for any
tile (tested).
"""
from __future__ import annotations

import statistics

import torch

from . import zc

CANDIDATES = (1, 2, 4, 8, 16)
DEFAULT_TILE = 4


def bucket_of(shape: "zc.Shape") -> tuple[int, int, int]:
    return (shape.gate, shape.m, 0 if shape.mu <= 13 else 1)


def _time_batch(b: "zc.Batch", reps: int) -> list[float]:
    """Seconds of each of `reps` launches of the uploaded batch."""
    b.upload()
    b.launch()  # warm
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.launch()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return ts


def tune(b: "zc.Batch", candidates=CANDIDATES, reps: int = 10, rounds: int = 1, log=None) -> dict:
    """Chooses a tile per bucket for batch b (sets b.arr[i].tile) and returns
    {bucket: {"tile", "median_ms", "spread_ms", "default_median_ms", "tried"}}.
    Leaves b uploaded with the chosen tiles."""
    buckets: dict = {}
    for i in range(b.n):
        buckets.setdefault(bucket_of(b.arr[i].shape), []).append(i)
    choice = {k: DEFAULT_TILE for k in buckets}

    def apply():
        for k, idx in buckets.items():
            for i in idx:
                b.arr[i].tile = choice[k]

    apply()
    cur = _time_batch(b, reps)
    default_median = statistics.median(cur)
    report = {}
    for _ in range(rounds):
        for k in sorted(buckets):
            keep = choice[k]
            tried = {keep: round(statistics.median(cur) * 1e3, 3)}
            for t in candidates:
                if t == keep:
                    continue
                choice[k] = t
                apply()
                ts = _time_batch(b, reps)
                tried[t] = round(statistics.median(ts) * 1e3, 3)
                if statistics.median(ts) < statistics.median(cur) - (max(cur) - min(cur)):
                    cur, keep = ts, t
            choice[k] = keep
            apply()
            report[k] = {"tile": keep, "median_ms": round(statistics.median(cur) * 1e3, 3),
                         "spread_ms": round((max(cur) - min(cur)) * 1e3, 3),
                         "default_median_ms": round(default_median * 1e3, 3), "tried": tried}
            if log:
                log(f"[autotune] bucket gate={k[0]} m={k[1]} {'mu>=14' if k[2] else 'mu<=13'} "
                    f"({len(buckets[k])} instances): tile {keep}, median {report[k]['median_ms']} ms "
                    f"(spread {report[k]['spread_ms']} ms); medians by tile {tried}")
    b.upload()
    return report
