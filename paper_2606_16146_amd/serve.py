"""Serving loop: proofs admitted by HBM footprint as they arrive, advanced
together one round per step (continuous batching).

Each request brings a shape, its packed tables (device resident, read only,
possibly a 2^mu-element window of a larger packed table: `pitch`), its r and
a tile.  The loop
* admits waiting requests in arrival order while a slot is free and their
  device footprint (workspace + outputs, plus a table copy when the request
  arrives with host tables) fits the memory budget;
* runs one step: every admitted request that is not finished runs its next
  round, all of them in the same launches (zc_serve_step), so a request that
  arrives while others are on the GPU joins at the next step and its work
  overlaps theirs;
* retires requests whose last step has completed on the device (HIP events),
  frees their workspace and slot, and records their completion time.
At most `ahead` steps are in flight, so admission keeps up with arrivals.
Outputs stay on the device.  Every request's bytes equal its zc_prove proof
(each instance owns its workspace; sharing a launch changes nothing it
computes).
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

import torch

from . import zc


@dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the run
    shape: "zc.Shape"
    tables: list                # packed device tables (uint32[8][2^mu]), or pinned host copies
    r: torch.Tensor             # device, mu x 8
    tile: int = 0
    host_tables: bool = False   # tables live in pinned host memory: copy at admission
    pitch: int = 0              # plane pitch of the tables (0: 2^mu, as zc_pack makes them)
    shared_tables: bool = False  # the tables are views into a pool resident for the whole run
    # filled by the loop
    t_admit: float = float("nan")
    t_done: float = float("nan")
    outputs: tuple = ()
    ws: torch.Tensor | None = None
    err: int = 0
    _dev_tables: list = field(default_factory=list)

    @property
    def points(self) -> int:
        return 1 << self.shape.mu

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def footprint(req: Request) -> int:
    """Device bytes a request holds while admitted: its workspace, its outputs
    and its k packed tables (copied to the device at admission for host
    tables, already resident otherwise).  Tables that are views into a pool
    resident for the whole run (shared_tables) are the pool's bytes, which the
    caller keeps out of the budget, so they count 0 here."""
    s = req.shape
    out = (s.mu * (zc.degree(s) + 2) + zc.table_count(s) + 1 + s.mu) * 32
    tabs = 0 if req.shared_tables else zc.table_count(s) * (1 << s.mu) * 32
    return zc.workspace_bytes(s) + out + tabs


class Server:
    def __init__(self, slots: int = 256, mem_budget: int | None = None, ahead: int = 2, device="cuda",
                 stream: torch.cuda.Stream | None = None):
        self.dev = torch.device(device)
        self.pool = zc.ServePool(slots, self.dev)
        self.slots = slots
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            mem_budget = int(free * 0.5)
        self.mem_budget = mem_budget
        self.ahead = ahead
        self.stream = stream or torch.cuda.current_stream(self.dev)

    def _admit(self, req: Request, slot: int, now: float):
        s = req.shape
        req.ws = zc.new_workspace(s, self.dev)
        req.outputs = zc.new_outputs(s, self.dev)
        if req.host_tables:
            req._dev_tables = [t.to(self.dev, non_blocking=True) for t in req.tables]
        else:
            req._dev_tables = req.tables
        ev, al, op = req.outputs
        req._tabarr = (ctypes.c_void_p * len(req._dev_tables))(*[t.data_ptr() for t in req._dev_tables])
        req._inst = zc.Instance(s, ctypes.cast(req._tabarr, ctypes.c_void_p), req.r.data_ptr(),
                                req.ws.data_ptr(), ev.data_ptr(), al.data_ptr(), op.data_ptr(), req.tile,
                                req.pitch)
        self.pool.admit(slot, req._inst)
        req.t_admit = now

    def run(self, requests: list[Request]) -> dict:
        """Serves the requests (arrival times relative to the call); returns stats."""
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        waiting: collections.deque = collections.deque()
        active: list = []           # [req, slot, round, last]
        in_flight: collections.deque = collections.deque()  # (event, [finished reqs])
        free_slots = list(range(self.slots - 1, -1, -1))
        mem_used = 0
        steps = 0
        with torch.cuda.stream(self.stream):
            t0 = time.perf_counter()
            while pending or waiting or active or in_flight:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                while waiting and free_slots:
                    need = footprint(waiting[0])
                    if mem_used + need > self.mem_budget and (active or in_flight):
                        break  # admit when memory frees up (an idle server admits anything)
                    req = waiting.popleft()
                    slot = free_slots.pop()
                    self._admit(req, slot, now)
                    req._bytes = need
                    mem_used += need
                    active.append([req, slot, 1, zc.serve_rounds(req.shape)])
                if active:
                    self.pool.step([a[1] for a in active], [a[2] for a in active], [a[0]._inst for a in active])
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    steps += 1
                    done = [a for a in active if a[2] == a[3]]
                    for a in active:
                        a[2] += 1
                    active = [a for a in active if a[2] <= a[3]]
                    for a in done:  # later launches are ordered after this step on the stream
                        free_slots.append(a[1])
                    in_flight.append((ev, [a[0] for a in done]))
                # retire completed steps; block when too far ahead or when idle otherwise
                while in_flight and (in_flight[0][0].query() or len(in_flight) > self.ahead or
                                     (not active and not waiting)):
                    ev, done = in_flight.popleft()
                    ev.synchronize()
                    t = time.perf_counter() - t0
                    for req in done:
                        req.t_done = t
                        mem_used -= req._bytes
                        # keep the error word (a stream-ordered copy), release the workspace
                        req._err_word = req.ws[:4].clone()
                        req.ws = None
                        req._dev_tables = []
                if not active and not in_flight and not waiting and pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.001)))
            wall = time.perf_counter() - t0
        torch.cuda.synchronize(self.dev)
        for req in requests:
            req.err = int(req._err_word.view(torch.int32)[0].item())
        lat = sorted(q.latency for q in requests)
        pts = sum(q.points for q in requests)

        def pct(vals, p):
            return vals[min(len(vals) - 1, int(round(p / 100.0 * (len(vals) - 1))))]

        by_mu = {}
        for mu in sorted({q.shape.mu for q in requests}):
            lm = sorted(q.latency for q in requests if q.shape.mu == mu)
            by_mu[str(mu)] = {"n": len(lm), "p50_ms": pct(lm, 50) * 1e3, "p99_ms": pct(lm, 99) * 1e3}
        return {"requests": len(requests), "points": pts, "wall_s": wall, "points_per_s": pts / wall,
                "p50_ms": pct(lat, 50) * 1e3, "p99_ms": pct(lat, 99) * 1e3, "steps": steps,
                "errors": sum(1 for q in requests if q.err != 0), "by_mu": by_mu}
