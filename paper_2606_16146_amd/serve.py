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

Fast path (`fast_queue` > 0, the default): while no step is running and at
most `fast_queue` requests wait, waiting requests are proved whole with
zc_prove (zc_prove_pitch for a window) instead of being stepped, up to
`lanes` proofs at once, each on a stream of its own (all at the default
priority).  A step runs every (gate, fold) group's round and finisher
launches for one round of each admitted request, which at low concurrency
costs a request several times its proof alone; zc_prove runs the
single-proof schedule (lane-split and fused rounds, the LDS tail in one
launch).  Proofs on distinct streams share the GPU: a small proof's chain of
short kernels runs in the gaps of a large proof's wide rounds rather than
after it.  The fast path takes the waiting request with the fewest hypercube
points (`order="sjf"`, shortest job first) unless the oldest has waited
`max_wait_s`, or the oldest (`order="fcfs"`).  Requests of 2^big_mu points
or more hold at most `big_lanes` lanes at once and (`share_big`) run with
ZC_FLAG_SHARED_GPU grids, whose shorter-lived blocks free compute units for
the small proofs' kernels during a large round.  While no other large
request waits (`split_big`), a large request is instead stepped through the
pool round by round, each large round in parts of about `part_blocks`
blocks (zc_serve_step_part), and its next part waits while small proofs
run (at most `hold_big_s`): small requests then run with the GPU nearly to
themselves, as under shortest-remaining-work-first.  A queue longer than
`fast_queue`, and arrivals while steps run, go to continuous batching.
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
    fast_path: bool = False     # proved whole by the fast path rather than stepped
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


_LANES: dict = {}


def _lane_streams(dev: torch.device, n: int) -> list:
    """Streams of `dev` at the default priority, created once per process and
    reused by every server: [0] carries only the loop's error-word reads,
    [1..n-1] are fast-path lanes beside the serving stream."""
    have = _LANES.setdefault(dev.index if dev.index is not None else torch.cuda.current_device(), [])
    while len(have) < max(n, 1):
        have.append(torch.cuda.Stream(dev))
    return have[:max(n, 1)]


class Server:
    def __init__(self, slots: int = 256, mem_budget: int | None = None, ahead: int = 2, device="cuda",
                 stream: torch.cuda.Stream | None = None, fast_queue: int = 16, order: str = "sjf",
                 max_wait_s: float = 0.05, lanes: int = 4, big_mu: int | None = 21, big_lanes: int = 1,
                 share_big: bool = True, split_big: bool = True, part_blocks: int = 256,
                 hold_big_s: float = 0.001):
        self.dev = torch.device(device)
        self.pool = zc.ServePool(slots, self.dev)
        self.slots = slots
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            mem_budget = int(free * 0.5)
        self.mem_budget = mem_budget
        self.ahead = ahead
        self.stream = stream or torch.cuda.current_stream(self.dev)
        if order not in ("sjf", "fcfs"):
            raise ValueError(f"order must be 'sjf' or 'fcfs', not {order!r}")
        if lanes < 1:
            raise ValueError("lanes must be >= 1")
        self.fast_queue = fast_queue
        self.lanes = [self.stream] + _lane_streams(self.dev, lanes)[1:]
        self.big_mu = big_mu          # requests with mu >= big_mu ...
        self.big_lanes = big_lanes    # ... hold at most this many lanes at once
        self.share_big = share_big and lanes > 1  # ... with ZC_FLAG_SHARED_GPU grids
        self.book = _lane_streams(self.dev, 1)[0]  # runs only the error-word reads
        # split_big: while no other large request waits, a large one is
        # stepped through the pool in parts of about part_blocks blocks
        # (zc_serve_step_part) on a stream of its own, its next part held back
        # while small proofs run (at most hold_big_s after its previous part
        # ended); otherwise it is proved whole like the others
        self.split_big = split_big and big_mu is not None
        self.part_blocks = part_blocks
        self.hold_big_s = hold_big_s
        self.big_stream = _lane_streams(self.dev, lanes + 1)[lanes]
        self.order = order
        self.max_wait_s = max_wait_s

    def _device_state(self, req: Request, stream: torch.cuda.Stream):
        """Workspace and outputs of a request that runs on `stream`.  They come
        from the serving stream's pool of the caching allocator whatever the
        lane (one pool rather than one per lane, so blocks freed by one lane
        serve the next request of any lane), marked as used on `stream`.  The
        workspace is not cleared: zc_prove and serve admission reset its
        control block."""
        s = req.shape
        with torch.cuda.stream(self.stream):
            req.ws = torch.empty(zc.workspace_bytes(s), dtype=torch.uint8, device=self.dev)
            req.outputs = zc.new_outputs(s, self.dev)
        if stream is not self.stream:
            for t in (req.ws, *req.outputs):
                t.record_stream(stream)
        if req.host_tables:
            with torch.cuda.stream(stream):
                req._dev_tables = [t.to(self.dev, non_blocking=True) for t in req.tables]
        else:
            req._dev_tables = req.tables

    def _big(self, req: Request) -> bool:
        return self.big_mu is not None and req.shape.mu >= self.big_mu

    def _pick(self, waiting, now: float, allow_big: bool) -> int:
        """Index in `waiting` of the request the fast path proves next, or -1."""
        ok = [j for j in range(len(waiting)) if allow_big or not self._big(waiting[j])]
        if not ok:
            return -1
        if self.order == "fcfs" or now - waiting[ok[0]].arrival >= self.max_wait_s:
            return ok[0]
        return min(ok, key=lambda j: (waiting[j].points, waiting[j].arrival))

    def _parts(self, mu: int, rnd: int, last: int, tile: int = 0) -> int:
        """Parts of round rnd of a split request: a power of two, so that they
        divide the round's blocks (zc_serve_step_part: 2^(mu - rnd) pairs in
        blocks of 256 x tile pairs, tile 0 meaning 4, at most 2048 blocks)."""
        if rnd == last:
            return 1
        per = 256 * (tile or 4)
        blocks = max(1, min(2048, ((1 << (mu - rnd)) + per - 1) // per))
        parts = 1
        while parts * 2 <= min(8, blocks // self.part_blocks):
            parts *= 2
        return parts

    def _prove_alone(self, req: Request, now: float, stream: torch.cuda.Stream):
        """The fast path: the whole proof, single-proof schedule, on `stream`
        (its workspace and outputs allocated in that stream's order)."""
        self._device_state(req, stream)
        s = req.shape
        if self.share_big and self._big(req):
            s = zc.shape(s.mu, s.gate, s.m, s.flags | zc.ZC_FLAG_SHARED_GPU)
        zc.prove(s, req._dev_tables, req.r, req.ws, outputs=req.outputs, stream=stream, pitch=req.pitch)
        req.t_admit = now
        req.fast_path = True

    def _admit(self, req: Request, slot: int, now: float, stream: torch.cuda.Stream | None = None):
        stream = stream or self.stream
        s = req.shape
        self._device_state(req, stream)
        ev, al, op = req.outputs
        req._tabarr = (ctypes.c_void_p * len(req._dev_tables))(*[t.data_ptr() for t in req._dev_tables])
        req._inst = zc.Instance(s, ctypes.cast(req._tabarr, ctypes.c_void_p), req.r.data_ptr(),
                                req.ws.data_ptr(), ev.data_ptr(), al.data_ptr(), op.data_ptr(), req.tile,
                                req.pitch)
        self.pool.admit(slot, req._inst, stream)
        req.t_admit = now

    def run(self, requests: list[Request]) -> dict:
        """Serves the requests (arrival times relative to the call); returns stats."""
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        waiting: collections.deque = collections.deque()
        active: list = []           # [req, slot, round, last]
        in_flight: list = []        # [event, [reqs it completes], lane or -1 for a step], oldest first
        lane_busy = [0] * len(self.lanes)
        big_running = 0
        bigs: list = []             # split large requests: [req, slot, round, last, part, parts, in flight, since]
        free_slots = list(range(self.slots - 1, -1, -1))
        mem_used = 0
        steps = 0
        fast_n = 0
        split_n = 0

        def retire(entry):
            nonlocal mem_used, big_running
            ev, done, lane = entry[:3]
            ev.synchronize()
            t = time.perf_counter() - t0
            if lane >= 0:
                lane_busy[lane] -= 1
                big_running -= sum(self._big(q) for q in done)
            elif lane == -2:  # a part of a split request
                b = entry[3]
                b[6] -= 1
                b[7] = t
                if done:
                    bigs.remove(b)
                    free_slots.append(b[1])  # its last part has completed
                    big_running -= 1
            for req in done:
                req.t_done = t
                mem_used -= req._bytes
                # the error word, read now on a stream that runs nothing else (so the
                # read is not queued behind a proof); the workspace is released after it
                with torch.cuda.stream(self.book):
                    self.book.wait_event(ev)
                    req.err = int(req.ws[:4].view(torch.int32).cpu()[0])
                req.ws = None
                req._dev_tables = []

        with torch.cuda.stream(self.stream):
            t0 = time.perf_counter()
            while pending or waiting or active or in_flight or bigs:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                launched = False
                fast = not active and 0 < len(waiting) <= self.fast_queue
                depth = 2 if len(self.lanes) == 1 else 1
                while fast and waiting:
                    lane = min(range(len(self.lanes)), key=lambda j: lane_busy[j])
                    allow_big = big_running < self.big_lanes
                    if lane_busy[lane] >= depth and not (self.split_big and allow_big and free_slots):
                        break
                    pick = self._pick(waiting, now, allow_big)
                    if pick < 0 or (mem_used + footprint(waiting[pick]) > self.mem_budget and in_flight):
                        break
                    req = waiting[pick]
                    # split a large request only while no other large one waits
                    # (light load); under load the whole-proof path keeps the
                    # throughput
                    light = not any(self._big(q) for q in waiting if q is not req)
                    if self.split_big and self._big(req) and free_slots and light:
                        del waiting[pick]
                        slot = free_slots.pop()
                        self._admit(req, slot, now, self.big_stream)
                        req._bytes = footprint(req)
                        mem_used += req._bytes
                        big_running += 1
                        bigs.append([req, slot, 1, zc.serve_rounds(req.shape), 0, 0, 0, now])
                        split_n += 1
                        launched = True
                        continue
                    if lane_busy[lane] >= depth:
                        break
                    del waiting[pick]
                    self._prove_alone(req, now, self.lanes[lane])
                    req._bytes = footprint(req)
                    mem_used += req._bytes
                    ev = torch.cuda.Event()
                    ev.record(self.lanes[lane])
                    lane_busy[lane] += 1
                    big_running += self._big(req)
                    in_flight.append([ev, [req], lane])
                    fast_n += 1
                    launched = True
                while waiting and free_slots and not fast:
                    need = footprint(waiting[0])
                    if mem_used + need > self.mem_budget and (active or in_flight):
                        break  # admit when memory frees up (an idle server admits anything)
                    req = waiting.popleft()
                    slot = free_slots.pop()
                    self._admit(req, slot, now)
                    req._bytes = need
                    mem_used += need
                    active.append([req, slot, 1, zc.serve_rounds(req.shape)])
                # split requests: the next part when small proofs leave the GPU
                small_running = sum(1 for e in in_flight if e[2] >= 0 and not any(self._big(q) for q in e[1]))
                for b in list(bigs):
                    if b[2] > b[3]:  # every part issued; retires when its last part completes
                        continue
                    if b[6] >= (1 if small_running else 2) or (small_running and now - b[7] < self.hold_big_s):
                        continue
                    req, slot, rnd, last = b[0], b[1], b[2], b[3]
                    if b[4] == 0:
                        b[5] = self._parts(req.shape.mu, rnd, last, req.tile)
                    self.pool.step_part(slot, rnd, b[4], b[5], req._inst, self.big_stream)
                    ev = torch.cuda.Event()
                    ev.record(self.big_stream)
                    b[4] += 1
                    finished = False
                    if b[4] == b[5]:
                        b[2] += 1
                        b[4] = 0
                        finished = b[2] > last
                    b[6] += 1
                    in_flight.append([ev, [req] if finished else [], -2, b])
                    launched = True
                if active:
                    self.pool.step([a[1] for a in active], [a[2] for a in active], [a[0]._inst for a in active])
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    steps += 1
                    launched = True
                    done = [a for a in active if a[2] == a[3]]
                    for a in active:
                        a[2] += 1
                    active = [a for a in active if a[2] <= a[3]]
                    for a in done:  # later launches are ordered after this step on the stream
                        free_slots.append(a[1])
                    in_flight.append([ev, [a[0] for a in done], -1])
                # retire completed work; block on the oldest step when too many are in flight
                for entry in [e for e in in_flight if e[0].query()]:
                    in_flight.remove(entry)
                    retire(entry)
                while sum(1 for e in in_flight if e[2] == -1) > self.ahead:
                    entry = next(e for e in in_flight if e[2] == -1)
                    in_flight.remove(entry)
                    retire(entry)
                if not launched and not in_flight and not waiting and pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.001)))
            wall = time.perf_counter() - t0
        torch.cuda.synchronize(self.dev)
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
                "fast_path_requests": fast_n, "split_requests": split_n,
                "errors": sum(1 for q in requests if q.err != 0), "by_mu": by_mu}
