"""Seeded synthetic ZeroCheck workloads.

This module only draws random field elements and lays them out; it holds no
step of the SumCheck prover (no eq table, no round polynomial, no fold, no
transcript).  It is the one piece of code that both the CPU oracle's tests
and the GPU path consume, so that both sides see the very same inputs.

Recipe (one independent stream per (seed, instance, table)):

* ``numpy.random.Generator(PCG64(SeedSequence([seed, inst, table_id])))``
  draws ``u32[N][8]`` little-endian limbs; the top two bits of limb 7 are
  cleared (value < 2^254 < 2p) and p is subtracted once when the value is
  >= p, which gives a canonical element of F_p.
* The eq point ``r`` uses ``table_id = 0xFFFF`` and the same recipe.
* The witness is made to satisfy the gate on every hypercube point by
  setting its last column: ``qC = -(qM*a*b + qL*a + qR*b + qO*c)`` for the
  vanilla gate, ``o = s*w1*...*wm`` for the product gate, and for the
  Table 1 shapes ``g1*...*gP + gP+1 + ... + gP+A`` the last additive term
  (minus the rest); a pure product (A = 0) is made to vanish by zeroing, on
  every row, one factor picked by a stream of its own (``table_id =
  0xFFFC``).  That column is computed here with Python integers modulo p; a wrong column
  would only make the witness non-satisfying, which the protocol-level
  tests (first claim equal to 0) detect independently of either prover.

Table order is the gate's column order: vanilla ``[a, b, c, qM, qL, qR, qO,
qC]``; product ``[s, w1, ..., wm, o]``.  These are the paper's workload
shapes (Table 1 lists degree / unique polynomials / additive terms; the
vanilla gate is the HyperPlonk-style gate, the product gate sweeps degree).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# BN254 scalar field modulus (decimal form).
P = 21888242871839275222246405745257275088548364400416034343698204186575808495617

GATE_VANILLA = 0
GATE_PROD = 1
GATE_SUMPROD = 2  # Table 1 shapes g1*...*gP + gP+1 + ... + gP+A, m = P + 16 A

# (P, A) of the six polynomials of Table 1
TABLE1_SHAPES = ((2, 0), (2, 1), (2, 2), (2, 3), (3, 0), (4, 0))

R_TABLE_ID = 0xFFFF
ZERO_TABLE_ID = 0xFFFC  # which factor of a pure product is zeroed, per row


def sumprod_m(pp: int, aa: int) -> int:
    return pp + 16 * aa


def sumprod_pa(m: int) -> tuple[int, int]:
    pa = (m & 15, m >> 4)
    if pa not in TABLE1_SHAPES:
        raise ValueError(f"not a Table 1 shape: m={m}")
    return pa


def gate_tables(gate: int, m: int) -> int:
    """Number of witness tables (eq not included) of a gate."""
    if gate == GATE_VANILLA:
        return 8
    if gate == GATE_PROD:
        if not 1 <= m <= 8:
            raise ValueError("product gate needs 1 <= m <= 8")
        return m + 2
    if gate == GATE_SUMPROD:
        pp, aa = sumprod_pa(m)
        return pp + aa
    raise ValueError(f"unknown gate {gate}")


def gate_degree(gate: int, m: int) -> int:
    """Total degree d of the gate polynomial in its multilinear inputs."""
    if gate == GATE_VANILLA:
        return 3
    if gate == GATE_PROD:
        return m + 1
    if gate == GATE_SUMPROD:
        return sumprod_pa(m)[0]
    raise ValueError(f"unknown gate {gate}")


def _stream(seed: int, inst: int, table_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, inst, table_id])))


_P_LIMBS = np.array([(P >> (32 * k)) & 0xFFFFFFFF for k in range(8)], dtype=np.int64)


def limbs_to_ints(a: np.ndarray) -> list:
    """u32[n][8] little-endian limbs -> list of Python ints."""
    b = np.ascontiguousarray(a, dtype=np.uint32).tobytes()
    return [int.from_bytes(b[i:i + 32], "little") for i in range(0, len(b), 32)]


def ints_to_limbs(vals) -> np.ndarray:
    """Python ints in [0, 2^256) -> u32[n][8] little-endian limbs."""
    b = b"".join(int(v).to_bytes(32, "little") for v in vals)
    return np.frombuffer(b, dtype=np.uint32).reshape(-1, 8).copy()


def _geq_p(raw: np.ndarray) -> np.ndarray:
    """Row-wise raw >= p for u32[n][8] limbs (lexicographic from the top limb)."""
    gt = np.zeros(raw.shape[0], dtype=bool)
    eq = np.ones(raw.shape[0], dtype=bool)
    for k in range(7, -1, -1):
        col = raw[:, k].astype(np.int64)
        gt |= eq & (col > _P_LIMBS[k])
        eq &= col == _P_LIMBS[k]
    return gt | eq


def _sub_p_rows(raw: np.ndarray, mask: np.ndarray) -> None:
    """raw[mask] -= p in place (rows known to be >= p)."""
    sel = raw[mask].astype(np.int64)
    borrow = np.zeros(sel.shape[0], dtype=np.int64)
    for k in range(8):
        dif = sel[:, k] - _P_LIMBS[k] - borrow
        borrow = (dif < 0).astype(np.int64)
        sel[:, k] = dif + (borrow << 32)
    raw[mask] = sel.astype(np.uint32)


def draw_elements(seed: int, inst: int, table_id: int, n: int) -> np.ndarray:
    """n canonical field elements as u32[n][8] (recipe in the module docstring)."""
    raw = _stream(seed, inst, table_id).integers(0, 1 << 32, size=(n, 8), dtype=np.uint32)
    raw[:, 7] &= np.uint32(0x3FFFFFFF)
    ge = _geq_p(raw)
    if ge.any():
        _sub_p_rows(raw, ge)
    return raw


@dataclass
class Instance:
    """One ZeroCheck instance: canonical tables u32[k][N][8] and r u32[mu][8]."""

    seed: int
    inst: int
    mu: int
    gate: int
    m: int
    tables: np.ndarray  # uint32[k][2^mu][8], canonical, little-endian limbs
    r: np.ndarray  # uint32[mu][8], canonical

    @property
    def k(self) -> int:
        return self.tables.shape[0]

    @property
    def degree(self) -> int:
        return gate_degree(self.gate, self.m)

    def tables_int(self) -> list[list[int]]:
        return [limbs_to_ints(t) for t in self.tables]

    def r_int(self) -> list[int]:
        return limbs_to_ints(self.r)


def _satisfying_column(gate: int, cols_limbs: np.ndarray, m: int = 0) -> np.ndarray:
    """The last column that makes the gate vanish on every row (Python ints)."""
    cols = [limbs_to_ints(c) for c in cols_limbs]
    if gate == GATE_VANILLA:
        last = [(-(qm * a % P * b + ql * a + qr * b + qo * c)) % P
                for a, b, c, qm, ql, qr, qo in zip(*cols)]
    elif gate == GATE_SUMPROD:
        pp, _ = sumprod_pa(m)
        last = []
        for row in zip(*cols):
            prod = 1
            for g in row[:pp]:
                prod = prod * g % P
            last.append((-(prod + sum(row[pp:]))) % P)
    else:
        last = cols[0]
        for w in cols[1:]:
            last = [x * y % P for x, y in zip(last, w)]
    return ints_to_limbs(last)


def _satisfying_chunk(args):
    gate, cols, m = args
    return _satisfying_column(gate, cols, m)


def make_instance(seed: int, inst: int, mu: int, gate: int, m: int = 0,
                  satisfying: bool = True, workers: int = 1) -> Instance:
    """Draw one instance.  ``satisfying=False`` leaves the last column random.
    ``workers`` > 1 computes the satisfying column in row chunks in parallel
    processes (same values)."""
    if mu < 1:
        raise ValueError("mu must be >= 1")
    k = gate_tables(gate, m)
    n = 1 << mu
    tabs = np.empty((k, n, 8), dtype=np.uint32)
    for t in range(k - 1):
        tabs[t] = draw_elements(seed, inst, t, n)
    if satisfying and gate == GATE_SUMPROD and sumprod_pa(m)[1] == 0:
        # a pure product vanishes where one of its factors does
        tabs[k - 1] = draw_elements(seed, inst, k - 1, n)
        zero = _stream(seed, inst, ZERO_TABLE_ID).integers(0, k, size=n)
        for t in range(k):
            tabs[t][zero == t] = 0
    elif satisfying:
        chunk = 1 << 16
        if workers > 1 and n > chunk:
            from concurrent.futures import ProcessPoolExecutor
            jobs = [(gate, tabs[:k - 1, i:i + chunk], m) for i in range(0, n, chunk)]
            with ProcessPoolExecutor(max_workers=workers) as ex:
                for i, part in zip(range(0, n, chunk), ex.map(_satisfying_chunk, jobs)):
                    tabs[k - 1, i:i + chunk] = part
        else:
            tabs[k - 1] = _satisfying_column(gate, tabs[:k - 1], m)
    else:
        tabs[k - 1] = draw_elements(seed, inst, k - 1, n)
    r = draw_elements(seed, inst, R_TABLE_ID, mu)
    return Instance(seed, inst, mu, gate, m, tabs, r)


# Named workloads (sizes and gate shapes of the paper's synthetic polynomials).
PRESETS = {
    "plain12": dict(seed=1, mu=12, gate=GATE_VANILLA, m=0),
    "plain20_d3": dict(seed=2, mu=20, gate=GATE_VANILLA, m=0),
    "plain20_d9": dict(seed=3, mu=20, gate=GATE_PROD, m=8),
}


def preset_instance(name: str, inst: int = 0) -> Instance:
    cfg = PRESETS[name]
    return make_instance(cfg["seed"], inst, cfg["mu"], cfg["gate"], cfg["m"])


# ---- batches of independent instances --------------------------------------------------

# Gate of each degree in a mixed batch: 3 the vanilla gate, otherwise the
# product gate s*w1*...*wm - o of degree m + 1.
DEGREE_GATES = {3: (GATE_VANILLA, 0), 5: (GATE_PROD, 4), 9: (GATE_PROD, 8)}
BATCH_TABLE_ID = 0xFFFE  # stream of the batch's shape draws

BATCH_PRESETS = {
    # 256 instances, mu uniform in 10..18, degree uniform in {3, 5, 9}
    "batch256": dict(seed=4, n=256, mu_lo=10, mu_hi=18, degrees=(3, 5, 9)),
}


def batch_specs(seed: int, n: int, mu_lo: int, mu_hi: int, degrees) -> list[tuple[int, int, int]]:
    """(mu, gate, m) of each instance of a batch, drawn from the batch's own stream."""
    rng = _stream(seed, 0, BATCH_TABLE_ID)
    mus = rng.integers(mu_lo, mu_hi + 1, size=n)
    degs = rng.choice(np.array(degrees), size=n)
    return [(int(mu), *DEGREE_GATES[int(d)]) for mu, d in zip(mus, degs)]


def _make_batch_item(args):
    seed, i, mu, gate, m = args
    return make_instance(seed, i, mu, gate, m)


def make_batch(seed: int, specs, workers: int = 1) -> list[Instance]:
    """Instance i of a batch is make_instance(seed, i, *specs[i])."""
    jobs = [(seed, i, mu, gate, m) for i, (mu, gate, m) in enumerate(specs)]
    if workers <= 1:
        return [_make_batch_item(j) for j in jobs]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make_batch_item, jobs, chunksize=4))


# Served stream: Poisson arrivals of single proofs, mu uniform in 14..24,
# degree 3 with probability 0.7, else 9.
SERVE_PRESETS = {
    "serve": dict(seed=5, n=500, mu_lo=14, mu_hi=24, p_d3=0.7, rhos=(0.5, 0.8, 0.95)),
}
SERVE_TABLE_ID = 0xFFFD  # stream of the requests' shape and arrival draws


def serve_specs(seed: int, n: int, mu_lo: int, mu_hi: int, p_d3: float) -> list[tuple[int, int, int]]:
    """(mu, gate, m) of each request of a served stream."""
    rng = _stream(seed, 0, SERVE_TABLE_ID)
    mus = rng.integers(mu_lo, mu_hi + 1, size=n)
    d3 = rng.random(size=n) < p_d3
    return [(int(mu), *DEGREE_GATES[3 if a else 9]) for mu, a in zip(mus, d3)]


def serve_arrivals(seed: int, n: int, rate: float, run: int = 0) -> np.ndarray:
    """Poisson arrival times (seconds) of n requests at `rate` per second."""
    rng = _stream(seed, 1 + run, SERVE_TABLE_ID)
    return np.cumsum(rng.exponential(1.0 / rate, size=n)) - 0.0


def serve_windows(seed: int, specs, top: int) -> list[int]:
    """Window index w_i of each request of a served stream: request i (size mu)
    reads rows [w_i 2^mu, (w_i + 1) 2^mu) of a 2^top-row pool, w_i uniform."""
    rng = _stream(seed, 2, SERVE_TABLE_ID)
    return [int(rng.integers(0, 1 << (top - mu))) for mu, _, _ in specs]
