"""CPU oracle for the multilinear ZeroCheck SumCheck prover and its verifier.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this file: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.

Plain, slow, obviously correct: Python integers modulo p, hashlib SHA-256,
nested loops.  Every function follows a passage of the paper "When Proofs
Meet Hardware: Comparing NTT and SumCheck in Zero-Knowledge Systems":

* Fig. 2 (right), "Multilinear ZeroCheck (SumCheck-based)": build eq_r,
  claim sum f_M(x) eq_r(x) = 0 (Eq. (1), Sec. 3.3), for i = 1..n send
  G_i(X_i) = sum over x_{i+1..n} of f_hat(alpha_1..alpha_{i-1}, X_i, x_{>i}),
  set alpha_i from a hash of G_i, finally open the MLEs at alpha.
* Sec. 3.3: the MLE interpolation form f~(x) = sum_b f(b) eq_x(b) with
  eq_x(b) = prod_i ((1-b_i)(1-x_i) + b_i x_i).
* Sec. 4.1 (SumCheck architecture): each round extends every table entry
  pair to the points of G_i, multiplies the extensions and accumulates
  over the hypercube; every round after the first first updates (folds)
  the tables with the previous challenge, halving them; eq_r is built once
  and then folded like the other tables.
* Sec. 3.4: the verifier checks G_i(0) + G_i(1) against the previous claim.

Readings taken where the paper is silent (each is listed in the design notes):

* variable order: table index b = sum_i x_i 2^(mu-i), so x_1 is the most
  significant bit and is bound first; round i pairs j and j + 2^(mu-i);
* G_i is sent as its d+2 values at X = 0..d+1 (degree d+1 = deg f_M + 1);
* Fiat-Shamir: T_0 = SHA-256("ZCv1" || u32le mu || u32le gate || u32le m ||
  enc(r_1) .. enc(r_mu)), T_i = SHA-256(T_{i-1} || enc(G_i(0)) .. enc(G_i(d+1))),
  alpha_i = (T_i read as a little-endian integer) mod p; enc = 32-byte
  little-endian canonical encoding;
* the verifier's check of Sec. 3.4 compares with G_{i-1}(alpha_{i-1});
* openings are the folded values (the commitment scheme is not modelled).
"""
from __future__ import annotations

import hashlib
import struct

# BN254 scalar field modulus.
P = 21888242871839275222246405745257275088548364400416034343698204186575808495617

GATE_VANILLA = 0
GATE_PROD = 1
GATE_SUMPROD = 2

# The polynomials of Table 1: g_1...g_P + g_{P+1} + ... + g_{P+A}, as (P, A);
# the gate parameter is m = P + 16 A.
TABLE1_SHAPES = ((2, 0), (2, 1), (2, 2), (2, 3), (3, 0), (4, 0))


def sumprod_pa(m: int) -> tuple[int, int]:
    pa = (m & 15, m >> 4)
    if pa not in TABLE1_SHAPES:
        raise ValueError(f"not a Table 1 shape: m={m}")
    return pa


# ----------------------------------------------------------------- field ---

def inv(x: int) -> int:
    """Inverse in F_p by Fermat's little theorem (p is prime)."""
    if x % P == 0:
        raise ZeroDivisionError("inverse of 0")
    return pow(x, P - 2, P)


def enc(x: int) -> bytes:
    """32-byte little-endian canonical encoding of a field element."""
    return (x % P).to_bytes(32, "little")


# ------------------------------------------------------------------ gate ---

def gate_degree(gate: int, m: int) -> int:
    if gate == GATE_VANILLA:
        return 3
    if gate == GATE_PROD:
        return m + 1
    if gate == GATE_SUMPROD:
        return sumprod_pa(m)[0]
    raise ValueError(f"unknown gate {gate}")


def gate_ntables(gate: int, m: int) -> int:
    if gate == GATE_VANILLA:
        return 8
    if gate == GATE_PROD:
        return m + 2
    if gate == GATE_SUMPROD:
        pp, aa = sumprod_pa(m)
        return pp + aa
    raise ValueError(f"unknown gate {gate}")


def gate_value(gate: int, m: int, v) -> int:
    """f_M evaluated on one value per witness table (gate column order).

    Vanilla gate [a, b, c, qM, qL, qR, qO, qC]:
        f = qM*a*b + qL*a + qR*b + qO*c + qC                      (degree 3)
    Product gate [s, w1, .., wm, o]:
        f = s*w1*...*wm - o                                        (degree m+1)
    Table 1 shapes [g1 .. gP, gP+1 .. gP+A] (m = P + 16 A):
        f = g1*...*gP + gP+1 + ... + gP+A                          (degree P)
    """
    if gate == GATE_VANILLA:
        a, b, c, qm, ql, qr, qo, qc = v
        return (qm * a * b + ql * a + qr * b + qo * c + qc) % P
    if gate == GATE_PROD:
        prod = v[0]
        for w in v[1:1 + m]:
            prod = prod * w % P
        return (prod - v[1 + m]) % P
    if gate == GATE_SUMPROD:
        pp, aa = sumprod_pa(m)
        prod = 1
        for g in v[:pp]:
            prod = prod * g % P
        return (prod + sum(v[pp:pp + aa])) % P
    raise ValueError(f"unknown gate {gate}")


# -------------------------------------------------------------------- eq ---

def eq1(x: int, r: int) -> int:
    """One factor (1-x)(1-r) + x r of eq (Sec. 3.3, Fig. 2 Build MLE)."""
    return ((1 - x) * (1 - r) + x * r) % P


def eq_point(x, r) -> int:
    """eq(x, r) = prod_i ((1-x_i)(1-r_i) + x_i r_i) for field points x, r."""
    acc = 1
    for xi, ri in zip(x, r, strict=True):
        acc = acc * eq1(xi, ri) % P
    return acc


def bits_msb_first(b: int, mu: int) -> list[int]:
    """(x_1, .., x_mu) of table index b, x_1 = most significant bit."""
    return [(b >> (mu - 1 - i)) & 1 for i in range(mu)]


def eq_table(r) -> list[int]:
    """Build MLE: E[b] = eq(bits(b), r) for every b, entry by entry (definition)."""
    mu = len(r)
    return [eq_point(bits_msb_first(b, mu), r) for b in range(1 << mu)]


# ------------------------------------------------------------- MLE form ---

def mle_eval(table, z) -> int:
    """MLE interpolation form of Sec. 3.3: sum_b table[b] * eq_z(b)."""
    mu = len(z)
    assert len(table) == 1 << mu
    acc = 0
    for b, tb in enumerate(table):
        acc += tb * eq_point(bits_msb_first(b, mu), z)
    return acc % P


# ------------------------------------------------------------ transcript ---

def transcript_init(mu: int, gate: int, m: int, r) -> bytes:
    msg = b"ZCv1" + struct.pack("<III", mu, gate, m) + b"".join(enc(x) for x in r)
    return hashlib.sha256(msg).digest()


def transcript_round(prev: bytes, evals) -> tuple[bytes, int]:
    """Absorb one round message; return (T_i, alpha_i)."""
    t = hashlib.sha256(prev + b"".join(enc(g) for g in evals)).digest()
    return t, int.from_bytes(t, "little") % P


# ---------------------------------------------------------------- prover ---

def round_poly(gate: int, m: int, tabs, d: int) -> list[int]:
    """G_i at X = 0..d+1 from the current (folded) tables, eq table last.

    For j < h = len/2 each table's pair (t[j], t[j+h]) is extended to
    t(X) = t[j] + X (t[j+h] - t[j]); the summand is f_M(ext) * eq(ext).
    """
    h = len(tabs[0]) // 2
    out = []
    for x in range(d + 2):
        s = 0
        for j in range(h):
            ext = [(t[j] + x * (t[j + h] - t[j])) % P for t in tabs]
            s += gate_value(gate, m, ext[:-1]) * ext[-1]
        out.append(s % P)
    return out


def fold(t, alpha: int) -> list[int]:
    """Bind the leading variable to alpha: t'[j] = t[j] + alpha (t[j+h] - t[j])."""
    h = len(t) // 2
    return [(t[j] + alpha * (t[j + h] - t[j])) % P for j in range(h)]


def prove(mu: int, gate: int, m: int, tables, r, keep_tables: bool = False):
    """Whole proof.  Returns dict with evals [mu][d+2], alphas [mu], openings.

    openings = the single value left in every witness table (gate order)
    after the last fold, then eq's.  With keep_tables, ``tables_after[i]``
    holds every table (eq last) after folding with alpha_{i+1}.
    """
    d = gate_degree(gate, m)
    assert len(tables) == gate_ntables(gate, m)
    assert len(r) == mu and all(len(t) == 1 << mu for t in tables)
    tabs = [[v % P for v in t] for t in tables] + [eq_table(r)]
    ts = transcript_init(mu, gate, m, r)
    evals, alphas, after = [], [], []
    for _ in range(mu):
        g = round_poly(gate, m, tabs, d)
        ts, alpha = transcript_round(ts, g)
        tabs = [fold(t, alpha) for t in tabs]
        evals.append(g)
        alphas.append(alpha)
        if keep_tables:
            after.append([list(t) for t in tabs])
    res = {"evals": evals, "alphas": alphas, "openings": [t[0] for t in tabs],
           "transcript": ts}
    if keep_tables:
        res["tables_after"] = after
    return res


# -------------------------------------------------------------- verifier ---

def lagrange_eval(vals, x: int) -> int:
    """Value at x of the polynomial of degree < len(vals) through (k, vals[k])."""
    n = len(vals)
    acc = 0
    for k in range(n):
        num, den = 1, 1
        for j in range(n):
            if j != k:
                num = num * (x - j) % P
                den = den * (k - j) % P
        acc += vals[k] * num * inv(den)
    return acc % P


def verify(mu: int, gate: int, m: int, r, evals, alphas, openings) -> bool:
    """Verifier of the non-interactive ZeroCheck (Fig. 2 right, Sec. 3.4).

    claim_0 = 0 (Eq. (1)); per round G_i(0)+G_i(1) = claim_{i-1}, alpha_i
    recomputed from the transcript, claim_i = G_i(alpha_i); at the end
    claim_mu = f_M(openings) * eq(alpha, r), with eq(alpha, r) computed
    from alpha and r directly, and the eq opening must equal it.
    """
    d = gate_degree(gate, m)
    k = gate_ntables(gate, m)
    if len(evals) != mu or len(alphas) != mu or len(openings) != k + 1:
        return False
    ts = transcript_init(mu, gate, m, r)
    claim = 0
    for i in range(mu):
        g = [v % P for v in evals[i]]
        if len(g) != d + 2 or (g[0] + g[1]) % P != claim:
            return False
        ts, alpha = transcript_round(ts, g)
        if alpha != alphas[i] % P:
            return False
        claim = lagrange_eval(g, alpha)
    e = eq_point(alphas, r)
    if openings[-1] % P != e:
        return False
    return claim == gate_value(gate, m, [o % P for o in openings[:-1]]) * e % P


# ----------------------------------------------- brute force (tiny mu) ---

def round_poly_bruteforce(gate: int, m: int, tables, r, alphas_prefix, d: int) -> list[int]:
    """G_i straight from Fig. 2: MLEs evaluated by the interpolation form.

    i = len(alphas_prefix) + 1.  No folding: every table's MLE and eq_r are
    evaluated at (alpha_1..alpha_{i-1}, X, x_{i+1}..x_mu) for every Boolean
    suffix.  Exponential cost; for mu <= 5.
    """
    mu = len(r)
    i = len(alphas_prefix) + 1
    rest = mu - i
    out = []
    for x in range(d + 2):
        s = 0
        for suf in range(1 << rest):
            z = list(alphas_prefix) + [x] + bits_msb_first(suf, rest)
            vals = [mle_eval(t, z) for t in tables]
            s += gate_value(gate, m, vals) * eq_point(z, r)
        out.append(s % P)
    return out
