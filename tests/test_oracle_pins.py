"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a textbook
identity, a published test vector, a different algorithm for the same
quantity, brute force from the MLE interpolation form, the protocol's own
invariants (Eq. (1), the round check of Sec. 3.4) or a hand-worked example.
"""
import hashlib
import random

import pytest

from oracle import zc_oracle as O
from paper_2606_16146_amd import inputs as I

P_HEX = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
BN_U = 4965661367192848881  # BN254 curve parameter


def _is_probable_prime(n, rounds=40):
    if n < 2:
        return False
    for sp in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % sp == 0:
            return n == sp
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(12345)
    for _ in range(rounds):
        a = rng.randrange(2, n - 2)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


# ------------------------------------------------------------- constants ---

def test_modulus_is_bn254_scalar_field():
    assert O.P == P_HEX == I.P
    # BN family: group order r(u) = 36u^4 + 36u^3 + 18u^2 + 6u + 1
    u = BN_U
    assert O.P == 36 * u**4 + 36 * u**3 + 18 * u**2 + 6 * u + 1
    assert O.P.bit_length() == 254
    assert _is_probable_prime(O.P)
    # 2-adicity 28
    assert (O.P - 1) % (1 << 28) == 0 and ((O.P - 1) >> 28) % 2 == 1


def test_sha256_fips180_vectors():
    # FIPS 180-4 / NIST example messages
    assert hashlib.sha256(b"abc").hexdigest() == (
        "ba7816bf8f01cfea414140de5dae2223b00361a396177a9cb410ff61f20015ad")
    assert hashlib.sha256(b"").hexdigest() == (
        "e3b0c44298fc1c149afbf4c8996fb92427ae41e4649b934ca495991b7852b855")
    assert hashlib.sha256(
        b"abcdbcdecdefdefgefghfghighijhijkijkljklmklmnlmnomnopnopq").hexdigest() == (
        "248d6a61d20638b8e5c026930c3e6039a33ce45964ff2167f6ecedd419db06c1")


def test_field_inverse_and_encoding():
    rng = random.Random(1)
    for _ in range(50):
        x = rng.randrange(1, O.P)
        assert x * O.inv(x) % O.P == 1
        assert int.from_bytes(O.enc(x), "little") == x
    assert O.enc(O.P) == bytes(32)
    assert O.enc(-1) == (O.P - 1).to_bytes(32, "little")


# -------------------------------------------------------------------- eq ---

def _eq_tree(r):
    """Tree construction of eq_r (doubling; a different algorithm)."""
    t = [1]
    for ri in r:
        nxt = []
        for v in t:
            nxt.append(v * (1 - ri) % O.P)
            nxt.append(v * ri % O.P)
        t = nxt
    return t


@pytest.mark.parametrize("mu", [1, 2, 3, 5, 7])
def test_eq_table_definition_vs_tree_and_sum(mu):
    rng = random.Random(mu)
    r = [rng.randrange(O.P) for _ in range(mu)]
    e = O.eq_table(r)
    assert e == _eq_tree(r)
    assert sum(e) % O.P == 1  # sum over the cube of prod (1-x)(1-r)+xr = prod 1


def test_eq_boolean_point_is_indicator_msb_first():
    mu = 4
    for b in range(1 << mu):
        r = O.bits_msb_first(b, mu)
        e = O.eq_table(r)
        assert e == [1 if j == b else 0 for j in range(1 << mu)]
    # x_1 is the most significant bit of the index
    assert O.bits_msb_first(0b1000, 4) == [1, 0, 0, 0]


# ------------------------------------------------------------------- MLE ---

def test_mle_interpolates_and_is_multilinear():
    rng = random.Random(7)
    mu = 4
    t = [rng.randrange(O.P) for _ in range(1 << mu)]
    for b in range(1 << mu):
        assert O.mle_eval(t, O.bits_msb_first(b, mu)) == t[b]
    z = [rng.randrange(O.P) for _ in range(mu)]
    for i in range(mu):
        z0, z1, z2 = list(z), list(z), list(z)
        z0[i], z1[i], z2[i] = 0, 1, 2
        f0, f1, f2 = (O.mle_eval(t, zz) for zz in (z0, z1, z2))
        assert (f2 - (2 * f1 - f0)) % O.P == 0  # affine in each variable


def test_folding_all_variables_equals_mle_at_point():
    rng = random.Random(8)
    mu = 5
    t = [rng.randrange(O.P) for _ in range(1 << mu)]
    a = [rng.randrange(O.P) for _ in range(mu)]
    f = t
    for ai in a:
        f = O.fold(f, ai)
    assert f == [O.mle_eval(t, a)]


# ------------------------------------------------------- prover vs MLE ---

T1 = [I.sumprod_m(pp, aa) for pp, aa in I.TABLE1_SHAPES]  # the polynomials of Table 1
CASES = [(3, O.GATE_VANILLA, 0), (4, O.GATE_VANILLA, 0), (3, O.GATE_PROD, 2),
         (4, O.GATE_PROD, 4), (2, O.GATE_PROD, 8), (3, O.GATE_PROD, 1)] + \
        [(3 + (i % 2), O.GATE_SUMPROD, m) for i, m in enumerate(T1)]


@pytest.mark.parametrize("mu,gate,m", CASES)
def test_round_polys_equal_bruteforce_interpolation_form(mu, gate, m):
    inst = I.make_instance(100 + mu, 0, mu, gate, m, satisfying=(gate == O.GATE_VANILLA))
    tabs, r = inst.tables_int(), inst.r_int()
    d = O.gate_degree(gate, m)
    res = O.prove(mu, gate, m, tabs, r)
    for i in range(mu):
        bf = O.round_poly_bruteforce(gate, m, tabs, r, res["alphas"][:i], d)
        assert res["evals"][i] == bf, f"round {i + 1}"
    # openings are the MLEs at alpha; the eq opening is eq(alpha, r)
    for t, o in zip(tabs, res["openings"][:-1]):
        assert o == O.mle_eval(t, res["alphas"])
    assert res["openings"][-1] == O.eq_point(res["alphas"], r)


@pytest.mark.parametrize("mu,gate,m", [(6, O.GATE_VANILLA, 0), (5, O.GATE_PROD, 4),
                                       (4, O.GATE_PROD, 8)] + [(5, O.GATE_SUMPROD, m) for m in T1])
def test_claim_chain_first_claim_zero_and_verifier(mu, gate, m):
    inst = I.make_instance(7, 1, mu, gate, m)
    tabs, r = inst.tables_int(), inst.r_int()
    res = O.prove(mu, gate, m, tabs, r)
    ev, al = res["evals"], res["alphas"]
    assert (ev[0][0] + ev[0][1]) % O.P == 0  # Eq. (1): the first claim is 0
    for i in range(1, mu):
        assert (ev[i][0] + ev[i][1]) % O.P == O.lagrange_eval(ev[i - 1], al[i - 1])
    assert O.verify(mu, gate, m, r, ev, al, res["openings"])


@pytest.mark.parametrize("gate,m", [(O.GATE_VANILLA, 0), (O.GATE_PROD, 2), (O.GATE_PROD, 8),
                                    (O.GATE_SUMPROD, 2), (O.GATE_SUMPROD, 50), (O.GATE_SUMPROD, 4)])
def test_round_poly_degree_extra_point_on_interpolant(gate, m):
    """G_i has degree d+1: its value at X=d+2 lies on the interpolant of 0..d+1."""
    mu = 4
    inst = I.make_instance(3, 2, mu, gate, m)
    tabs = inst.tables_int() + [O.eq_table(inst.r_int())]
    d = O.gate_degree(gate, m)
    rng = random.Random(5)
    for _ in range(mu):
        g = O.round_poly(gate, m, tabs, d + 1)  # d+3 values
        assert O.lagrange_eval(g[: d + 2], d + 2) == g[d + 2]
        tabs = [O.fold(t, rng.randrange(O.P)) for t in tabs]


def test_transcript_rule():
    r = [1, 2, 3]
    t0 = O.transcript_init(3, 0, 0, r)
    msg = b"ZCv1" + (3).to_bytes(4, "little") + bytes(8) + b"".join(
        x.to_bytes(32, "little") for x in r)
    assert t0 == hashlib.sha256(msg).digest()
    t1, a1 = O.transcript_round(t0, [O.P - 1, 5])
    assert t1 == hashlib.sha256(t0 + (O.P - 1).to_bytes(32, "little") + (5).to_bytes(32, "little")).digest()
    assert a1 == int.from_bytes(t1, "little") % O.P and 0 <= a1 < O.P


# ---------------------------------------------------------- special cases ---

def test_r_zero_selects_index_zero_pair():
    mu = 4
    inst = I.make_instance(9, 0, mu, O.GATE_VANILLA, 0, satisfying=False)
    tabs = inst.tables_int()
    r = [0] * mu
    res = O.prove(mu, O.GATE_VANILLA, 0, tabs, r)
    h = 1 << (mu - 1)
    want = []
    for x in range(5):
        ext = [(t[0] + x * (t[h] - t[0])) % O.P for t in tabs]
        want.append(O.gate_value(O.GATE_VANILLA, 0, ext) * (1 - x) % O.P)
    assert res["evals"][0] == want


def test_all_zero_tables_give_zero_polys():
    mu = 5
    tabs = [[0] * (1 << mu) for _ in range(8)]
    r = [11, 22, 33, 44, 55]
    res = O.prove(mu, O.GATE_VANILLA, 0, tabs, r)
    assert all(v == 0 for g in res["evals"] for v in g)
    assert O.verify(mu, O.GATE_VANILLA, 0, r, res["evals"], res["alphas"], res["openings"])


def test_mu1_hand_worked_example():
    """mu=1, product gate m=1: f = s*w1 - o with s=[2,3], w1=[5,7], o=[10,21], r=5.

    s(X)=2+X, w(X)=5+2X, o(X)=10+11X, so f(X) = 2X^2 - 2X; eq(X,5) = 1-5-X+10X = 9X-4.
    G(0)=0, G(1)=0, G(2)=4*14=56, G(3)=12*23=276.
    """
    res = O.prove(1, O.GATE_PROD, 1, [[2, 3], [5, 7], [10, 21]], [5])
    assert res["evals"] == [[0, 0, 56, 276]]
    a = res["alphas"][0]
    assert res["openings"] == [(2 + a) % O.P, (5 + 2 * a) % O.P, (10 + 11 * a) % O.P,
                               (9 * a - 4) % O.P]
    assert O.verify(1, O.GATE_PROD, 1, [5], res["evals"], res["alphas"], res["openings"])


# ---------------------------------------------------------------- negative ---

def test_nonsatisfying_witness_is_rejected():
    mu = 5
    inst = I.make_instance(21, 0, mu, O.GATE_VANILLA, 0)
    tabs, r = inst.tables_int(), inst.r_int()
    tabs[7][3] = (tabs[7][3] + 1) % O.P  # perturb one qC entry
    res = O.prove(mu, O.GATE_VANILLA, 0, tabs, r)
    assert (res["evals"][0][0] + res["evals"][0][1]) % O.P != 0
    assert not O.verify(mu, O.GATE_VANILLA, 0, r, res["evals"], res["alphas"], res["openings"])


def test_tampered_messages_are_rejected():
    mu = 4
    inst = I.make_instance(22, 0, mu, O.GATE_PROD, 2)
    tabs, r = inst.tables_int(), inst.r_int()
    res = O.prove(mu, O.GATE_PROD, 2, tabs, r)
    ev, al, op = res["evals"], res["alphas"], res["openings"]
    assert O.verify(mu, O.GATE_PROD, 2, r, ev, al, op)
    bad = [list(g) for g in ev]
    bad[2][3] = (bad[2][3] + 1) % O.P
    assert not O.verify(mu, O.GATE_PROD, 2, r, bad, al, op)
    bad_op = list(op)
    bad_op[1] = (bad_op[1] + 1) % O.P
    assert not O.verify(mu, O.GATE_PROD, 2, r, ev, al, bad_op)
    bad_al = list(al)
    bad_al[0] = (bad_al[0] + 1) % O.P
    assert not O.verify(mu, O.GATE_PROD, 2, r, ev, bad_al, op)


# --------------------------------------------------------------- generator ---

@pytest.mark.parametrize("gate,m", [(O.GATE_VANILLA, 0), (O.GATE_PROD, 4), (O.GATE_PROD, 8)] +
                         [(O.GATE_SUMPROD, m) for m in T1])
def test_generator_witness_satisfies_gate(gate, m):
    inst = I.make_instance(5, 3, 6, gate, m)
    tabs = inst.tables_int()
    assert all(0 <= v < O.P for t in tabs for v in t)
    for b in range(1 << 6):
        assert O.gate_value(gate, m, [t[b] for t in tabs]) == 0


def test_generator_is_deterministic_and_streams_differ():
    a = I.make_instance(5, 0, 5, O.GATE_VANILLA, 0)
    b = I.make_instance(5, 0, 5, O.GATE_VANILLA, 0)
    c = I.make_instance(5, 1, 5, O.GATE_VANILLA, 0)
    assert (a.tables == b.tables).all() and (a.r == b.r).all()
    assert not (a.tables == c.tables).all()
    assert len({bytes(t) for t in a.tables}) == a.k


def test_table1_gate_values_by_hand():
    """The Table 1 polynomials on small integers, written out by hand."""
    v = [2, 3, 5, 7, 11]
    assert O.gate_value(O.GATE_SUMPROD, I.sumprod_m(2, 0), v[:2]) == 6            # g1 g2
    assert O.gate_value(O.GATE_SUMPROD, I.sumprod_m(2, 1), v[:3]) == 6 + 5        # g1 g2 + g3
    assert O.gate_value(O.GATE_SUMPROD, I.sumprod_m(2, 2), v[:4]) == 6 + 5 + 7
    assert O.gate_value(O.GATE_SUMPROD, I.sumprod_m(2, 3), v[:5]) == 6 + 5 + 7 + 11
    assert O.gate_value(O.GATE_SUMPROD, I.sumprod_m(3, 0), v[:3]) == 30           # g1 g2 g3
    assert O.gate_value(O.GATE_SUMPROD, I.sumprod_m(4, 0), v[:4]) == 210          # g1 g2 g3 g4
    # degree, unique polynomials and additive terms as Table 1 lists them
    for (pp, aa), (d, uniq, terms) in zip(I.TABLE1_SHAPES, [(2, 2, 1), (2, 3, 2), (2, 4, 3), (2, 5, 4),
                                                             (3, 3, 1), (4, 4, 1)]):
        m = I.sumprod_m(pp, aa)
        assert O.gate_degree(O.GATE_SUMPROD, m) == d
        assert O.gate_ntables(O.GATE_SUMPROD, m) == uniq
        assert aa + 1 == terms
    with pytest.raises(ValueError):
        O.gate_degree(O.GATE_SUMPROD, I.sumprod_m(3, 1))  # not in Table 1
