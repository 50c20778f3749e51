"""Parity of the HIP prover with the CPU oracle (GPU).

Small instances are compared with the Python oracle element by element
(round polynomials, challenges, openings and, through the stepping API,
every folded table); full-size instances (mu = 20, degree 3 and 9) with the
C oracle, which itself matches the Python oracle byte for byte.
"""
import numpy as np
import pytest
import torch

from oracle import c_oracle as C
from oracle import zc_oracle as O
from paper_2606_16146_amd import inputs as I
from tests._helpers import P, R_MONT, dev, gpu_prove, ints_of, limbs_of, same_as_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zc():
    from paper_2606_16146_amd import zc as z
    z.lib()
    return z


SMALL = [(1, 0, 0), (2, 0, 0), (3, 0, 0), (5, 0, 0), (9, 0, 0), (10, 0, 0),
         (1, 1, 1), (4, 1, 1), (6, 1, 2), (7, 1, 3), (8, 1, 4), (5, 1, 5), (6, 1, 6), (4, 1, 7),
         (7, 1, 8), (2, 1, 8),
         # the polynomials of Table 1
         (1, 2, 2), (7, 2, 2), (8, 2, 18), (6, 2, 34), (9, 2, 50), (5, 2, 3), (10, 2, 4)]


@pytest.mark.parametrize("mu,gate,m", SMALL)
def test_prove_matches_python_oracle(zc, mu, gate, m):
    inst = I.make_instance(500 + mu, m, mu, gate, m)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = O.prove(mu, gate, m, inst.tables_int(), inst.r_int())
    same_as_oracle(res, ora)


def test_plain12_matches_python_oracle_and_verifies(zc):
    inst = I.preset_instance("plain12")
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = O.prove(inst.mu, inst.gate, inst.m, inst.tables_int(), inst.r_int())
    same_as_oracle(res, ora)
    ev = [ints_of(res["evals"][i]) for i in range(inst.mu)]
    assert O.verify(inst.mu, inst.gate, inst.m, inst.r_int(), ev, ints_of(res["alphas"]),
                    ints_of(res["openings"]))


@pytest.mark.parametrize("mu,gate,m", [(6, 0, 0), (5, 1, 4), (4, 1, 8)])
def test_nonsatisfying_witness_still_matches(zc, mu, gate, m):
    inst = I.make_instance(77, 0, mu, gate, m, satisfying=False)
    res = gpu_prove(inst)
    ora = O.prove(mu, gate, m, inst.tables_int(), inst.r_int())
    same_as_oracle(res, ora)
    assert not O.verify(mu, gate, m, inst.r_int(), ora["evals"], ora["alphas"], ora["openings"])


@pytest.mark.parametrize("gate,m", [(0, 0), (1, 8), (1, 4)])
def test_extreme_values_worst_case_extensions(zc, gate, m):
    """Every pair is (0, p-1) in the internal form: Delta = p-1, the largest extensions."""
    mu = 5
    k = 8 if gate == 0 else m + 2
    n = 1 << mu
    top = (P - 1) * pow(R_MONT, -1, P) % P  # packs to p-1
    vals = [0] * (n // 2) + [top] * (n // 2)
    tables = np.stack([limbs_of(vals) for _ in range(k)])
    r = limbs_of([P - 1] * mu)
    inst = I.Instance(0, 0, mu, gate, m, tables, r)
    res = gpu_prove(inst)
    ora = O.prove(mu, gate, m, inst.tables_int(), inst.r_int())
    same_as_oracle(res, ora)


@pytest.mark.parametrize("mu,gate,m", [(7, 0, 0), (6, 1, 8), (5, 1, 2)])
def test_stepping_matches_fused_and_folded_tables(zc, mu, gate, m):
    inst = I.make_instance(900 + mu, 0, mu, gate, m)
    fused = gpu_prove(inst)
    ora = O.prove(mu, gate, m, inst.tables_int(), inst.r_int(), keep_tables=True)
    s = zc.shape(mu, gate, m)
    ws = zc.new_workspace(s)
    tabs = [zc.pack(dev(t), ws) for t in inst.tables]
    r = dev(inst.r)
    ev, al, _ = zc.new_outputs(s)
    n = 1 << mu
    for i in range(1, mu + 1):
        zc.round_(s, tabs, r, ws, i, ev, al)
        zc.fold(s, tabs, ws, i)
        live = n >> i
        after = ora["tables_after"][i - 1]
        for t in range(len(tabs)):
            assert ints_of(zc.unpack(tabs[t], live)) == after[t], (i, t)
    assert zc.read_error(ws) == 0
    assert (ev.cpu().numpy() == fused["evals"]).all()
    assert (al.cpu().numpy() == fused["alphas"]).all()
    openings = [ints_of(zc.unpack(t, 1))[0] for t in tabs]
    assert openings == ints_of(fused["openings"])[:-1]


def test_stepping_out_of_order_is_flagged(zc):
    mu = 4
    inst = I.make_instance(3, 0, mu, 0, 0)
    s = zc.shape(mu, 0, 0)
    ws = zc.new_workspace(s)
    tabs = [zc.pack(dev(t), ws) for t in inst.tables]
    r = dev(inst.r)
    ev, al, _ = zc.new_outputs(s)
    zc.round_(s, tabs, r, ws, 1, ev, al)
    zc.round_(s, tabs, r, ws, 2, ev, al)  # fold(1) skipped
    assert zc.read_error(ws) == zc.ZC_ESTATE


def test_pack_flags_noncanonical_and_unpack_roundtrips(zc):
    s = zc.shape(4, 0)
    ws = zc.new_workspace(s)
    vals = [0, 1, P - 1, 12345, P, (1 << 256) - 1]
    t = zc.pack(dev(limbs_of(vals)), ws)
    assert zc.read_error(ws) == zc.ZC_ERANGE
    ok = [0, 1, P - 1, 12345, P // 3]
    t = zc.pack(dev(limbs_of(ok)), ws)
    assert ints_of(zc.unpack(t)) == ok
    # packed form is x * 2^261 mod p, limb-planar
    planar = t.cpu().numpy()
    assert ints_of(planar.T.copy()) == [x * R_MONT % P for x in ok]


def test_r_not_canonical_is_flagged(zc):
    inst = I.make_instance(4, 0, 3, 0, 0)
    inst.r[1] = limbs_of([P])[0]
    res = gpu_prove(inst)
    assert res["err"] == zc.ZC_ERANGE


def test_repeat_runs_are_identical_and_tables_untouched(zc):
    inst = I.make_instance(8, 0, 11, 1, 4)
    res = gpu_prove(inst)
    before = [t.clone() for t in res["tables"]]
    again = zc.prove(res["shape"], res["tables"], res["r"], res["ws"])
    torch.cuda.synchronize()
    for a, b in zip(before, res["tables"]):
        assert torch.equal(a, b)
    assert (again[0].cpu().numpy() == res["evals"]).all()
    assert (again[2].cpu().numpy() == res["openings"]).all()


@pytest.mark.parametrize("m", [2, 18, 34, 50, 3, 4])
def test_table1_shapes_mu16_match_c_oracle(zc, m):
    inst = I.make_instance(41, m, 16, 2, m)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = C.prove(16, 2, m, inst.tables, inst.r)
    assert np.array_equal(res["evals"], ora["evals"]) and np.array_equal(res["alphas"], ora["alphas"])
    assert np.array_equal(res["openings"], ora["openings"])


@pytest.mark.parametrize("gate,m", [(0, 0), (1, 8), (1, 2), (2, 34), (2, 4)])
def test_extreme_values_thread_per_pair_rounds(zc, gate, m):
    """Internal values 0 and p-1 mixed at random (seeded) at mu = 16, where
    round 1 and the next rounds run the thread-per-pair kernels and their
    lazy bounds: every combination of extremes in a pair (t[j], t[j+q]),
    among them the largest unreduced difference (0, p-1), reaches the round-1
    extensions and products; r mixes p-1 and 1."""
    mu, n = 16, 1 << 16
    k = zc.table_count(zc.shape(mu, gate, m))
    top = limbs_of([(P - 1) * pow(R_MONT, -1, P) % P])[0]  # packs to p-1
    rng = np.random.default_rng(2024 + 16 * gate + m)
    tables = np.stack([np.where(rng.integers(0, 2, (n, 1)) == 1, top, 0).astype(np.uint32) for _ in range(k)])
    r = limbs_of([P - 1 if b else 1 for b in rng.integers(0, 2, mu)])
    inst = I.Instance(0, 0, mu, gate, m, tables, r)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = C.prove(mu, gate, m, inst.tables, inst.r)
    assert np.array_equal(res["evals"], ora["evals"]) and np.array_equal(res["alphas"], ora["alphas"])
    assert np.array_equal(res["openings"], ora["openings"])


@pytest.mark.parametrize("mu,gate,m", [(16, 0, 0), (17, 0, 0), (18, 0, 0), (17, 1, 2), (17, 1, 1), (17, 2, 3),
                                       (17, 2, 50), (18, 2, 2), (17, 2, 4), (17, 1, 3),
                                       (16, 1, 8), (17, 1, 8), (18, 1, 8), (19, 1, 4)])
def test_fused_schedule_boundaries_match_c_oracle(zc, mu, gate, m):
    """Around the sizes where the fused lane-split rounds switch on (at least
    two thread-per-pair rounds: from mu = 17): speculative for gates of
    degree <= 3, waiting for the challenge beside the finisher for degree 4,
    5 and 9, against the C oracle."""
    import ctypes
    s = zc.shape(mu, gate, m)
    kinds = [zc.lib().zc_prove_round_kernel(ctypes.byref(s), i) for i in range(1, mu + 1)]
    assert (5 in kinds) == (mu >= 17), kinds
    inst = I.make_instance(60 + mu, m, mu, gate, m)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = C.prove(mu, gate, m, inst.tables, inst.r)
    assert np.array_equal(res["evals"], ora["evals"]) and np.array_equal(res["alphas"], ora["alphas"])
    assert np.array_equal(res["openings"], ora["openings"])


def test_profiled_prove_equals_prove(zc):
    """The event-bracketed proof (the bench's path) gives the same bytes as
    zc_prove, on a speculative schedule."""
    inst = I.make_instance(71, 0, 17, 0, 0)
    s = zc.shape(17, 0, 0)
    ref = gpu_prove(inst)
    ws = zc.new_workspace(s)
    tabs = [zc.pack(dev(t), ws) for t in inst.tables]
    ev = zc.HipEvents(2 * 17)
    out = zc.prove_profiled(s, tabs, dev(inst.r), ws, ev)
    assert zc.read_error(ws) == 0
    for a, b in zip(out, (ref["evals"], ref["alphas"], ref["openings"])):
        assert np.array_equal(a.cpu().numpy(), b)
    assert all(ev.elapsed_ms(2 * i, 2 * i + 1) >= 0 for i in range(17))


@pytest.mark.parametrize("mu,gate,m,seed", [(17, 0, 0, 1), (19, 0, 0, 2), (19, 1, 8, 3), (19, 2, 18, 4),
                                            (18, 0, 0, 5), (18, 1, 8, 6), (21, 1, 5, 7)])
def test_two_wave_round_matches_c_oracle(zc, mu, gate, m, seed):
    """The last thread-per-pair round (32768 pairs) in its two-wave form:
    from the caller's tables at mu = 17 (round 2), out of place in the moved
    region of the folded tables at mu = 19 and 21 (points split for the
    product and Table 1 gates, terms split for the vanilla gate); at mu = 18
    it runs on one wave in place.  Against the C oracle."""
    inst = I.make_instance(70 + seed, m, mu, gate, m, workers=8)
    print(f"two-wave round mu={mu} gate={gate} m={m}", flush=True)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = C.prove(mu, gate, m, inst.tables, inst.r)
    assert np.array_equal(res["evals"], ora["evals"]) and np.array_equal(res["alphas"], ora["alphas"])
    assert np.array_equal(res["openings"], ora["openings"])


@pytest.mark.parametrize("name", ["plain20_d3", "plain20_d9"])
def test_full_size_matches_c_oracle(zc, name):
    inst = I.preset_instance(name)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = C.prove(inst.mu, inst.gate, inst.m, inst.tables, inst.r)
    assert (res["evals"] == ora["evals"]).all()
    assert (res["alphas"] == ora["alphas"]).all()
    assert (res["openings"] == ora["openings"]).all()


@pytest.mark.parametrize("mu,gate,m", [(24, I.GATE_VANILLA, 0), (23, I.GATE_PROD, 8)])
def test_large_mu_multichunk_lazy_sums_match_c_oracle(zc, mu, gate, m):
    """mu = 23-24: round 1's grid is one resident generation (one 256-thread
    block per CU at these kernels' register use), so its 2^(mu-1) pairs give
    every thread 64 or 128 pairs, several chunks of lazily summed pairs with
    a reduction between them (mu = 20 has 8 pairs per thread, a single
    chunk); the grid-stride loops of rounds 2-5 also take several pairs per
    thread.  Compared with the C oracle."""
    inst = I.make_instance(7, 0, mu, gate, m, workers=8)
    res = gpu_prove(inst)
    assert res["err"] == 0
    ora = C.prove(inst.mu, inst.gate, inst.m, inst.tables, inst.r)
    assert (res["evals"] == ora["evals"]).all()
    assert (res["alphas"] == ora["alphas"]).all()
    assert (res["openings"] == ora["openings"]).all()


@pytest.mark.parametrize("mu,gate,m,top,win,extra", [
    (17, 0, 0, 18, 1, 96),   # speculative rounds, plane pitch not a power of two
    (12, 1, 8, 14, 3, 0),    # degree 9, window 3 of a mu = 14 pool
    (9, 2, 34, 10, 1, 5),    # a Table 1 polynomial, odd pitch
    (1, 0, 0, 3, 3, 0),      # one round, the last window
])
def test_prove_pitch_on_a_window_matches_c_oracle_and_copy(zc, mu, gate, m, top, win, extra):
    """zc_prove_pitch reads a 2^mu-row window of larger packed tables in place
    (planes `pitch` apart): the same bytes as zc_prove on a copy of the window
    and as the C oracle on those rows; the pool is left untouched."""
    base = I.make_instance(81, mu, top, gate, m, workers=8)
    s = zc.shape(mu, gate, m)
    ws = zc.new_workspace(s)
    pitch = (1 << top) + extra
    pool = []
    for t in base.tables:
        wide = torch.zeros((8, pitch), dtype=torch.uint32, device="cuda")
        wide[:, :1 << top] = zc.pack(dev(t), ws)
        pool.append(wide)
    before = [p.clone() for p in pool]
    off, n = win << mu, 1 << mu
    r = I.draw_elements(82, mu, I.R_TABLE_ID, mu)
    got = zc.prove(s, [p[:, off:off + n] for p in pool], dev(r), ws, pitch=pitch)
    got = [o.cpu().numpy() for o in got]
    assert zc.read_error(ws) == 0
    canon = np.ascontiguousarray(base.tables[:, off:off + n])
    ora = C.prove(mu, gate, m, canon, r)
    assert np.array_equal(got[0], ora["evals"]) and np.array_equal(got[1], ora["alphas"])
    assert np.array_equal(got[2], ora["openings"])
    ws2 = zc.new_workspace(s)
    copy = zc.prove(s, [p[:, off:off + n].contiguous() for p in pool], dev(r), ws2)
    assert all(np.array_equal(a, b.cpu().numpy()) for a, b in zip(got, copy))
    assert all(torch.equal(a, b) for a, b in zip(pool, before))


@pytest.mark.parametrize("mu,gate,m", [(20, 0, 0), (21, 1, 8), (17, 0, 0), (12, 2, 34)])
def test_shared_gpu_grids_give_the_same_bytes(zc, mu, gate, m):
    """ZC_FLAG_SHARED_GPU launches the thread-per-pair rounds with up to 2048
    short-lived blocks instead of one resident generation; the block sums
    are exact field additions, so every output byte is the same."""
    inst = I.make_instance(83, mu, mu, gate, m, workers=8)
    outs = []
    for flags in (0, zc.ZC_FLAG_SHARED_GPU):
        s = zc.shape(mu, gate, m, flags)
        ws = zc.new_workspace(s)
        tabs = [zc.pack(dev(t), ws) for t in inst.tables]
        outs.append([o.cpu().numpy() for o in zc.prove(s, tabs, dev(inst.r), ws)])
        assert zc.read_error(ws) == 0
    assert all(np.array_equal(a, b) for a, b in zip(*outs))


@pytest.mark.parametrize("mu,gate,m", [(3, 0, 0), (9, 1, 8), (12, 0, 0), (17, 0, 0), (20, 1, 8), (18, 1, 2),
                                       (10, 2, 34), (11, 2, 4), (6, 1, 5)])
def test_assume_satisfied_gives_the_same_bytes_on_satisfying_witnesses(zc, mu, gate, m):
    """ZC_FLAG_ASSUME_SATISFIED: round 1 evaluates X >= 2 only (thread per
    pair or 16 lanes per pair, every gate family, with and without the
    product gate's separate o sums); on a witness that satisfies the gate the
    proof is byte for byte the one without the flag, i.e. the oracle's."""
    inst = I.make_instance(84, mu, mu, gate, m, workers=8)
    outs = []
    for flags in (0, zc.ZC_FLAG_ASSUME_SATISFIED):
        s = zc.shape(mu, gate, m, flags)
        ws = zc.new_workspace(s)
        tabs = [zc.pack(dev(t), ws) for t in inst.tables]
        outs.append([o.cpu().numpy() for o in zc.prove(s, tabs, dev(inst.r), ws)])
        assert zc.read_error(ws) == 0
    assert all(np.array_equal(a, b) for a, b in zip(*outs))
    assert not outs[0][0][0, :2].any()  # G_1(0) = G_1(1) = 0 for a satisfying witness


def test_assume_satisfied_on_a_nonsatisfying_witness_zeroes_round_1(zc):
    """With the flag the caller's assertion is taken as given: on a witness
    that does not satisfy the gate, G_1(0) and G_1(1) come out 0 (the honest
    proof's do not) while G_1(2), G_1(3) are still evaluated."""
    inst = I.make_instance(85, 0, 10, 0, 0, satisfying=False)
    res = []
    for flags in (0, zc.ZC_FLAG_ASSUME_SATISFIED):
        s = zc.shape(10, 0, 0, flags)
        ws = zc.new_workspace(s)
        tabs = [zc.pack(dev(t), ws) for t in inst.tables]
        res.append([o.cpu().numpy() for o in zc.prove(s, tabs, dev(inst.r), ws)])
    honest, flagged = res
    assert honest[0][0, :2].any() and not flagged[0][0, :2].any()
    assert np.array_equal(honest[0][0, 2:4], flagged[0][0, 2:4])
