"""The optional device self-checks (ZC_FLAG_CHECK_CLAIMS): every round checks
G_i(0) + G_i(1) against the previous claim G_{i-1}(alpha_{i-1}) (0 before
round 1, Sec. 3.4), and the last step checks G_mu(alpha_mu) against
f_M(openings) eq_r(alpha).  Honest proofs of satisfying witnesses pass with
the same bytes as without the flag; a witness that does not satisfy the gate
fails the first check; a table altered between two stepping rounds fails the
next round's check.  Failures come back as ZC_ECLAIM through zc_read_error."""
import numpy as np
import pytest
import torch

from paper_2606_16146_amd import inputs as I
from tests._helpers import dev, limbs_of, P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zc():
    from paper_2606_16146_amd import zc as z
    z.lib()
    return z


def _prove(zc, inst, flags):
    s = zc.shape(inst.mu, inst.gate, inst.m, flags)
    ws = zc.new_workspace(s)
    tabs = [zc.pack(dev(t), ws) for t in inst.tables]
    out = zc.prove(s, tabs, dev(inst.r), ws)
    err = zc.read_error(ws)
    return [o.cpu().numpy() for o in out], err


# thread-per-pair, lane-split, speculative (degree <= 3, mu >= 17) and tail
# rounds, every gate family
SHAPES = [(1, 0, 0), (7, 0, 0), (12, 1, 8), (9, 1, 4), (17, 0, 0), (10, 2, 34), (8, 2, 4), (17, 2, 3)]


@pytest.mark.parametrize("mu,gate,m", SHAPES)
def test_checks_pass_on_honest_proofs_with_same_bytes(zc, mu, gate, m):
    inst = I.make_instance(71, mu, mu, gate, m, workers=8)
    plain, err0 = _prove(zc, inst, 0)
    checked, err1 = _prove(zc, inst, zc.ZC_FLAG_CHECK_CLAIMS)
    assert err0 == 0 and err1 == 0
    assert all(np.array_equal(a, b) for a, b in zip(plain, checked))


@pytest.mark.parametrize("mu,gate,m", [(6, 0, 0), (12, 1, 8), (17, 0, 0)])
def test_nonsatisfying_witness_fails_the_first_check(zc, mu, gate, m):
    inst = I.make_instance(72, mu, mu, gate, m, satisfying=False)
    plain, err0 = _prove(zc, inst, 0)
    checked, err1 = _prove(zc, inst, zc.ZC_FLAG_CHECK_CLAIMS)
    assert err0 == 0 and err1 == zc.ZC_ECLAIM
    assert all(np.array_equal(a, b) for a, b in zip(plain, checked))


@pytest.mark.parametrize("mu,gate,m,t", [(9, 0, 0, 4), (8, 1, 8, 2)])
def test_table_altered_between_rounds_fails_the_next_check(zc, mu, gate, m, t):
    inst = I.make_instance(73, mu, mu, gate, m)
    s = zc.shape(mu, gate, m, zc.ZC_FLAG_CHECK_CLAIMS)
    ws = zc.new_workspace(s)
    tabs = [zc.pack(dev(x), ws) for x in inst.tables]
    r = dev(inst.r)
    ev, al, _ = zc.new_outputs(s)
    for i in range(1, t + 1):
        zc.round_(s, tabs, r, ws, i, ev, al)
        zc.fold(s, tabs, ws, i)
    assert zc.read_error(ws) == 0
    # replace entry 0 of table 1 (still a valid element, < p)
    other = zc.pack(dev(limbs_of([12345 % P])), ws)
    tabs[1][:, 0] = other[:, 0]
    zc.round_(s, tabs, r, ws, t + 1, ev, al)
    assert zc.read_error(ws) == zc.ZC_ECLAIM


def test_flag_travels_through_a_batch(zc):
    specs = [(9, 0, 0, True), (11, 1, 8, False), (7, 1, 4, True)]
    items, want = [], []
    for i, (mu, gate, m, sat) in enumerate(specs):
        inst = I.make_instance(74, i, mu, gate, m, satisfying=sat)
        s = zc.shape(mu, gate, m, zc.ZC_FLAG_CHECK_CLAIMS)
        ws = zc.new_workspace(s)
        tabs = [zc.pack(dev(x), ws) for x in inst.tables]
        items.append((s, tabs, dev(inst.r), ws, zc.new_outputs(s), 0))
        want.append(0 if sat else zc.ZC_ECLAIM)
    torch.cuda.synchronize()
    b = zc.Batch(items)
    b.prove()
    assert [zc.read_error(it[3]) for it in items] == want
