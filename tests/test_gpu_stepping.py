"""The stepping form of the proof (zc_round / zc_fold, Fig. 2 right taken one
round at a time) at full shape: mu = 17 and 20, where zc_round runs its
thread-per-pair kernel for the rounds with more than 16384 pairs and its
lane-split kernel after them, and zc_fold folds tables of up to 2^19
entries.  Round polynomials, challenges and the folded openings are compared
with the C oracle; a proof stopped after round t, whose tables and workspace
are copied, resumes on the copies to the same bytes."""
import numpy as np
import pytest
import torch

from oracle import c_oracle as C
from paper_2606_16146_amd import inputs as I
from tests._helpers import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zc():
    from paper_2606_16146_amd import zc as z
    z.lib()
    return z


def _packed(zc, inst):
    s = zc.shape(inst.mu, inst.gate, inst.m)
    ws = zc.new_workspace(s)
    return s, ws, [zc.pack(dev(t), ws) for t in inst.tables]


def _step(zc, s, tabs, r, ws, ev, al, rounds):
    for i in rounds:
        zc.round_(s, tabs, r, ws, i, ev, al)
        zc.fold(s, tabs, ws, i)


@pytest.mark.parametrize("mu,gate,m", [(17, 0, 0), (17, 1, 8), (20, 0, 0)])
def test_stepping_full_shape_matches_c_oracle(zc, mu, gate, m):
    inst = I.make_instance(950 + mu, gate, mu, gate, m, workers=8)
    s, ws, tabs = _packed(zc, inst)
    r = dev(inst.r)
    ev, al, _ = zc.new_outputs(s)
    print(f"stepping mu={mu} gate={gate} m={m}", flush=True)
    _step(zc, s, tabs, r, ws, ev, al, range(1, mu + 1))
    assert zc.read_error(ws) == 0
    ora = C.prove(mu, gate, m, inst.tables, inst.r)
    assert np.array_equal(ev.cpu().numpy(), ora["evals"])
    assert np.array_equal(al.cpu().numpy(), ora["alphas"])
    openings = np.stack([zc.unpack(t, 1).cpu().numpy()[0] for t in tabs])
    assert np.array_equal(openings, ora["openings"][:-1])


@pytest.mark.parametrize("mu,gate,m,t", [(17, 0, 0, 3), (17, 1, 8, 9), (12, 1, 4, 11)])
def test_stop_copy_state_resume_gives_same_bytes(zc, mu, gate, m, t):
    inst = I.make_instance(960 + mu, t, mu, gate, m)
    r = dev(inst.r)
    # uninterrupted
    s, ws, tabs = _packed(zc, inst)
    ev, al, _ = zc.new_outputs(s)
    _step(zc, s, tabs, r, ws, ev, al, range(1, mu + 1))
    # stopped after round t: the state is the folded tables plus the workspace
    s2, ws2, tabs2 = _packed(zc, inst)
    ev2, al2, _ = zc.new_outputs(s2)
    _step(zc, s2, tabs2, r, ws2, ev2, al2, range(1, t + 1))
    torch.cuda.synchronize()
    ws3, tabs3 = ws2.clone(), [x.clone() for x in tabs2]
    ws2.zero_()
    for x in tabs2:
        x.zero_()
    ev3, al3 = ev2.clone(), al2.clone()
    _step(zc, s2, tabs3, r, ws3, ev3, al3, range(t + 1, mu + 1))
    assert zc.read_error(ws3) == 0
    assert torch.equal(ev3, ev) and torch.equal(al3, al)
    for a, b in zip(tabs3, tabs):
        assert torch.equal(zc.unpack(a, 1), zc.unpack(b, 1))
