"""Batched proofs (zc_batch_*) through the C ABI: every instance of a batch
must be byte-identical to its single-instance zc_prove and to the C oracle
(the oracle is pinned against the paper in test_oracle_pins.py), whatever
the mix of sizes, gates and launch tiles, and also when the launch
sequence is captured into a HIP graph and replayed."""
import numpy as np
import pytest
import torch

from oracle import c_oracle as C
from paper_2606_16146_amd import inputs as I
from paper_2606_16146_amd import zc
from tests._helpers import P, dev, gpu_prove

pytestmark = pytest.mark.gpu

# (mu, gate, m, tile): sizes from one round to several round-kernel rounds,
# every tail entry point, all gate groups of a mixed batch
MIX = [
    (1, 0, 0, 0), (3, 1, 2, 1), (5, 0, 0, 2), (6, 1, 8, 0), (7, 0, 0, 1), (7, 1, 4, 4),
    (8, 1, 1, 8), (9, 0, 0, 0), (10, 1, 8, 2), (11, 1, 5, 0), (12, 0, 0, 16), (13, 1, 4, 1),
    (9, 2, 2, 0), (6, 2, 50, 2), (11, 2, 4, 1), (8, 2, 18, 4),  # Table 1 shapes
]


def _setup(specs, seed=21):
    items, insts = [], []
    for i, (mu, gate, m, tile) in enumerate(specs):
        inst = I.make_instance(seed, i, mu, gate, m)
        s = zc.shape(mu, gate, m)
        ws = zc.new_workspace(s)
        tabs = [zc.pack(dev(t), ws) for t in inst.tables]
        items.append((s, tabs, dev(inst.r), ws, zc.new_outputs(s), tile))
        insts.append(inst)
    torch.cuda.synchronize()
    return items, insts


def _outputs(item):
    return [o.cpu().numpy().copy() for o in item[4]]


def test_batch_matches_single_prove_and_c_oracle():
    items, insts = _setup(MIX)
    b = zc.Batch(items)
    b.prove()
    torch.cuda.synchronize()
    for it, inst in zip(items, insts):
        print(f"instance mu={inst.mu} gate={inst.gate} m={inst.m}", flush=True)
        assert zc.read_error(it[3]) == 0
        ev, al, op = _outputs(it)
        single = gpu_prove(inst)
        assert single["err"] == 0
        assert np.array_equal(ev, single["evals"]) and np.array_equal(al, single["alphas"])
        assert np.array_equal(op, single["openings"])
        ora = C.prove(inst.mu, inst.gate, inst.m, inst.tables, inst.r)
        assert np.array_equal(ev, ora["evals"]) and np.array_equal(al, ora["alphas"])
        assert np.array_equal(op, ora["openings"])


def test_batch_repeat_is_identical_and_inputs_untouched():
    items, insts = _setup(MIX[:6], seed=22)
    before = [[t.clone() for t in it[1]] for it in items]
    b = zc.Batch(items)
    b.prove()
    first = [_outputs(it) for it in items]
    for it in items:
        for o in it[4]:
            o.zero_()
    b.launch()  # descriptors already uploaded
    torch.cuda.synchronize()
    for it, f, tb in zip(items, first, before):
        assert all(np.array_equal(x, y) for x, y in zip(_outputs(it), f))
        assert all(torch.equal(t0, t1) for t0, t1 in zip(tb, it[1]))


def test_batch_graph_replays_match_eager():
    items, _ = _setup(MIX[2:10], seed=23)
    b = zc.Batch(items)
    b.prove()
    torch.cuda.synchronize()
    eager = [_outputs(it) for it in items]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            b.launch(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:  # the program's own eager work between replays
            for o in it[4]:
                o.fill_(rep + 1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, e in zip(items, eager):
            assert zc.read_error(it[3]) == 0
            assert all(np.array_equal(x, y) for x, y in zip(_outputs(it), e)), f"replay {rep}"


def test_batch_error_stays_in_its_instance():
    items, insts = _setup(MIX[:4], seed=24)
    bad = 2
    r_bad = items[bad][2]
    r_bad[0] = torch.from_numpy(np.frombuffer(P.to_bytes(32, "little"), dtype=np.uint32).copy()).cuda()
    b = zc.Batch(items)
    b.prove()
    torch.cuda.synchronize()
    for i, (it, inst) in enumerate(zip(items, insts)):
        err = zc.read_error(it[3])
        if i == bad:
            assert err == zc.ZC_ERANGE
            continue
        assert err == 0
        ora = C.prove(inst.mu, inst.gate, inst.m, inst.tables, inst.r)
        ev, al, op = _outputs(it)
        assert np.array_equal(ev, ora["evals"]) and np.array_equal(op, ora["openings"])
