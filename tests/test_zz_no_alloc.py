"""zc_prove_static (the proof with the library's own per-device workspace,
for callers that cannot allocate) against zc_prove with a caller workspace,
through the C ABI: two calls in a row on the same array, the second with a
smaller shape of another gate, each byte-identical to zc_prove and to the C
oracle; then a call whose r is not canonical reports ZC_ERANGE through its
status word, and a clean call after it reports ZC_OK again."""
import numpy as np
import pytest
import torch

from oracle import c_oracle as C
from paper_2606_16146_amd import inputs as I
from tests._helpers import P, dev, gpu_prove, limbs_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zc():
    from paper_2606_16146_amd import zc as z
    z.lib()
    return z


def _static(zc, inst):
    s = zc.shape(inst.mu, inst.gate, inst.m)
    scratch = zc.new_workspace(zc.shape(4, 0))  # only zc_pack's error word
    tabs = [zc.pack(dev(t), scratch) for t in inst.tables]
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    out = zc.prove_static(s, tabs, dev(inst.r), status=status)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out], int(status.item())


@pytest.mark.parametrize("first,second", [((17, 0, 0), (12, 1, 8)), ((16, 1, 8), (9, 2, 34))])
def test_static_equals_prove_on_two_calls_second_smaller(zc, first, second):
    for mu, gate, m in (first, second):
        print(f"zc_prove_static mu={mu} gate={gate} m={m}", flush=True)
        inst = I.make_instance(88, mu, mu, gate, m)
        got, status = _static(zc, inst)
        assert status == zc.ZC_OK
        ref = gpu_prove(inst)
        assert ref["err"] == 0
        for a, b in zip(got, (ref["evals"], ref["alphas"], ref["openings"])):
            assert np.array_equal(a, b)
        ora = C.prove(mu, gate, m, inst.tables, inst.r)
        assert np.array_equal(got[0], ora["evals"]) and np.array_equal(got[1], ora["alphas"])
        assert np.array_equal(got[2], ora["openings"])


def test_static_reports_noncanonical_r_then_clears(zc):
    inst = I.make_instance(89, 0, 6, 0, 0)
    inst.r[2] = limbs_of([P])[0]
    _, status = _static(zc, inst)
    assert status == zc.ZC_ERANGE
    inst = I.make_instance(89, 1, 6, 0, 0)
    got, status = _static(zc, inst)
    assert status == zc.ZC_OK
    ref = gpu_prove(inst)
    assert np.array_equal(got[0], ref["evals"]) and np.array_equal(got[2], ref["openings"])
