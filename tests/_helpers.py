"""Shared helpers of the tests: conversions between numpy limbs, Python
ints and device tensors, and running a proof through the C ABI."""
import numpy as np
import torch

P = 21888242871839275222246405745257275088548364400416034343698204186575808495617
R_MONT = 1 << 261  # the library's Montgomery radix (internal form of packed tables)


def ints_of(a) -> list:
    """uint32[..., 8] (numpy or tensor) -> flat list of Python ints."""
    if isinstance(a, torch.Tensor):
        a = a.cpu().numpy()
    a = np.ascontiguousarray(a, dtype=np.uint32).reshape(-1, 8)
    b = a.tobytes()
    return [int.from_bytes(b[i:i + 32], "little") for i in range(0, len(b), 32)]


def limbs_of(vals) -> np.ndarray:
    b = b"".join(int(v).to_bytes(32, "little") for v in vals)
    return np.frombuffer(b, dtype=np.uint32).reshape(-1, 8).copy()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32)).cuda()


def gpu_prove(inst, ws=None, stream=None):
    """Pack an inputs.Instance on the GPU and run zc_prove; returns numpy outputs."""
    from paper_2606_16146_amd import zc
    s = zc.shape(inst.mu, inst.gate, inst.m)
    if ws is None:
        ws = zc.new_workspace(s)
    tabs = [zc.pack(dev(t), ws) for t in inst.tables]
    r = dev(inst.r)
    ev, al, op = zc.prove(s, tabs, r, ws)
    err = zc.read_error(ws)
    return {"evals": ev.cpu().numpy(), "alphas": al.cpu().numpy(), "openings": op.cpu().numpy(),
            "err": err, "tables": tabs, "ws": ws, "shape": s, "r": r}


def same_as_oracle(res, ora):
    """Compare GPU numpy outputs with a Python-oracle result dict (ints)."""
    mu = len(ora["evals"])
    ev = [ints_of(res["evals"][i]) for i in range(mu)]
    assert ev == ora["evals"], "round polynomials differ"
    assert ints_of(res["alphas"]) == ora["alphas"], "challenges differ"
    assert ints_of(res["openings"]) == ora["openings"], "openings differ"
