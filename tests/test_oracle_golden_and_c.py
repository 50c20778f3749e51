"""Frozen oracle outputs, and the C oracle against the Python oracle (CPU)."""
import glob
import json
import os

import numpy as np
import pytest

from oracle import c_oracle as C
from oracle import zc_oracle as O
from paper_2606_16146_amd import inputs as I

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json")))


def _ints(a):
    return [int.from_bytes(np.ascontiguousarray(x).tobytes(), "little") for x in a]


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p) for p in GOLDEN])
def test_python_oracle_matches_frozen_golden(path):
    g = json.load(open(path))
    x = I.make_instance(g["seed"], g["inst"], g["mu"], g["gate"], g["m"])
    res = O.prove(g["mu"], g["gate"], g["m"], x.tables_int(), x.r_int())
    assert [[format(v, "064x") for v in e] for e in res["evals"]] == g["evals"]
    assert [format(v, "064x") for v in res["alphas"]] == g["alphas"]
    assert [format(v, "064x") for v in res["openings"]] == g["openings"]
    assert O.verify(g["mu"], g["gate"], g["m"], x.r_int(), res["evals"], res["alphas"],
                    res["openings"])


@pytest.mark.parametrize("mu,gate,m,sat", [(1, 0, 0, True), (4, 0, 0, True), (9, 0, 0, True),
                                           (7, 0, 0, False), (5, 1, 1, True), (6, 1, 2, True),
                                           (6, 1, 4, False), (5, 1, 8, True),
                                           (6, 2, 2, True), (5, 2, 18, True), (7, 2, 34, False),
                                           (4, 2, 50, True), (6, 2, 3, True), (5, 2, 4, True)])
def test_c_oracle_equals_python_oracle(mu, gate, m, sat):
    x = I.make_instance(40 + mu, 0, mu, gate, m, satisfying=sat)
    a = C.prove(mu, gate, m, x.tables, x.r)
    b = O.prove(mu, gate, m, x.tables_int(), x.r_int())
    assert [_ints(e) for e in a["evals"]] == b["evals"]
    assert _ints(a["alphas"]) == b["alphas"]
    assert _ints(a["openings"]) == b["openings"]


def test_c_oracle_thread_count_does_not_change_bytes():
    x = I.make_instance(77, 0, 10, 1, 4)
    a = C.prove(10, 1, 4, x.tables, x.r, nthreads=1)
    b = C.prove(10, 1, 4, x.tables, x.r, nthreads=3)
    for key in a:
        assert (a[key] == b[key]).all()


def test_c_oracle_rejects_noncanonical_input_and_bad_gate():
    x = I.make_instance(78, 0, 3, 0, 0)
    t = x.tables.copy()
    t[2, 5] = np.array([(O.P >> (32 * k)) & 0xFFFFFFFF for k in range(8)], np.uint32)  # = p
    with pytest.raises(ValueError):
        C.prove(3, 0, 0, t, x.r)
    with pytest.raises(ValueError):
        C.prove(3, 7, 0, x.tables, x.r)
