"""Writes the frozen oracle outputs under tests/golden/ (calls only oracle/).

Each fixture records a small seeded instance (generator recipe: seed, inst,
mu, gate, m) and the oracle's round polynomials, challenges and openings as
hex strings.  The paper prints no worked numeric example for the multilinear
ZeroCheck (Fig. 2, right); these fixtures freeze the oracle, whose pins are
in tests/test_oracle_pins.py, so that any later change to its arithmetic is
visible.  Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import zc_oracle as O  # noqa: E402
from paper_2606_16146_amd import inputs as I  # noqa: E402

CASES = [
    # (name, seed, inst, mu, gate, m)
    ("vanilla_mu4", 11, 0, 4, O.GATE_VANILLA, 0),
    ("vanilla_mu8", 12, 0, 8, O.GATE_VANILLA, 0),
    ("prod2_mu5", 13, 0, 5, O.GATE_PROD, 2),
    ("prod4_mu6", 14, 0, 6, O.GATE_PROD, 4),
    ("prod8_mu4", 15, 0, 4, O.GATE_PROD, 8),
]


def hx(v):
    return format(v, "064x")


def main():
    for name, seed, inst, mu, gate, m in CASES:
        x = I.make_instance(seed, inst, mu, gate, m)
        res = O.prove(mu, gate, m, x.tables_int(), x.r_int())
        doc = {
            "source": "multilinear ZeroCheck via SumCheck, Fig. 2 (right) and Sec. 3.3 Eq. (1); "
                      "written by tests/golden/make_golden.py from oracle/zc_oracle.py",
            "seed": seed, "inst": inst, "mu": mu, "gate": gate, "m": m,
            "evals": [[hx(v) for v in g] for g in res["evals"]],
            "alphas": [hx(v) for v in res["alphas"]],
            "openings": [hx(v) for v in res["openings"]],
            "transcript": res["transcript"].hex(),
        }
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(doc, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
