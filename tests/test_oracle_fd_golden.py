"""The stored FP64 oracle finite differences of the 256 x 256 gradient
workload (tests/golden/cfg4_oracle_fd.json, written by make_cfg4_fd.py with
the oracle only): what they say about the workload itself.

With n = 0.7 and the [0.1, 10] nu0 viscosity clamp, the oracle's central
differences of Nu_bar in n do not converge as the step shrinks (h = 1e-2,
1e-3, 1e-4 relative), while those in Ra do: Nu_bar after 5000 steps has a
sensitivity floor in the viscosity law that no pointwise derivative
describes (the exact adjoint of that trajectory grows without bound, and the
library reports it).  The tangent-linear model of the same trajectory
(cfg4_tangent_growth.json, make_cfg4_tangent.py) grows a unit perturbation
by orders of magnitude within 100 steps; with a [0.1, 2] clamp it does not.
"""
import json
import os

import pytest

from paper_2011_15073_amd import inputs

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(HERE, name)) as fh:
        return json.load(fh)


def fd(entries, h):
    return next(e["fd"] for e in entries if e["h"] == h)


def test_stored_differences_use_the_seeded_cells():
    gold = load("cfg4_oracle_fd.json")
    cells = [int(c) for c in inputs.fd_cells(256, seed=1, k=16)]
    for v in gold["variants"].values():
        assert v["cells"] == cells and len(v["cell_fd"]) == 16
        assert v["params"]["N"] == 256 and v["params"]["T"] == 5000
        for e in v["cell_fd"]:
            assert e["fd"] == pytest.approx((e["J_plus"] - e["J_minus"]) / (2 * e["h"]), rel=1e-12)


def test_n07_differences_in_n_do_not_converge_but_in_ra_do():
    v = load("cfg4_oracle_fd.json")["variants"]["n0.7"]
    dn = [fd(v["n_fd"], h) for h in (1e-2, 1e-3, 1e-4)]
    dR = [fd(v["Ra_fd"], h) for h in (1e-2, 1e-3, 1e-4)]
    print("dNu/dn", dn, "dNu/dRa", dR)
    assert abs(dn[2] - dn[0]) > 0.3 * abs(dn[0])
    assert max(dR) - min(dR) < 0.03 * abs(dR[0])


def test_tangent_linear_growth_separates_the_clamps():
    runs = load("cfg4_tangent_growth.json")["runs"]
    grow10 = max(r["max_norm"] for r in runs["clamp_0.1_10"])
    grow2 = max(r["max_norm"] for r in runs["clamp_0.1_2"])
    print("max-norm growth over 100 steps: [0.1, 10]", grow10, "[0.1, 2]", grow2)
    assert grow10 > 100.0 and grow2 < 10.0
