"""GPU: the paper's own runs (its validation table and its parametric table,
160 x 160) on the built solver, as one batched FP64 sweep to steady state,
against the Nusselt numbers the paper prints (tests/golden/paper_nu_tables.json).

Reading of the paper's runs: its equations as printed (eps = 1, the Darcy
term only; the validation runs a clear fluid), its modified power law with
the shear-rate thresholds gamma1 = 0.01, gamma2 = 1e6 (Eq. 21), 160 x 160
(the parametric table's grid; the validation grid is not given), lattice
Mach number 0.05 (not given; at 0.1 the two low-Ra shear-thinning cases do
not settle below 1e-8 per 1000 steps).

Bounds, from that reading:
  * every trend the paper reports holds: Nu falls with n, rises with Da and
    with Ra;
  * where the power law is not shear-thinning at high Ra -- n = 1 and 1.4,
    and n = 0.6 at Ra = 1e3 and 1e4 -- within 3%: the paper's two benchmark
    sources differ by 0.7% on the clear-fluid n = 1 case, and halving the
    Mach number or doubling the grid moves these values by up to 1.5%;
  * the shear-thinning cases at Ra = 1e5 are not reproduced: the paper's
    Da = 1e-2 and 1e-1 values are 12-14% above ours and its clear-fluid one
    11% below, and neither clamp, nor the Mach number, nor the grid (160 or
    320) moves ours by more than 4%.  Only their trends are checked.
"""
import json
import os

import pytest

import paper_2011_15073_amd as P

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
N = 160
READING = dict(eps=1.0, forchheimer=0, clamp_mode=1, nu_lo=0.01, nu_hi=1e6, mach=0.05, dtype="fp64")


@pytest.fixture(scope="module")
def runs():
    tab = json.load(open(os.path.join(HERE, "golden", "paper_nu_tables.json")))
    rows = [("validation", r) for r in tab["validation"]] + [("parametric", r) for r in tab["parametric"]]
    cases = []
    for table, r in rows:
        kw = dict(nx=N, n=r["n"], Ra=r["Ra"], Pr=r["Pr"], **READING)
        if table == "parametric":
            kw["Da"] = r["Da"]
        cases.append(kw)
    sw = P.Sweep(cases)
    steps, res = sw.run(tol=1e-8, check_every=1000, max_steps=2_000_000)
    out = []
    for i, (table, r) in enumerate(rows):
        nu = sw.case(i).nu()
        print(f"{table} {r}: Nu {nu:.6f} ({nu / r['nu'] - 1:+.4f}), {steps[i]} steps, r {res[i]:.1e}",
              flush=True)
        out.append((table, r, nu, steps[i], res[i]))
    return out


def pick(runs, table, **kw):
    for t, r, nu, _, _ in runs:
        if t == table and all(r.get(k) == v for k, v in kw.items()):
            return r["nu"], nu
    raise KeyError((table, kw))


def test_every_case_reaches_steady_state(runs):
    for t, r, nu, steps, res in runs:
        assert res < 1e-8 and steps < 2_000_000, (t, r, steps, res)


def test_trends_match_the_paper(runs):
    val = [pick(runs, "validation", n=n)[1] for n in (0.6, 1.0, 1.4)]
    assert val[0] > val[1] > val[2]
    case1 = [pick(runs, "parametric", n=n, Da=1e-3, Ra=1e5)[1] for n in (0.6, 1.0, 1.4)]
    assert case1[0] > case1[1] > case1[2]
    case2 = [pick(runs, "parametric", n=0.6, Da=da, Ra=1e5)[1] for da in (1e-3, 1e-2, 1e-1)]
    assert case2[0] < case2[1] < case2[2]
    case3 = [pick(runs, "parametric", n=0.6, Da=1e-2, Ra=ra)[1] for ra in (1e3, 1e4, 1e5)]
    assert case3[0] < case3[1] < case3[2]


def test_values_where_the_power_law_is_not_shear_thinning_at_high_ra(runs):
    checked = 0
    for t, r, nu, _, _ in runs:
        if r["n"] >= 1.0 or r["Ra"] <= 1e4:
            assert nu == pytest.approx(r["nu"], rel=3e-2), (t, r, nu)
            checked += 1
    assert checked == 6
