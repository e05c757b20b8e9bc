"""GPU: 16-bit population storage (PM_FP16: IEEE half shifted populations,
FP32 arithmetic, stochastically rounded stores) against the FP64 oracle.

Bars, from the measured loss of half-precision storage (a half ulp is 2^-11
relative, against 2^-24 for FP32):
  * one step from a random non-equilibrium state: every stored population
    within two half ulps (2^-9 relative) of the oracle's step from the same
    half-rounded state -- the stochastic conversion moves a value by less
    than one half spacing;
  * 64^2 cavities after 20 000 steps from rest: the error is rounding noise,
    so it is measured over realizations of it -- the rest state and seven
    rest states perturbed by 1e-6 relative (far below the error; every
    random word of the rounding changes).  Over 24 realizations the fields
    were within 9.5e-4 (median) / 1.3e-3 (max) for the Newtonian cavity and
    8.2e-3 / 9.9e-3 for the power law at Ra = 1e5, Nu within 1.5e-3 / 3.4e-3
    and 2.1e-3 / 4.0e-3; the bars are 1.5 times those, on the median and on
    the largest of the eight.  Nu is limited by noise: Eq. (24) weighs the
    two wall columns' theta by N (8 - 9 theta_0 + theta_1) / 3, so the
    rounding noise of the stored thermal populations reaches Nu amplified
    about twenty times at Nu ~ 1.  Round-to-nearest half storage is 40 to
    100 times worse (it accumulates its fixed rounding pattern in the slow
    modes).
"""
import numpy as np
import pytest
import torch

import paper_2011_15073_amd as P
from paper_2011_15073_amd import inputs
from pairs import compare_fields, compare_nu, gpu_for, oracle_for

pytestmark = pytest.mark.gpu

W9 = inputs.W9
W5 = inputs.W5


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("kw", [dict(n=0.7, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6),
                                dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6)], ids=["n0.7", "n1.0"])
@pytest.mark.parametrize("pre", [0, 1])
def test_fp16_step_within_two_half_ulps(kw, pre):
    nx, ny = 70, 19
    f0, g0 = inputs.random_state(nx, ny, seed=13, amp=0.03, amp_T=0.2)
    cav = gpu_for(nx, ny, dtype="fp16", **kw)
    cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    cav.step(pre)
    fh, gh = (t.cpu().numpy() for t in cav.populations(torch.float64))  # the stored (half) state
    orc = oracle_for(nx, ny, **kw)
    orc.set_state(fh, gh)
    orc.step(1)
    fr, gr = orc.state()
    cav.step(1)
    fg, gg = (t.cpu().numpy() for t in cav.populations(torch.float64))
    worst = 0.0
    for got, ref, inp, w in ((fg, fr, fh, W9), (gg, gr, gh, W5 * 0.5)):
        for q in range(got.shape[0]):
            d_ref, d_in = ref[q] - w[q], inp[q] - w[q]   # the shifted values the kernels store
            scale = max(2.0 ** -14, np.abs(d_ref).max(), np.abs(d_in).max())
            err = np.abs(got[q] - ref[q]).max()
            worst = max(worst, err / (2.0 ** -9 * scale))
            assert err <= 2.0 ** -9 * scale, (q, err, scale)
    log(f"fp16 one step {kw} pre={pre}: worst error {worst:.3f} of the two-half-ulp bound")


def _bracket(exact):
    """The two halves (as float64 arrays) that bracket each value of exact."""
    h = exact.astype(np.float16)
    above = h.astype(np.float64) > exact
    down = np.nextafter(h, np.float16(-np.inf)).astype(np.float64)
    up = np.nextafter(h, np.float16(np.inf)).astype(np.float64)
    hv = h.astype(np.float64)
    return np.where(above, down, hv), np.where(above, hv, up)


@pytest.mark.parametrize("pre", [0, 1])
def test_fp16_stochastic_rounding_is_unbiased(pre):
    """A uniform state on a doubly periodic 64 x 64 grid (after one more step
    for the odd parity): every node computes its update in FP32 and stores,
    chosen by its own random word, one of the two halves that bracket it.
    Over the 4096 nodes the mean rounding error of every population is
    within 0.05 of a half spacing (its standard deviation is at most 0.008
    spacing).  Checked for the populations whose shifted value is at least
    a tenth of the largest one's: there the FP32 arithmetic before the
    rounding is within a few thousandths of a half spacing of the oracle's
    FP64 value (smaller ones, down to subnormal halves, are only reported).
    Round-to-nearest storage is off by its fixed rounding error instead."""
    N = 64
    kw = dict(n=0.7, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6, periodic_x=1, periodic_y=1)
    f0, g0 = inputs.uniform_state(N, N, seed=21)
    worst, checked = {}, []
    for rounding in ("auto", "nearest"):
        cav = gpu_for(N, N, dtype="fp16", rounding=rounding, **kw)
        cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
        cav.step(pre)
        fh, gh = (t.cpu().numpy() for t in cav.populations(torch.float64))
        orc = oracle_for(N, N, **kw)
        orc.set_state(fh, gh)
        orc.step(1)
        fr, gr = orc.state()
        cav.step(1)
        fg, gg = (t.cpu().numpy() for t in cav.populations(torch.float64))
        biases, checked = [], []
        # the library shifts by the FP32 weights; with them, got - w is the
        # stored half exactly and ref - w the update it was rounded from
        for got, ref, w in ((fg, fr, W9.astype(np.float32).astype(np.float64)),
                            (gg, gr, W5.astype(np.float32).astype(np.float64) * 0.5)):
            big = max(abs(ref[q].mean() - w[q]) for q in range(got.shape[0]))
            for q in range(got.shape[0]):
                exact = ref[q] - w[q]                 # the shifted values the kernels store
                lo, hi = _bracket(exact)
                sp = hi - lo
                stored = got[q] - w[q]
                biases.append(float(((stored - exact) / sp).mean()))
                if abs(exact.mean()) >= 0.1 * big:
                    near = np.minimum(np.abs(stored - lo), np.abs(stored - hi)) / sp
                    assert near.max() <= 0.02, (rounding, q, near.max())   # one of the two bracketing halves
                    checked.append(abs(biases[-1]))
        worst[rounding] = max(checked)
        log(f"fp16 uniform state, {rounding}, pre={pre}: mean rounding error in half spacings "
            f"{np.round(biases, 3).tolist()}")
    assert len(checked) >= 10
    assert worst["auto"] <= 0.05
    assert worst["nearest"] > 0.1


CFG0 = dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6)
PLAW = dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)


# (median, max) bars for the fields and for Nu, per cavity
BARS = {"newtonian": ((1.5e-3, 2.0e-3), (2.3e-3, 5.0e-3)),
        "power-law": ((1.25e-2, 1.5e-2), (3.2e-3, 6.0e-3))}


@pytest.mark.parametrize("name,kw", [("newtonian", CFG0), ("power-law", PLAW)], ids=["newtonian", "power-law"])
def test_fp16_cavity_64_20000_steps(name, kw):
    orc = oracle_for(64, **kw).step(20000)
    fields, nus = [], []
    for s in range(8):
        cav = gpu_for(64, dtype="fp16", **kw)
        if s:
            f0, g0 = inputs.random_state(64, 64, seed=1000 + s, amp=1e-6, T0=0.5, amp_T=1e-6)
            cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
        cav.step(20000)
        fields.append(max(compare_fields(cav, orc).values()))
        nus.append(compare_nu(cav, orc))
    near = gpu_for(64, dtype="fp16", rounding="nearest", **kw)
    near.step(20000)
    fn = max(compare_fields(near, orc).values())
    (fmed, fmax), (nmed, nmax) = BARS[name]
    log(f"fp16 64^2 {name}: fields median {np.median(fields):.2e} max {max(fields):.2e}, Nu median "
        f"{np.median(nus):.2e} max {max(nus):.2e} over 8 realizations; round-to-nearest fields {fn:.2e}, "
        f"Nu {compare_nu(near, orc):.2e}")
    assert np.median(fields) <= fmed and max(fields) <= fmax
    assert np.median(nus) <= nmed and max(nus) <= nmax
    assert fn > 3 * np.median(fields)


def test_fp16_state_round_trip_and_checkpoint():
    kw = dict(PLAW)
    a = gpu_for(48, 40, dtype="fp16", **kw)
    a.step(301)
    snap = a.save_state()
    f1, g1 = a.populations(torch.float32)
    a.step(200)
    b = gpu_for(48, 40, dtype="fp16", **kw)
    b.load_state(snap)
    fb, gb = b.populations(torch.float32)
    assert torch.equal(f1, fb) and torch.equal(g1, gb)
    b.step(200)
    fa, ga = a.populations(torch.float32)
    fb, gb = b.populations(torch.float32)
    assert torch.equal(fa, fb) and torch.equal(ga, gb) and a.nu() == b.nu()
    # an FP32 context of the same grid refuses the FP16 state (another dtype)
    c = gpu_for(48, 40, dtype="fp32", **kw)
    with pytest.raises(P.PmError):
        c.load_state(snap)
    # get -> set returns the same stored (half) populations, read back exactly in FP64
    # (at an even step count: after an odd one the populations that crossed a
    # thermal wall carry the anti-bounce-back constant, which is not a half)
    a.step(1)
    fa64, ga64 = a.populations(torch.float64)
    c16 = gpu_for(48, 40, dtype="fp16", **kw)
    c16.set_populations(fa64, ga64)
    fc, gc = c16.populations(torch.float64)
    assert torch.equal(fa64, fc) and torch.equal(ga64, gc)


def test_fp16_is_refused_where_unsupported():
    with pytest.raises(P.PmError, match="FP16"):
        P.Sweep([dict(nx=32, dtype="fp16", **CFG0)])
    cav = gpu_for(32, dtype="fp16", logda=torch.from_numpy(inputs.logda_field(32, seed=1)), **CFG0)
    with pytest.raises(P.PmError, match="FP16"):
        P.Adjoint(cav, 10)
    with pytest.raises(P.PmError, match="single|FP32"):
        gpu_for(4096, dtype="fp16", step_kernel="pair", **CFG0)
