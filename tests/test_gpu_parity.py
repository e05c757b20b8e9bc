"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars (field error = max|X_gpu - X_ref| / max|X_ref| for X in U, V, theta;
Nusselt number |dNu|/Nu):
  * FP64 kernels: <= 1e-11;
  * FP32 storage and arithmetic (FP64 reductions): <= 1e-4;
  * single steps from random non-equilibrium states, FP64: populations agree
    to 1e-13 absolute (every branch of the collision, walls and viscosity).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_2011_15073_amd as P
from paper_2011_15073_amd import inputs
from pairs import compare_fields, compare_nu, gpu_for, gpu_fields, oracle_for, rel_err

pytestmark = pytest.mark.gpu

CFG0 = dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6)
TOL = {"fp64": 1e-11, "fp32": 1e-4}


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_cavity_64_newtonian_20000_steps(dtype):
    """The 64x64 porous cavity, Newtonian, Da = 0.1, Ra = 1e3, Pr = 10,
    eps = 0.6, 20000 steps from rest."""
    log("case: 64^2", dtype, CFG0)
    cav = gpu_for(64, dtype=dtype, **CFG0)
    cav.step(20000)
    orc = oracle_for(64, **CFG0).step(20000)
    errs = compare_fields(cav, orc)
    dnu = compare_nu(cav, orc)
    log(dtype, errs, dnu, cav.nu())
    assert max(errs.values()) <= TOL[dtype] and dnu <= TOL[dtype]


def test_cavity_64_fp32_stochastic_rounding():
    """The 64x64 cavity of the first test in FP32 with stochastically rounded
    updates: within the FP32 bar of the oracle after 20000 steps, and
    deterministic (two runs bitwise equal)."""
    runs = []
    for _ in range(2):
        cav = gpu_for(64, dtype="fp32", rounding="stochastic", **CFG0)
        cav.step(20000)
        runs.append(cav)
    orc = oracle_for(64, **CFG0).step(20000)
    errs = compare_fields(runs[0], orc)
    dnu = compare_nu(runs[0], orc)
    log("fp32 stochastic", errs, dnu)
    assert max(errs.values()) <= 1e-4 and dnu <= 1e-4
    fa, ga = runs[0].populations(torch.float32)
    fb, gb = runs[1].populations(torch.float32)
    assert torch.equal(fa, fb) and torch.equal(ga, gb)


RANDOM_CASES = [
    dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6),
    dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6),
    dict(n=1.4, Da=math.inf, Ra=1e5, Pr=100.0, eps=1.0, forchheimer=0),
    dict(n=0.7, Da=1e-2, Ra=1e4, Pr=6.2, eps=0.6, clamp_mode=1, nu_lo=0.01, nu_hi=1e6),
    dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6, periodic_x=1),
    dict(n=0.5, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.5, periodic_y=1, gx=1e-5, gy=-2e-5),
    dict(n=1.2, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.7, periodic_x=1, periodic_y=1),
]


@pytest.mark.parametrize("ci", range(len(RANDOM_CASES)))
@pytest.mark.parametrize("logda", [False, True])
@pytest.mark.parametrize("grid", [(37, 21), (200, 23)])
def test_random_state_steps_fp64(ci, logda, grid):
    """Random non-equilibrium states on ragged grids: populations after 1, 2
    and 5 steps (both AA parities, every wall and corner; on the 200-wide grid
    the interior waves take the branch-free path of the streaming step)."""
    kw = RANDOM_CASES[ci]
    nx, ny = grid
    f0, g0 = inputs.random_state(nx, ny, seed=100 + ci, amp=0.05)
    ld = inputs.logda_field(max(nx, ny), seed=ci)[:ny, :nx].copy() if logda else None
    log("case:", ci, kw, "logda" if logda else "")
    cav = gpu_for(nx, ny, dtype="fp64", logda=ld, **kw)
    cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    orc = oracle_for(nx, ny, logda=ld, **kw)
    orc.set_state(f0, g0)
    for k in (1, 1, 3):
        cav.step(k)
        orc.step(k)
        fg, gg = (t.cpu().numpy() for t in cav.populations(torch.float64))
        fr, gr = orc.state()
        ef, eg = np.abs(fg - fr).max(), np.abs(gg - gr).max()
        log("  after", orc.steps, "steps: pop err", ef, eg)
        assert ef <= 1e-13 and eg <= 1e-13
    nu_g = cav.viscosity(torch.float64).cpu().numpy()
    assert rel_err(nu_g, orc.macros()["nu"]) <= 1e-12


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_random_state_mid_size(dtype):
    """A 600 x 500 grid from a random non-equilibrium state: above 512^2 the
    single-step kernels run 128-node (FP64) and 256-node (FP32) row segments
    per workgroup.  FP64 populations to 1e-13 after 1, 2 and 5 steps; FP32
    fields to the 1e-4 bar."""
    kw = RANDOM_CASES[1]
    nx, ny = 600, 500
    f0, g0 = inputs.random_state(nx, ny, seed=21, amp=0.05)
    log("case: 600x500 random state", dtype, kw)
    cav = gpu_for(nx, ny, dtype=dtype, **kw)
    cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    orc = oracle_for(nx, ny, **kw)
    orc.set_state(f0, g0)
    for k in (1, 1, 3):
        cav.step(k)
        orc.step(k)
        if dtype == "fp64":
            fg, gg = (t.cpu().numpy() for t in cav.populations(torch.float64))
            fr, gr = orc.state()
            ef, eg = np.abs(fg - fr).max(), np.abs(gg - gr).max()
            log("  after", orc.steps, "steps: pop err", ef, eg)
            assert ef <= 1e-13 and eg <= 1e-13
        else:
            errs = compare_fields(cav, orc)
            log("  after", orc.steps, "steps:", errs)
            assert max(errs.values()) <= 1e-4


@pytest.mark.parametrize("grid", [(2, 2), (2, 5), (5, 2), (3, 3)])
def test_smallest_grids(grid):
    """Grids where every node touches a wall (the 2 x 2 minimum, one-node-wide
    strips): FP64 populations against the oracle from a random state after 1,
    2 and 5 steps, for a power-law and a Newtonian case; step(0) changes
    nothing."""
    nx, ny = grid
    for ci in (0, 1):
        kw = RANDOM_CASES[ci]
        f0, g0 = inputs.random_state(nx, ny, seed=31 + ci, amp=0.05)
        cav = gpu_for(nx, ny, dtype="fp64", **kw)
        cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
        cav.step(0)
        assert cav.steps == 0
        fz, gz = (t.cpu().numpy() for t in cav.populations(torch.float64))
        assert np.abs(fz - f0).max() <= 1e-15 and np.abs(gz - g0).max() <= 1e-15
        orc = oracle_for(nx, ny, **kw)
        orc.set_state(f0, g0)
        for k in (1, 1, 3):
            cav.step(k)
            orc.step(k)
            fg, gg = (t.cpu().numpy() for t in cav.populations(torch.float64))
            fr, gr = orc.state()
            assert np.abs(fg - fr).max() <= 1e-13 and np.abs(gg - gr).max() <= 1e-13, (grid, ci, orc.steps)
        assert abs(cav.nu() - orc.nu_bar()) <= 1e-12 * max(1.0, abs(orc.nu_bar()))


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_grid_taller_than_launch_y_dimension(dtype):
    """A 5 x 70001 grid: more rows than a launch's y dimension takes (65535),
    so the population copy-in, copy-out and field kernels loop over rows.
    Populations (FP64, to 1e-13) and fields (U, V, theta, nu) against the
    oracle after 1, 2 and 5 steps from a random state; the copy-in and
    copy-out return the state unchanged (FP32: rounded once)."""
    kw = RANDOM_CASES[1]
    nx, ny = 5, 70001
    f0, g0 = inputs.random_state(nx, ny, seed=41, amp=0.05)
    log("case: 5x70001 random state", dtype, kw)
    cav = gpu_for(nx, ny, dtype=dtype, **kw)
    cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    fz, gz = (t.cpu().numpy() for t in cav.populations(torch.float64))
    if dtype == "fp64":
        assert np.abs(fz - f0).max() <= 1e-15 and np.abs(gz - g0).max() <= 1e-15
    else:
        assert np.abs(fz - f0).max() <= 1e-7 and np.abs(gz - g0).max() <= 1e-7
    orc = oracle_for(nx, ny, **kw)
    orc.set_state(f0, g0)
    for k in (1, 1, 3):
        cav.step(k)
        orc.step(k)
        errs = compare_fields(cav, orc)
        errs["nu"] = rel_err(cav.viscosity(torch.float64).cpu().numpy(), orc.macros()["nu"])
        if dtype == "fp64":
            fg, gg = (t.cpu().numpy() for t in cav.populations(torch.float64))
            fr, gr = orc.state()
            ef, eg = np.abs(fg - fr).max(), np.abs(gg - gr).max()
            log("  after", orc.steps, "steps: pop err", ef, eg, errs)
            assert ef <= 1e-13 and eg <= 1e-13
            assert max(errs.values()) <= 1e-11
        else:
            log("  after", orc.steps, "steps:", errs)
            assert max(errs.values()) <= 1e-4


SIZES = [(8, 8), (33, 33), (96, 96), (257, 40), (300, 37)]


@pytest.mark.parametrize("size", SIZES)
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [0.5, 1.0, 1.5])
def test_ragged_grids_and_step_counts(size, dtype, n):
    """Grids that are not multiples of the 256-node row tile, non-square,
    odd and even step counts.  Ra = 1e3 and the clamp [0.5, 2] nu0 keep
    tau >= 0.6 so the transient stays well conditioned (as tau -> 1/2 the
    flow amplifies round-off differences); early fields are tiny, so errors
    are taken relative to max(max|ref|, 1e-2)."""
    nx, ny = size
    kw = dict(n=n, Da=1e-2, Ra=1e3, Pr=6.2, eps=0.6, nu_lo=0.5, nu_hi=2.0)
    log("case:", size, dtype, kw)
    cav = gpu_for(nx, ny, dtype=dtype, **kw)
    orc = oracle_for(nx, ny, **kw)
    done = 0
    for k in (1, 1, 499, 499):
        cav.step(k)
        orc.step(k)
        done += k
        Ug, Vg, Tg = gpu_fields(cav)
        Ur, Vr, Tr = orc.fields()
        errs = {name: float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-2))
                for name, a, b in (("U", Ug, Ur), ("V", Vg, Vr), ("theta", Tg, Tr))}
        dnu = compare_nu(cav, orc)
        log("  steps", done, errs, dnu)
        assert max(errs.values()) <= TOL[dtype] and dnu <= TOL[dtype]


def test_powerlaw_cavity_fp32():
    kw = dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6)
    cav = gpu_for(64, dtype="fp32", **kw)
    orc = oracle_for(64, **kw)
    cav.step(6000)
    orc.step(6000)
    errs = compare_fields(cav, orc)
    dnu = compare_nu(cav, orc)
    log("power-law fp32", errs, dnu)
    assert max(errs.values()) <= 1e-4 and dnu <= 1e-4


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_residual_matches_temperature_change(dtype):
    kw = dict(n=0.8, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6)
    cav = gpu_for(40, dtype=dtype, **kw)
    orc = oracle_for(40, **kw)
    T0 = orc.fields()[2]
    for _ in range(2):
        cav.step(1000)
        orc.step(1000)
        T1 = orc.fields()[2]
        r_ref = np.abs(T1 - T0).max()
        r = cav.residual()
        log(dtype, "residual", r, r_ref)
        # theta is O(1): the residual inherits the field bar as an absolute bound
        assert abs(r - r_ref) <= (1e-13 if dtype == "fp64" else 1e-4)
        T0 = T1
    # run_to_steady stops at the first check with r < tol
    r, steps = cav.run_to_steady(tol=1e-3, check_every=500, max_steps=20000)
    assert r < 1e-3 and steps % 500 == 0 and steps <= 20000


def test_graph_replay_equals_single_launches():
    kw = dict(n=0.7, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)
    a = gpu_for(50, 30, dtype="fp32", **kw)
    b = gpu_for(50, 30, dtype="fp32", **kw)
    a.step(3)
    a.step(300)  # odd start parity, graph chunks plus a tail
    for _ in range(303):
        b.step(1)
    fa, ga = a.populations(torch.float32)
    fb, gb = b.populations(torch.float32)
    assert torch.equal(fa, fb) and torch.equal(ga, gb)
    assert a.steps == b.steps == 303


def test_checkpoint_resume_is_bitwise():
    kw = dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6)
    a = gpu_for(48, dtype="fp32", **kw)
    a.step(777)
    snap = a.save_state()
    a.step(500)
    b = gpu_for(48, dtype="fp32", **kw)
    b.load_state(snap)
    assert b.steps == 777
    b.step(500)
    fa, ga = a.populations(torch.float32)
    fb, gb = b.populations(torch.float32)
    assert torch.equal(fa, fb) and torch.equal(ga, gb)
    c = gpu_for(40, dtype="fp32", **kw)
    with pytest.raises(Exception):
        c.load_state(snap)
    # a state saved with other physics is refused (PM_ESTATE) and nothing is loaded
    d = gpu_for(48, dtype="fp32", **dict(kw, n=0.8))
    f0, g0 = d.populations(torch.float32)
    with pytest.raises(P.PmError, match="other physics") as ei:
        d.load_state(snap)
    assert ei.value.code == -4 and d.steps == 0
    fd, gd = d.populations(torch.float32)
    assert torch.equal(f0, fd) and torch.equal(g0, gd)
    # the same physics with the default rates given explicitly loads
    e = gpu_for(48, dtype="fp32", s_e=1.4, s_eps=1.4, s_q=1.2, **kw)
    e.load_state(snap)
    assert e.steps == 777


def test_checkpoint_keeps_the_residual_snapshot():
    """A checkpoint taken between two residual checks carries the snapshot of
    the last check, so the next check after a resume equals the uninterrupted
    run's, at the same step."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6)
    a = gpu_for(40, dtype="fp64", **kw)
    a.step(1000)
    r1, at1 = a.residual(with_step=True)
    assert at1 == 1000 and r1 > 0
    a.step(300)
    snap = a.save_state()
    a.step(700)
    ra, sa = a.residual(with_step=True)
    b = gpu_for(40, dtype="fp64", **kw)
    b.load_state(snap)
    b.step(700)
    rb, sb = b.residual(with_step=True)
    assert (ra, sa) == (rb, sb) and sa == 2000


@pytest.mark.parametrize("max_steps", [6000, 6500, 40_000])
def test_run_to_steady_history_follows_the_library_loop(max_steps):
    """run_to_steady with a history list drives the same chunks and stopping
    rule as pm_run_to_steady (a cap that is not a multiple of the chunk, a
    cap that is reached, a run that settles): same steps, same residual,
    bitwise the same state; the history holds every check's step count,
    residual and Nu, the last being the run's own."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6)
    tol, check = 1e-7, 1000
    a = gpu_for(40, dtype="fp64", **kw)
    ra, sa = a.run_to_steady(tol=tol, check_every=check, max_steps=max_steps)
    b = gpu_for(40, dtype="fp64", **kw)
    hist = []
    rb, sb = b.run_to_steady(tol=tol, check_every=check, max_steps=max_steps, history=hist)
    log(f"cap {max_steps}: {sa} steps, r {ra:.3e}; history {[(s, f'{r:.2e}') for s, r, _ in hist]}")
    assert (ra, sa) == (rb, sb)
    assert [s for s, _, _ in hist] == [min(check * (i + 1), max_steps) for i in range(len(hist))]
    assert hist[-1][0] == sb and hist[-1][1] == rb and hist[-1][2] == b.nu() == a.nu()
    assert all(r >= tol for _, r, _ in hist[:-1])
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert torch.equal(fa, fb) and torch.equal(ga, gb)
    if max_steps == 40_000:
        assert rb < tol and sb < max_steps


def test_runs_are_deterministic():
    kw = dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6)
    outs = []
    for _ in range(2):
        c = gpu_for(130, dtype="fp32", **kw)
        c.step(2000)
        outs.append((c.nu(), c.residual(), [t.cpu() for t in c.fields(torch.float32)]))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    assert all(torch.equal(x, y) for x, y in zip(outs[0][2], outs[1][2]))


def test_nan_is_reported_as_divergence():
    kw = dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6)
    c = gpu_for(16, dtype="fp32", **kw)
    f, g = inputs.random_state(16, 16, seed=5, amp=0.0, amp_T=0.0)
    g[2, 7, 0] = np.nan  # planted from the host in the hot-wall column
    c.set_populations(torch.from_numpy(f), torch.from_numpy(g))
    c.step(3)
    with pytest.raises(Exception) as e:
        c.residual()
    assert getattr(e.value, "code", None) == -3
    with pytest.raises(Exception):
        c.nu()


def test_full_size_4096_fp32_sampled():
    """The 4096^2 throughput workload (FP32, n = 0.8, Da = 1e-2, Ra = 1e5,
    eps = 0.6) in the launch configuration the benchmark times, after 16
    steps, against the oracle at the same size."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)
    N, steps = 4096, 16
    log("case: 4096^2 fp32", kw, steps, "steps")
    cav = gpu_for(N, dtype="fp32", **kw)
    cav.step(steps)
    Ug, Vg, Tg = gpu_fields(cav)
    nu_g = cav.nu()
    del cav
    torch.cuda.empty_cache()
    orc = oracle_for(N, **kw).step(steps)
    Ur, Vr, Tr = orc.fields()
    errs = dict(U=rel_err(Ug, Ur), V=rel_err(Vg, Vr), theta=rel_err(Tg, Tr))
    dnu = abs(nu_g - orc.nu_bar()) / orc.nu_bar()
    log("4096^2:", errs, dnu)
    assert max(errs.values()) <= 1e-4 and dnu <= 1e-4
    # far from the walls the fluid is still exactly at rest after 16 steps
    assert np.all(Ug[100:-100, 100:-100] == 0.0) and np.all(Tg[100:-100, 100:-100] == 0.5)


@pytest.mark.parametrize("rounding", ["nearest", "stochastic"])
def test_full_size_4096_fp32_random_state(rounding):
    """The same 4096^2 workload and launch configuration, started from a random
    non-equilibrium state so that every node moves and the viscosity solve
    runs on the power-law branch everywhere: all fields, every node, against
    the oracle after 5 steps (two-step passes, then one single step) and after
    5 more (a single step, then two-step passes).  This covers every strip and
    row-block edge of the two-step pass at the size it is timed at, including
    the partial last strip and the partial last row block."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)
    N = 4096
    f0, g0 = inputs.random_state(N, N, seed=11, amp=0.02, amp_T=0.1)
    log("case: 4096^2 fp32 from a random state (seed 11)", kw, rounding)
    cav = gpu_for(N, dtype="fp32", rounding=rounding, **kw)
    cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    orc = oracle_for(N, **kw)
    orc.set_state(f0, g0)
    del f0, g0
    for k in (5, 5):
        cav.step(k)
        orc.step(k)
        Ug, Vg, Tg = gpu_fields(cav)
        Ur, Vr, Tr = orc.fields()
        errs = dict(U=rel_err(Ug, Ur), V=rel_err(Vg, Vr), theta=rel_err(Tg, Tr))
        dnu = compare_nu(cav, orc)
        log("  after", orc.steps, "steps:", errs, dnu)
        assert max(errs.values()) <= 1e-4 and dnu <= 1e-4
    del cav
    torch.cuda.empty_cache()


def _wall_map(n, m=64):
    """For each of n indices, the index in an m-wide grid at the same distance
    from the nearer wall (the first and last m/2); all others map to m/2."""
    h = m // 2
    i = np.arange(n)
    return np.where(i < h, i, np.where(i >= n - h, i - (n - m), h))


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_largest_grid_from_rest(dtype):
    """The largest grid the library takes: 32768 x 32767 nodes, just under
    2^30, with population offsets far past 2^32 elements.  The test runs 16
    steps from rest (FP32: single steps and two-step passes).  From a uniform
    rest state with uniform walls, after k steps only nodes within k of the
    hot and cold walls have moved, and each node's state depends only on its
    distance to the walls near it.  So the oracle on a 64 x 64 grid with the
    same lattice constants fixes every node:
      * corners map to corners;
      * the rest of each 32-wide border strip maps to the small grid's middle
        row or column;
      * everything else is exactly at rest.
    Also checked: Nu against Eq. (24) over the rows so mapped.

    FP32 bar: 1e-4 of max|X| (as elsewhere).  FP64 bar: 1e-13 absolute in
    lattice units, the bar the random-state tests put on populations: |dU|
    U_lb, |dV| U_lb, |dtheta| <= 1e-13.  Sixteen steps from rest the
    velocities are ~1e-7 of the O(1) populations, so the oracle's FP64
    rounding of those populations (it stores them unshifted) reaches ~1e-9
    of max|U|, and a bar relative to max|U| would measure that rounding."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)
    nx, ny, m, steps = 32768, 32767, 64, 16
    h = m // 2
    tol = TOL[dtype]
    need = P.workspace_bytes(P.make_params(nx, ny, dtype=dtype, **kw)) + 3 * nx * ny * (4 if dtype == "fp32" else 8)
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    lat = O.map_physics(O.physics(nx, ny, **kw))
    lat.nx, lat.ny = m, m
    S = O.Oracle(lat).step(steps).fields()
    # the premise: the small grid's middle rows are alike, its middle columns
    # untouched (a margin of 16 nodes to the 32-node strips)
    for X in S:
        assert np.array_equal(X[16:48], np.broadcast_to(X[h], (32, m)))
        assert np.array_equal(X[:, 16:48], np.broadcast_to(X[:, h:h + 1], (m, 32)))
    log("case: largest grid", nx, "x", ny, dtype, kw, steps, "steps from rest")
    cav = gpu_for(nx, ny, dtype=dtype, **kw)
    cav.step(1)
    cav.step(steps - 1)
    assert cav.steps == steps
    nu_g = cav.nu()
    G = cav.fields(torch.float32 if dtype == "fp32" else torch.float64)
    rmap, cmap = _wall_map(ny, m), _wall_map(nx, m)
    errs = {}
    for name, X, R in zip(("U", "V", "theta"), G, S):
        strips = ((X[:, :h], R[rmap][:, :h]), (X[:, -h:], R[rmap][:, -h:]),
                  (X[:h, :], R[:h][:, cmap]), (X[-h:, :], R[-h:][:, cmap]))
        e = max(np.abs(x.cpu().double().numpy() - r).max() for x, r in strips)
        if dtype == "fp32":
            errs[name] = e / np.abs(R).max()  # relative to max|X|
        else:
            errs[name] = e * (lat.U_lb if name != "theta" else 1.0)  # absolute, lattice units
    inner = [X[h:-h, h:-h] for X in G]
    assert int(torch.count_nonzero(inner[0])) == 0 and int(torch.count_nonzero(inner[1])) == 0
    assert bool(torch.all(inner[2] == 0.5))
    th = S[2]
    nu_r = float(np.sum(nx * (8.0 - 9.0 * th[rmap, 0] + th[rmap, 1]) / 3.0) / ny)
    dnu = abs(nu_g - nu_r) / abs(nu_r)
    log("  fields", errs, "Nu", nu_g, nu_r, dnu)
    del G, inner, cav
    torch.cuda.empty_cache()
    bar = 1e-4 if dtype == "fp32" else 1e-13
    assert max(errs.values()) <= bar and dnu <= tol


def test_stream_function():
    """psi from the GPU against its definition applied to the oracle's U
    (midpoint rule up each column, psi = 0 on the bottom wall), FP64; at the
    steady 64 x 64 Newtonian cavity the top-wall value (each column's net
    flux) is small, and integrating -V along x from the left wall gives
    nearly the same psi."""
    N, steps = 64, 20000
    cav = gpu_for(N, **CFG0)
    cav.step(steps)
    psi = cav.stream_function().cpu().numpy()
    orc = oracle_for(N, **CFG0).step(steps)
    U, V, _ = orc.fields()
    ref = (np.cumsum(U, axis=0) - 0.5 * U) / N
    scale = np.abs(ref).max()
    assert np.abs(psi - ref).max() <= 1e-11 * scale
    top = (np.cumsum(U, axis=0)[-1]) / N
    psi_x = -(np.cumsum(V, axis=1) - 0.5 * V) / N
    print(f"max|psi| {scale:.4e}, max|column flux| {np.abs(top).max():.3e}, "
          f"max|psi_y - psi_x| {np.abs(ref - psi_x).max():.3e}")
    # both vanish only up to the discretisation error of the nodal velocity
    # (3e-3 of max|psi| measured at 64 x 64)
    assert np.abs(top).max() <= 1e-2 * scale
    assert np.abs(ref - psi_x).max() <= 1e-2 * scale
    psi32 = cav.stream_function(torch.float32).cpu().numpy()
    assert np.abs(psi32 - psi).max() <= 1e-6 * scale


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_stream_function_tall_grid(dtype):
    """The column scan over several row blocks with a ragged last block (37 x
    150 and 300 x 1030, from random states): psi against its definition applied
    to the same cavity's U field, in FP64."""
    for nx, ny in ((37, 150), (300, 1030)):
        f0, g0 = inputs.random_state(nx, ny, seed=7, amp=0.05)
        cav = gpu_for(nx, ny, dtype=dtype, **CFG0)
        cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
        cav.step(3)
        U = cav.fields(torch.float64)[0].cpu().numpy()
        psi = cav.stream_function().cpu().numpy()
        ref = (np.cumsum(U, axis=0) - 0.5 * U) / nx
        err = np.abs(psi - ref).max() / np.abs(ref).max()
        log(f"psi {nx}x{ny} {dtype}: max|psi| {np.abs(ref).max():.3e}, rel err {err:.2e}")
        assert err <= 1e-12


PAIR_SIZES = [(8, 8), (33, 21), (252, 70), (300, 130), (520, 67), (1100, 400)]


@pytest.mark.parametrize("size", PAIR_SIZES)
@pytest.mark.parametrize("n,logda,rounding", [(1.0, False, "nearest"), (0.6, False, "nearest"),
                                              (0.8, True, "nearest"), (0.6, False, "stochastic")])
def test_two_step_kernel_equals_single_steps(size, n, logda, rounding):
    """The two-step kernel (forced with PM_STEP_PAIR: by default it runs only
    on grids large enough to fill the GPU) against the single-step kernel:
    both must give the same populations bit for bit -- on grids narrower and
    wider than one 252-column strip, with partial 24-row chunks, and on
    1100 x 400 (5 strips x 25 row groups), whose first 64 tiles are dealt to
    the XCDs in blocks and the rest in launch order -- from a random state,
    and across a graph-replayed run (k >= 128, starting at an odd step
    count)."""
    nx, ny = size
    kw = dict(n=n, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6, rounding=rounding)
    ld = inputs.logda_field(max(nx, ny), seed=2)[:ny, :nx].copy() if logda else None
    a = gpu_for(nx, ny, dtype="fp32", logda=ld, step_kernel="pair", **kw)
    b = gpu_for(nx, ny, dtype="fp32", logda=ld, step_kernel="single", **kw)
    f0, g0 = inputs.random_state(nx, ny, seed=21, amp=0.02, amp_T=0.1)
    for c in (a, b):
        c.set_populations(torch.from_numpy(f0).float(), torch.from_numpy(g0).float())
    for rep in range(3):
        a.step(4)
        for _ in range(4):
            b.step(1)
    a.step(1)
    b.step(1)
    a.step(130)  # odd start: one single step, 32 two-step pairs, one single step (graph replay)
    for _ in range(130):
        b.step(1)
    fa, ga = a.populations(torch.float32)
    fb, gb = b.populations(torch.float32)
    assert a.steps == b.steps == 143
    assert torch.equal(fa, fb) and torch.equal(ga, gb)
    assert a.nu() == b.nu()

