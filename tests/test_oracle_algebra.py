"""Pins of the oracle's single-node algebra against definitions that do not
come from the oracle itself.

- The moment transforms are invertible and orthogonal (Eq. (12) needs M^-1).
- The equilibrium and forcing populations satisfy the moment constraints that
  define them (rho, rho u, rho c_s^2 I + rho u u / eps; Guo-Zhao forcing:
  0, rho F, rho (uF + Fu)/eps), and their moments in the M basis equal the
  closed forms written out in the design notes.
- The strain rate of Eqs. (22)-(23) recovers an imposed velocity gradient
  from the Chapman-Enskog non-equilibrium populations of that gradient.
- With every rate equal to 1/tau the MRT update (Eq. 12) reduces to the
  textbook single-relaxation-time (BGK) update with Guo forcing, and the
  D2Q5 MRT update (Eq. 18) to BGK advection-diffusion.
- The viscosity solve returns the fixed point of Eq. (21) with Eqs. (22)-(23).
"""
import math

import numpy as np
import pytest

import oracle as O

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
EX5 = np.array([0, 1, 0, -1, 0])
EY5 = np.array([0, 0, 1, 0, -1])
W5 = np.array([1 / 3] + [1 / 6] * 4)


def test_transforms_invertible_and_orthogonal():
    M, Mi, N, Ni = O.matrices()
    assert np.abs(M @ Mi - np.eye(9)).max() < 1e-15
    assert np.abs(N @ Ni - np.eye(5)).max() < 1e-15
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert list(np.diag(G)) == [9, 36, 36, 6, 12, 6, 12, 4, 4]
    H = N @ N.T
    assert np.abs(H - np.diag(np.diag(H))).max() == 0.0
    assert list(np.diag(H)) == [5, 2, 2, 20, 4]
    # the first rows are the conserved moments: density and momentum
    assert np.array_equal(M[0], np.ones(9)) and np.array_equal(M[3], EX) and np.array_equal(M[5], EY)
    assert np.array_equal(N[0], np.ones(5))


@pytest.mark.parametrize("eps", [1.0, 0.6, 0.35])
def test_equilibrium_moment_constraints(eps):
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        ux, uy = 0.1 * rng.standard_normal(2)
        f = O.feq(eps, rho, ux, uy)
        assert abs(f.sum() - rho) < 1e-15
        assert abs((EX * f).sum() - rho * ux) < 1e-15
        assert abs((EY * f).sum() - rho * uy) < 1e-15
        # second moment: rho c_s^2 delta + rho u u / eps
        assert abs((EX * EX * f).sum() - (rho / 3 + rho * ux * ux / eps)) < 1e-15
        assert abs((EY * EY * f).sum() - (rho / 3 + rho * uy * uy / eps)) < 1e-15
        assert abs((EX * EY * f).sum() - rho * ux * uy / eps) < 1e-15
        M, _, _, _ = O.matrices()
        uu = ux * ux + uy * uy
        closed = np.array([rho, -2 * rho + 3 * rho * uu / eps, rho - 3 * rho * uu / eps,
                           rho * ux, -rho * ux, rho * uy, -rho * uy,
                           rho * (ux * ux - uy * uy) / eps, rho * ux * uy / eps])
        assert np.abs(M @ f - closed).max() < 1e-14


@pytest.mark.parametrize("eps", [1.0, 0.6])
def test_forcing_moment_constraints(eps):
    rng = np.random.default_rng(4)
    M, _, _, _ = O.matrices()
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        ux, uy, Fx, Fy = 0.1 * rng.standard_normal(4)
        Fi = O.forcing(eps, rho, ux, uy, Fx, Fy)
        assert abs(Fi.sum()) < 1e-16
        assert abs((EX * Fi).sum() - rho * Fx) < 1e-16
        assert abs((EY * Fi).sum() - rho * Fy) < 1e-16
        assert abs((EX * EX * Fi).sum() - 2 * rho * ux * Fx / eps) < 1e-16
        assert abs((EY * EY * Fi).sum() - 2 * rho * uy * Fy / eps) < 1e-16
        assert abs((EX * EY * Fi).sum() - rho * (ux * Fy + uy * Fx) / eps) < 1e-16
        uF = ux * Fx + uy * Fy
        closed = rho * np.array([0, 6 * uF / eps, -6 * uF / eps, Fx, -Fx, Fy, -Fy,
                                 2 * (ux * Fx - uy * Fy) / eps, (ux * Fy + uy * Fx) / eps])
        assert np.abs(M @ Fi - closed).max() < 1e-15


def test_thermal_equilibrium_moments():
    rng = np.random.default_rng(5)
    _, _, N, _ = O.matrices()
    for _ in range(20):
        T = rng.uniform(0, 1)
        ux, uy = 0.1 * rng.standard_normal(2)
        g = O.geq(T, ux, uy)
        assert abs(g.sum() - T) < 1e-15
        assert abs((EX5 * g).sum() - T * ux) < 1e-15
        assert abs((EY5 * g).sum() - T * uy) < 1e-15
        # isotropic second moment c_s^2 T with c_s^2 = 1/3
        assert abs((EX5 * EX5 * g).sum() - T / 3) < 1e-15
        assert abs((EY5 * EY5 * g).sum() - T / 3) < 1e-15
        assert abs((EX5 * EY5 * g).sum()) < 1e-15
        assert np.abs(N @ g - np.array([T, ux * T, uy * T, -2 * T / 3, 0])).max() < 1e-15


@pytest.mark.parametrize("tau", [0.6, 1.0, 2.3])
def test_strain_rate_recovers_imposed_gradient(tau):
    """Chapman-Enskog: f = f_eq - 3 tau w_i rho (e_a e_b - delta/3) S_ab (c_s^2
    = 1/3) is the first-order non-equilibrium of a flow with symmetric velocity
    gradient S.  With s_e = s_nu = 1/tau, Eqs. (22)-(23) must give exactly
    gamma_ab = S_ab, |gamma|^2 = 2 S:S."""
    rng = np.random.default_rng(6)
    lat = O.lattice(4, eps=1.0, s_e=1 / tau)
    for _ in range(10):
        rho = 1 + 0.05 * rng.standard_normal()
        vx, vy = 0.05 * rng.standard_normal(2)
        a, b, c = 1e-3 * rng.standard_normal(3)
        S = np.array([[a, c], [c, b]])
        Q = np.stack([EX * EX - 1 / 3, EX * EY, EX * EY, EY * EY - 1 / 3])
        fneq = -3 * tau * W9 * rho * (Q[0] * S[0, 0] + Q[1] * S[0, 1] + Q[2] * S[1, 0] + Q[3] * S[1, 1])
        f = O.feq(1.0, rho, vx, vy) + fneq
        g2 = O.shear_sq(lat, f, rho, vx, vy, 1 / tau)
        assert g2 == pytest.approx(2 * (S * S).sum(), rel=1e-9)


def _bgk_guo_reference(lat, f, g, K):
    """Textbook single-relaxation-time update with Guo forcing (porous form of
    Guo & Zhao 2002) and BGK advection-diffusion; written independently of the
    moment-space oracle."""
    eps, nu = lat.eps, lat.nu0
    tau = 3 * nu + 0.5
    rho = f.sum()
    T = g.sum()
    Gx, Gy = lat.gx, lat.gy + lat.gbeta * (T - lat.T_m)
    vx = (EX * f).sum() / rho + eps * Gx / 2
    vy = (EY * f).sum() / rho + eps * Gy / 2
    invK = 0.0 if math.isinf(K) else 1 / K
    c0 = 0.5 * (1 + eps * nu * invK / 2)
    c1 = eps * lat.Feps * math.sqrt(invK) / 2
    den = c0 + math.sqrt(c0 * c0 + c1 * math.hypot(vx, vy))
    ux, uy = vx / den, vy / den
    um = math.hypot(ux, uy)
    Fx = -eps * nu * invK * ux - eps * lat.Feps * math.sqrt(invK) * um * ux + eps * Gx
    Fy = -eps * nu * invK * uy - eps * lat.Feps * math.sqrt(invK) * um * uy + eps * Gy
    eu = EX * ux + EY * uy
    eF = EX * Fx + EY * Fy
    feq = W9 * rho * (1 + 3 * eu + 4.5 * eu * eu / eps - 1.5 * (ux * ux + uy * uy) / eps)
    Fi = W9 * rho * (3 * eF + 9 * eu * eF / eps - 3 * (ux * Fx + uy * Fy) / eps)
    fo = f - (f - feq) / tau + (1 - 1 / (2 * tau)) * Fi
    taug = 3 * lat.alpha + 0.5
    geq = W5 * T * (1 + 3 * (EX5 * ux + EY5 * uy))
    go = g - (g - geq) / taug
    return fo, go


@pytest.mark.parametrize("porous", [False, True])
def test_mrt_with_equal_rates_is_bgk(porous):
    rng = np.random.default_rng(7)
    nu, alpha = 0.07, 0.11
    s = 1 / (3 * nu + 0.5)
    sg = 1 / (3 * alpha + 0.5)
    kw = dict(nu0=nu, nu_min=nu, nu_max=nu, alpha=alpha, s_e=s, s_eps=s, s_q=s,
              sT_e=sg, sT_nu=sg, gbeta=3e-3, gx=1e-4, gy=-2e-4)
    if porous:
        kw.update(eps=0.6, K=40.0, Feps=0.3)
    lat = O.lattice(4, **kw)
    for _ in range(10):
        f = W9 * (1 + 0.05 * rng.standard_normal(9))
        g = W5 * (0.5 + 0.2 * rng.standard_normal(5))
        fo, go, _ = O.collide_node(lat, lat.K, f, g)
        fr, gr = _bgk_guo_reference(lat, f, g, lat.K)
        assert np.abs(fo - fr).max() < 1e-15
        assert np.abs(go - gr).max() < 1e-15


@pytest.mark.parametrize("npow", [0.4, 0.6, 0.8, 1.3, 1.6])
def test_viscosity_is_fixed_point_of_power_law(npow):
    """nu = clamp(nu0 (gamma_scale |gamma(s(nu))|)^(n-1), nu_min, nu_max),
    s(nu) = 1/(3 nu + 1/2): Eq. (21) with Eqs. (15), (22), (23)."""
    rng = np.random.default_rng(8)
    nu0 = 0.05
    lat = O.lattice(4, npow=npow, nu0=nu0, nu_min=0.1 * nu0, nu_max=10 * nu0,
                    gamma_scale=500.0, eps=0.8)
    hits = {"lo": 0, "hi": 0, "mid": 0}
    for trial in range(300):
        amp = 10 ** rng.uniform(-13, 1)
        rho = 1 + 0.02 * rng.standard_normal()
        vx, vy = 0.05 * rng.standard_normal(2)
        f = O.feq(lat.eps, rho, vx, vy) + amp * rng.standard_normal(9) * W9
        f -= W9 * (f.sum() - rho)  # keep rho exact
        nu = O.viscosity(lat, f, rho, vx, vy)
        s = 1 / (3 * nu + 0.5)
        gam = math.sqrt(O.shear_sq(lat, f, rho, vx, vy, s))
        target = min(max(nu0 * (lat.gamma_scale * gam) ** (npow - 1), lat.nu_min), lat.nu_max)
        assert nu == pytest.approx(target, rel=1e-13)
        if nu == lat.nu_min:
            hits["lo"] += 1
        elif nu == lat.nu_max:
            hits["hi"] += 1
        else:
            hits["mid"] += 1
    assert hits["mid"] > 20 and hits["lo"] + hits["hi"] > 10


def test_viscosity_newtonian_and_rest():
    lat = O.lattice(4, npow=1.0, nu0=0.05, nu_min=0.005, nu_max=0.5)
    f = O.feq(1.0, 1.0, 0.01, 0.02) + 1e-4 * W9
    assert O.viscosity(lat, f, 1.0, 0.01, 0.02) == 0.05
    # at rest there is no shear: shear-thinning fluid sits at the upper bound,
    # shear-thickening at the lower bound (the clamp of Eq. 21)
    f0 = O.feq(1.0, 1.0, 0.0, 0.0)
    lat.npow = 0.6
    assert O.viscosity(lat, f0, 1.0, 0.0, 0.0) == lat.nu_max
    lat.npow = 1.4
    assert O.viscosity(lat, f0, 1.0, 0.0, 0.0) == lat.nu_min


def test_physics_mapping_reproduces_groups():
    """Step 0: at n = 1 the lattice parameters give back Ra = g beta L^3/(nu
    alpha) and Pr = nu/alpha (Eq. 6), and the known values of the 64^2 case."""
    p = O.physics(64, n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6)
    L = O.map_physics(p)
    N = 64
    assert L.gbeta * N ** 3 / (L.nu0 * L.alpha) == pytest.approx(1e3, rel=1e-14)
    assert L.nu0 / L.alpha == pytest.approx(10.0, rel=1e-14)
    assert L.nu0 == pytest.approx(1.16848, rel=1e-5)
    assert L.alpha == pytest.approx(0.116848, rel=1e-5)
    assert L.K == pytest.approx(409.6, rel=1e-15)
    assert L.Feps == pytest.approx(0.3074437, rel=1e-6)
    # power-law scaling: Ra = g beta L^(2n+1) / (nu alpha^n), Pr = nu/(alpha^(2-n) L^(2(n-1)))
    p = O.physics(256, n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6)
    L = O.map_physics(p)
    N, U = 256, L.U_lb
    # in lattice units the "nu" of Eq. (6) is the consistency coefficient
    # K_c = nu0_lb (N/U)^(n-1) of nu = K_c gamma^(n-1)
    Kc = L.nu0 * (N / U) ** (0.6 - 1)
    assert L.gbeta * N ** (2 * 0.6 + 1) / (Kc * L.alpha ** 0.6) == pytest.approx(1e5, rel=1e-12)
    assert Kc / (L.alpha ** (2 - 0.6) * N ** (2 * (0.6 - 1))) == pytest.approx(10.0, rel=1e-12)
    with pytest.raises(ValueError):
        O.map_physics(O.physics(64, eps=1.5))


@pytest.mark.parametrize("npow", [0.6, 1.4])
@pytest.mark.parametrize("g1,g2", [(0.3, 30.0), (0.01, 1e6)])
def test_viscosity_with_shear_rate_thresholds(npow, g1, g2):
    """PM_CLAMP_GAMMA (clamp_mode 1): Eq. (21) with the shear-rate thresholds
    gamma1, gamma2 made continuous, nu = nu0 clamp(gamma*, gamma1, gamma2)^(n-1),
    gamma* = (N / U_lb) |gamma| the nondimensional shear rate.  Checked at
    states on both sides of each threshold (the paper's 0.01 and 1e6, and a
    narrower pair that the sampled shear rates straddle on both ends)."""
    N = 64
    lat = O.map_physics(O.physics(N, n=npow, Ra=1e5, Pr=10.0, eps=0.8, clamp_mode=1,
                                  nu_lo=g1, nu_hi=g2))
    U = 0.1 / math.sqrt(3.0)
    assert lat.gamma_scale == pytest.approx(N / U, rel=1e-15)
    nu0 = 10.0 / math.sqrt(1e5) ** (2 - npow) * U * N  # Eq. (21)'s nu0 in lattice units
    assert lat.nu0 == pytest.approx(nu0, rel=1e-14)
    rng = np.random.default_rng(21)
    side = {"below": 0, "between": 0, "above": 0}
    for trial in range(400):
        amp = 10 ** rng.uniform(-9, 1)
        rho = 1 + 0.02 * rng.standard_normal()
        vx, vy = 0.05 * rng.standard_normal(2)
        f = O.feq(lat.eps, rho, vx, vy) + amp * rng.standard_normal(9) * W9
        f -= W9 * (f.sum() - rho)
        nu = O.viscosity(lat, f, rho, vx, vy)
        gstar = lat.gamma_scale * math.sqrt(O.shear_sq(lat, f, rho, vx, vy, 1 / (3 * nu + 0.5)))
        expect = nu0 * min(max(gstar, g1), g2) ** (npow - 1)
        assert nu == pytest.approx(expect, rel=1e-12), (gstar, nu, expect)
        side["below" if gstar < g1 else "above" if gstar > g2 else "between"] += 1
    assert side["below"] > 10 and side["between"] > 10, side
    if g2 < 1e3:
        assert side["above"] > 10, side
