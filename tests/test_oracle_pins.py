"""Pins of the oracle's full update (collision + streaming + walls) against
closed-form solutions, a brute-force boundary-value solve, and exact
invariants -- none of which comes from the oracle itself.

Flow (D2Q9 MRT, Eq. 12, halfway bounce-back walls):
  * Newtonian Poiseuille: with the qx/qy rate chosen so that
    (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16, the bounce-back wall sits exactly
    halfway and the Stokes-limit profile is reproduced to round-off; at the
    paper's s_q = 1.2 the error is second order in N.
  * Power-law Poiseuille with the clamped viscosity of Eq. (21): piecewise
    closed form; second-order convergence of velocity and shear rate.
  * Brinkman channel (porous drag): cosh closed form.
  * Forchheimer channel: 1-D BVP solved by brute force (Newton on a fine
    finite-difference grid).
  * Natural convection between differentially heated vertical plates:
    linear temperature and the cubic velocity profile -- pins the buoyancy
    term's sign and magnitude and the eps factor of the force.
Thermal (D2Q5 MRT, Eq. 18, anti-bounce-back Dirichlet walls):
  * Conduction: theta = 1 - x/N exactly, Nu = 1 (Eq. 24).
  * Eq. (24) exact for theta quadratic in X with a wall slope varying in Y.
  * 1-D transient diffusion against its Fourier series.
  * Advection of a sine wave by a uniform flow (periodic box).
Invariants: exact mass conservation; the discrete energy balance through the
two Dirichlet walls; the rest state; centro-symmetry of the cavity restored at
second order in 1/N.
"""
import math

import numpy as np
import pytest

import oracle as O


def channel(N, nx=2, **kw):
    """Flow along x between walls at y = 0 and y = N (periodic in x)."""
    return O.lattice(nx, N, periodic_x=1, **kw)


def magic_sq(nu):
    tau = 3 * nu + 0.5
    return 1 / (0.5 + (3 / 16) / (tau - 0.5))


def test_newtonian_poiseuille_exact_at_magic_rate():
    N, nu, gx = 16, 0.1, 1e-7
    o = O.Oracle(channel(N, nu0=nu, nu_min=nu, nu_max=nu, gx=gx, s_q=magic_sq(nu)))
    o.step(int(25 * N * N / nu))
    ux = o.macros()["ux"][:, 0]
    y = np.arange(N) + 0.5
    ua = gx * y * (N - y) / (2 * nu)
    assert np.abs(ux - ua).max() / ua.max() < 1e-9


def test_newtonian_poiseuille_second_order_at_paper_rates():
    nu, errs = 0.1, []
    for N in (8, 16, 32):
        gx = 1e-7
        o = O.Oracle(channel(N, nu0=nu, nu_min=nu, nu_max=nu, gx=gx))
        o.step(int(20 * N * N / nu))
        ux = o.macros()["ux"][:, 0]
        y = np.arange(N) + 0.5
        ua = gx * y * (N - y) / (2 * nu)
        errs.append(np.abs(ux - ua).max() / ua.max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < p < 2.2 for p in orders), (errs, orders)


def powerlaw_profile(y, N, gx, nu0, n, c, nu_min, nu_max):
    """Closed-form velocity and shear rate of a clamped power-law fluid in a
    plane channel driven by the body force gx (unit density): stress
    sigma = gx |N/2 - y|, nu(gamma) = clamp(nu0 (c gamma)^(n-1), nu_min,
    nu_max), gamma(sigma) inverts sigma = nu(gamma) gamma."""
    Kc = nu0 * c ** (n - 1)  # sigma = Kc gamma^n on the power branch
    # branch points in gamma and sigma
    ga = (nu_max / Kc) ** (1 / (n - 1)) if n != 1 else 0.0
    gb = (nu_min / Kc) ** (1 / (n - 1)) if n != 1 else np.inf
    if n > 1:
        ga, gb = gb, ga  # low-shear branch is nu_min for shear-thickening
    nu_low = nu_max if n < 1 else nu_min
    nu_high = nu_min if n < 1 else nu_max
    sa, sb = nu_low * ga, nu_high * gb

    def gamma(s):
        return np.where(s <= sa, s / nu_low,
                        np.where(s <= sb, (np.maximum(s, 0) / Kc) ** (1 / n), s / nu_high))

    def Gam(s):  # int_0^s gamma(t) dt
        s = np.asarray(s, dtype=float)
        p1 = np.minimum(s, sa)
        out = p1 ** 2 / (2 * nu_low)
        p2 = np.clip(s, sa, sb)
        out = out + (p2 ** (1 + 1 / n) - sa ** (1 + 1 / n)) / ((1 + 1 / n) * Kc ** (1 / n))
        p3 = np.maximum(s, sb)
        out = out + (p3 ** 2 - sb ** 2) / (2 * nu_high)
        return out

    sig = gx * np.abs(N / 2 - y)
    sw = gx * N / 2
    return (Gam(sw) - Gam(sig)) / gx, gamma(sig), (sa, sb, sw)


@pytest.mark.parametrize("n", [0.5, 1.5])
def test_powerlaw_poiseuille_converges_to_closed_form(n):
    """Eq. (21) with the shear rate of Eqs. (22)-(23): the profile and the local
    shear rate converge to the closed form, with all three viscosity branches
    active across the channel."""
    errs_u, errs_g = [], []
    for N in (16, 32, 64):
        # the same nondimensional problem at each N: nu ~ N at fixed U
        U = 0.02 if n < 1 else 0.004
        nu0 = 0.1 * N / 32
        c = N / U
        sw = (16.0 if n < 1 else 60.0) * nu0 * U / N  # wall stress
        gx = 2 * sw / N
        nu_min, nu_max = 0.3 * nu0, 3.0 * nu0
        o = O.Oracle(channel(N, nu0=nu0, npow=n, nu_min=nu_min, nu_max=nu_max,
                             gamma_scale=c, gx=gx))
        o.step(int(4 * N * N / nu_min))
        m = o.macros()
        y = np.arange(N) + 0.5
        ua, gam, (sa, sb, sw_) = powerlaw_profile(y, N, gx, nu0, n, c, nu_min, nu_max)
        assert 0 < sa < sb < sw_
        errs_u.append(np.abs(m["ux"][:, 0] - ua).max() / ua.max())
        # local shear rate through the stress balance nu * gamma = sigma
        gam_lb = gx * np.abs(N / 2 - y) / m["nu"][:, 0]
        errs_g.append(np.abs(gam_lb - gam).max() / gam.max())
    # the kinks of the clamped law limit the order; a wrong exponent, clamp or
    # strain-rate factor would give O(1) errors
    assert errs_u[2] < 1e-3 and errs_u[0] / errs_u[2] > 3, errs_u
    assert errs_g[2] < 2e-2 and errs_g[0] > errs_g[2], errs_g


def test_brinkman_channel():
    errs = []
    for N in (16, 32, 64):
        nu, eps, gx = 0.1, 0.6, 1e-7
        K = (N / 8) ** 2  # Da = 1/64 fixed as N varies
        o = O.Oracle(channel(N, nu0=nu, nu_min=nu, nu_max=nu, gx=gx, eps=eps, K=K))
        o.step(int(3 * N * N / nu))
        y = np.arange(N) + 0.5
        r = math.sqrt(eps / K)
        ua = gx * K / nu * (1 - np.cosh(r * (y - N / 2)) / math.cosh(r * N / 2))
        errs.append(np.abs(o.macros()["ux"][:, 0] - ua).max() / ua.max())
    assert errs[2] < 2e-3 and errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs


def forchheimer_bvp(N, nu, eps, K, Feps, gx, m=4000):
    """Brute force: nu u'' - eps nu u/K - eps F u|u|/sqrt(K) + eps gx = 0,
    u(0) = u(N) = 0, by Newton's method on a fine central-difference grid
    (second order in 1/m; m = 4000 makes that error ~1e-7 relative)."""
    from scipy.linalg import solve_banded
    x = np.linspace(0, N, m + 1)
    h = x[1] - x[0]
    u = np.zeros(m + 1)
    for _ in range(60):
        ui = u[1:-1]
        R = nu * (u[2:] - 2 * ui + u[:-2]) / h ** 2 - eps * nu * ui / K \
            - eps * Feps * ui * np.abs(ui) / math.sqrt(K) + eps * gx
        d = -2 * nu / h ** 2 - eps * nu / K - 2 * eps * Feps * np.abs(ui) / math.sqrt(K)
        ab = np.zeros((3, m - 1))
        ab[0, 1:] = nu / h ** 2
        ab[1] = d
        ab[2, :-1] = nu / h ** 2
        du = solve_banded((1, 1), ab, -R)
        u[1:-1] += du
        if np.abs(du).max() <= 1e-15 * np.abs(u).max():
            break
    return x, u


def test_forchheimer_channel_against_bvp():
    errs = []
    for N in (16, 32, 64):
        nu, eps, Feps = 0.05 * N / 32, 0.6, 0.3074
        K = (N / 8) ** 2
        U = 0.03
        gx = 32 * U * nu / N ** 2 * 8  # drives u_max of order U
        o = O.Oracle(channel(N, nu0=nu, nu_min=nu, nu_max=nu, gx=gx, eps=eps, K=K,
                             Feps=Feps))
        o.step(int(3 * N * N / nu))
        x, u = forchheimer_bvp(N, nu, eps, K, Feps, gx)
        y = np.arange(N) + 0.5
        ua = np.interp(y, x, u)
        if N == 32:
            # the Darcy-only solution differs: the quadratic drag is active
            xd, ud = forchheimer_bvp(N, nu, eps, K, 0.0, gx)
            assert np.abs(np.interp(y, xd, ud) - ua).max() / ua.max() > 0.05
        errs.append(np.abs(o.macros()["ux"][:, 0] - ua).max() / ua.max())
    assert errs[2] < 2e-3 and errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs


@pytest.mark.parametrize("eps", [1.0, 0.6])
def test_natural_convection_between_vertical_plates(eps):
    """Hot wall x = 0, cold wall x = N, periodic in y: conduction profile and
    the cubic V(xi) = eps g beta N^2 / (12 nu) xi (1 - xi)(1 - 2 xi)."""
    errs = []
    for N in (16, 32):
        nu, alpha, gb = 0.1, 0.1, 1e-6 / N
        lat = O.lattice(N, 2, periodic_y=1, nu0=nu, nu_min=nu, nu_max=nu,
                        alpha=alpha, gbeta=gb, eps=eps)
        o = O.Oracle(lat)
        o.step(int(4 * N * N / min(nu, alpha)))
        m = o.macros()
        xi = (np.arange(N) + 0.5) / N
        assert np.abs(m["T"][0] - (1 - xi)).max() < 1e-12
        va = eps * gb * N ** 2 / (12 * nu) * xi * (1 - xi) * (1 - 2 * xi)
        assert np.all(m["uy"][0, : N // 2 - 1] > 0)  # hot fluid rises
        errs.append(np.abs(m["uy"][0] - va).max() / np.abs(va).max())
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 3.5, errs


def test_conduction_nusselt_is_one():
    for N in (8, 13, 32):
        o = O.Oracle(O.lattice(N, N + 3, alpha=0.3))
        o.step(int(15 * N * N / 0.3))
        T = o.macros()["T"]
        x = (np.arange(N) + 0.5) / N
        assert np.abs(T - (1 - x)[None, :]).max() < 1e-12
        assert abs(o.nu_bar() - 1.0) < 1e-12


def test_nusselt_is_exact_for_quadratic_temperature():
    """Eq. (24) read as a one-sided second-order gradient through the wall
    value and the first two nodes, averaged by the midpoint rule in Y: exact
    for theta quadratic in X with a wall slope that varies along the wall.  (A
    linear profile cannot tell this from a first-order gradient; the
    curvature term b here can.)"""
    N, ny = 24, 10
    X = (np.arange(N) + 0.5) / N
    Y = (np.arange(ny) + 0.5) / ny
    a = -0.7 + 0.3 * np.cos(2 * math.pi * Y)  # wall slope d theta / dX at X = 0
    b = 0.45
    theta = 1.0 + a[:, None] * X[None, :] + b * X[None, :] ** 2
    w9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    w5 = np.array([1 / 3] + [1 / 6] * 4)
    o = O.Oracle(O.lattice(N, ny, alpha=0.2))
    f = np.broadcast_to(w9[:, None, None], (9, ny, N)).copy()
    g = w5[:, None, None] * theta[None]
    o.set_state(f, g)
    assert abs(o.nu_bar() - 0.7) < 1e-13
    # a first-order one-sided gradient would be off by b / (2 N)
    first_order = np.mean((1.0 - theta[:, 0]) / (0.5 / N))
    assert abs(first_order - 0.7) > 0.5 * b / (2 * N)


def test_transient_diffusion_against_fourier_series():
    errs = []
    for N in (16, 32, 64):
        alpha = 0.1
        t = int(round(0.05 * N * N / alpha))
        o = O.Oracle(O.lattice(N, 3, alpha=alpha))
        o.step(t)
        T = o.macros()["T"][1]
        x = np.arange(N) + 0.5
        th = 1 - x / N
        for k in range(2, 400, 2):
            th -= 2 / (k * math.pi) * np.sin(k * math.pi * x / N) * math.exp(-alpha * (k * math.pi / N) ** 2 * t)
        errs.append(np.abs(T - th).max())
    assert errs[2] < 1e-3 and errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs


def test_advection_of_a_sine_wave():
    """Uniform flow u0 in a periodic box carries theta = 1/2 + A sin(k(x - u0 t))
    with amplitude decay exp(-alpha_eff k^2 t); alpha_eff includes the known
    -(tau_g - 1/2) u0^2 numerical diffusion of the linear D2Q5 equilibrium."""
    N, u0, alpha, A = 64, 0.05, 0.05, 0.1
    lat = O.lattice(N, 4, periodic_x=1, periodic_y=1, alpha=alpha, nu0=0.1, nu_min=0.1,
                    nu_max=0.1)
    o = O.Oracle(lat)
    k = 2 * math.pi / N
    x = np.arange(N) + 0.5
    T0 = 0.5 + A * np.sin(k * x)
    f = np.stack([O.feq(1.0, 1.0, u0, 0.0)] * (N * 4), axis=1).reshape(9, 4, N)
    g = np.stack([O.geq(t, u0, 0.0) for t in np.tile(T0, 4)], axis=1).reshape(5, 4, N)
    o.set_state(f, g)
    t = int(N / u0)  # one full period
    o.step(t)
    T = o.macros()["T"][0]
    c = np.sum((T - 0.5) * np.sin(k * (x - u0 * t))) * 2 / N
    s = np.sum((T - 0.5) * np.cos(k * (x - u0 * t))) * 2 / N
    taug = 3 * alpha + 0.5
    amp_expected = A * math.exp(-(alpha - (taug - 0.5) * u0 ** 2) * k * k * t)
    assert math.hypot(c, s) == pytest.approx(amp_expected, rel=2e-3)
    assert abs(math.atan2(s, c)) < 0.01  # phase error < 0.01 rad after one period


def test_mass_conservation_and_energy_balance():
    p = O.physics(24, n=0.7, Da=1e-2, Ra=1e4, Pr=5.0, eps=0.6)
    o = O.Oracle.from_physics(p)
    m0 = o.macros()["rho"].sum()
    w1 = 1 / 6
    o.step(300)
    for _ in range(5):
        f, g = o.state()
        T0 = g.sum()
        o.step(1)
        f1, g1 = o.state()
        # net wall flux: hot wall incoming g1 at i = 0, cold wall incoming g3 at i = N-1
        flux = (2 * g1[1, :, 0] - 2 * w1 * 1.0).sum() + (2 * g1[3, :, -1] - 2 * w1 * 0.0).sum()
        assert abs(g1.sum() - T0 - flux) < 1e-13
    assert abs(o.macros()["rho"].sum() - m0) / m0 < 1e-13


def test_rest_state_is_invariant():
    lat = O.lattice(12, 10, T_hot=0.5, T_cold=0.5, T_init=0.5, gbeta=1e-3, npow=0.6,
                    nu0=0.05, nu_min=0.005, nu_max=0.5, gamma_scale=1e3, eps=0.6,
                    K=20.0, Feps=0.3)
    o = O.Oracle(lat)
    f0, g0 = o.state()
    o.step(200)
    f1, g1 = o.state()
    # round-off only (the rest populations w_i are not exact binary fractions)
    assert np.abs(f1 - f0).max() < 1e-15 and np.abs(g1 - g0).max() < 1e-15
    m = o.macros()
    assert np.abs(m["ux"]).max() < 1e-15 and np.abs(m["uy"]).max() < 1e-15


def centro_asymmetry(o):
    U, V, th = o.fields()
    a = max(np.abs(U + U[::-1, ::-1]).max(), np.abs(V + V[::-1, ::-1]).max()) / np.abs(V).max()
    return a, np.abs(th - (1 - th[::-1, ::-1])).max()


def test_cavity_centro_symmetry_is_restored_with_resolution():
    """The continuum cavity problem is invariant under the 180-degree rotation
    with (U, V) -> -(U, V) and theta -> 1 - theta.  The flow update is exactly
    equivariant; the thermal equilibrium is not (its flux w T (1 + 3 e.u)
    advects the constant part of T through the D2Q5 stencil), so the asymmetry
    is a second-order discretisation error that shrinks ~4x per doubling of N
    at fixed physical parameters and time."""
    res = []
    for N in (16, 32):
        p = O.physics(N, n=0.8, Da=1e-1, Ra=1e4, Pr=2.0, eps=0.6, mach=0.1)
        o = O.Oracle.from_physics(p)
        o.step(int(round(1.0 * N / (0.1 / math.sqrt(3)))))
        res.append(centro_asymmetry(o))
    ratio_u = res[0][0] / res[1][0]
    ratio_t = res[0][1] / res[1][1]
    assert res[1][0] < 2e-3 and res[1][1] < 3e-3, res
    assert ratio_u > 2.8 and ratio_t > 2.8, res


def two_layer_brinkman(y, N, nu, eps, K1, K2, gx):
    """Closed form of nu u'' - eps nu u / K(y) + eps gx = 0 between no-slip
    walls at y = 0 and y = N, K = K1 below y = N/2 and K2 above: a cosh/sinh
    pair plus the Darcy value gx K / nu in each layer, with u and u'
    continuous at y = N/2."""
    r1, r2, h = math.sqrt(eps / K1), math.sqrt(eps / K2), N / 2
    d1, d2 = gx * K1 / nu, gx * K2 / nu
    # u1 = -d1 cosh(r1 y) + B1 sinh(r1 y) + d1; u2 = -d2 cosh(r2 z) + B2 sinh(r2 z) + d2, z = N - y
    A = np.array([[math.sinh(r1 * h), -math.sinh(r2 * h)],
                  [r1 * math.cosh(r1 * h), r2 * math.cosh(r2 * h)]])
    b = np.array([d1 * math.cosh(r1 * h) - d1 - d2 * math.cosh(r2 * h) + d2,
                  r1 * d1 * math.sinh(r1 * h) + r2 * d2 * math.sinh(r2 * h)])
    B1, B2 = np.linalg.solve(A, b)
    z = N - y
    u1 = -d1 * np.cosh(r1 * y) + B1 * np.sinh(r1 * y) + d1
    u2 = -d2 * np.cosh(r2 * z) + B2 * np.sinh(r2 * z) + d2
    return np.where(y < h, u1, u2)


def test_per_cell_permeability_uniform_plane_is_brinkman():
    """K(x) = 10^logDa(x) N^2 (Eq. 6, Da = K / L^2 with L = nx): a uniform
    per-cell log10(Da) plane reproduces the Brinkman channel's cosh closed form
    with K = Da nx^2 -- a dropped N^2, another base or a flipped sign of the
    exponent each moves K by a factor of at least 4."""
    errs = []
    for N in (16, 32, 64):
        nx, nu, eps, gx = 4, 0.1, 0.6, 1e-7
        K = (N / 8) ** 2
        lat = channel(N, nx=nx, nu0=nu, nu_min=nu, nu_max=nu, gx=gx, eps=eps, K=1e300)
        assert lat.K_scale == nx * nx
        logda = np.full((N, nx), math.log10(K / nx ** 2))
        o = O.Oracle(lat, logda=logda)
        o.step(int(3 * N * N / nu))
        y = np.arange(N) + 0.5
        r = math.sqrt(eps / K)
        ua = gx * K / nu * (1 - np.cosh(r * (y - N / 2)) / math.cosh(r * N / 2))
        ux = o.macros()["ux"]
        assert np.abs(ux - ux[:, :1]).max() <= 1e-12 * ua.max()  # uniform along the channel
        errs.append(np.abs(ux[:, 0] - ua).max() / ua.max())
    assert errs[2] < 2e-3 and errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs
    # the physical mapping uses the same scale: K_scale = nx^2 for the cavity
    assert O.map_physics(O.physics(48, 40, Da=1e-2)).K_scale == 48.0 ** 2


def test_per_cell_permeability_two_layers():
    """A two-layer log10(Da) plane (Da = 1/64 below mid-channel, 1/16 above):
    the profile converges to the piecewise cosh/sinh closed form, so each
    node takes the permeability of its own cell."""
    errs = []
    for N in (16, 32, 64):
        nx, nu, eps, gx = 2, 0.1, 0.6, 1e-7
        K1, K2 = (N / 8) ** 2, (N / 4) ** 2
        lat = channel(N, nx=nx, nu0=nu, nu_min=nu, nu_max=nu, gx=gx, eps=eps, K=1e300)
        logda = np.empty((N, nx))
        logda[: N // 2] = math.log10(K1 / nx ** 2)
        logda[N // 2:] = math.log10(K2 / nx ** 2)
        o = O.Oracle(lat, logda=logda)
        o.step(int(4 * N * N / nu))
        y = np.arange(N) + 0.5
        ua = two_layer_brinkman(y, N, nu, eps, K1, K2, gx)
        if N == 32:
            # the layers matter: either uniform permeability is far off
            for K in (K1, K2):
                r = math.sqrt(eps / K)
                uu = gx * K / nu * (1 - np.cosh(r * (y - N / 2)) / math.cosh(r * N / 2))
                assert np.abs(uu - ua).max() / ua.max() > 0.1
        errs.append(np.abs(o.macros()["ux"][:, 0] - ua).max() / ua.max())
    assert errs[2] < 3e-3 and errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs


def test_hot_and_cold_wall_nusselt_balance_at_steady_state():
    """At steady state the heat entering through the hot wall leaves through
    the cold wall, so Eq. (24) evaluated at either wall (the one-sided
    quadratic gradient through the wall value and the first two nodes) gives
    the same Nusselt number up to discretisation error, which shrinks with
    the grid.  Also: the oracle's Nu is Eq. (24) applied to its own fields."""
    out = []
    for N in (24, 32):
        o = O.Oracle.from_physics(O.physics(N, n=1.0, Da=1e-2, Ra=1e4, Pr=5.0, eps=0.6))
        r, _ = o.run_to_steady(tol=1e-12, check_every=1000, max_steps=200_000)
        assert r < 1e-12
        _, _, th = o.fields()
        hot = np.mean(N * (8.0 - 9.0 * th[:, 0] + th[:, 1]) / 3.0)
        cold = np.mean(N * (9.0 * th[:, -1] - th[:, -2]) / 3.0)
        assert o.nu_bar() == pytest.approx(hot, rel=1e-14)
        out.append(abs(hot - cold) / hot)
    assert out[0] < 1e-4 and out[1] < out[0] / 2, out
