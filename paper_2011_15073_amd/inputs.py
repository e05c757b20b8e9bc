"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Random draws only -- none of the method's arithmetic lives here.

Recipes (numpy.random.default_rng):
  * sweep grid sides: rng(seed).choice([128, 192, 256, 384, 512], 27), one
    per case in itertools.product(n, Da, Ra) order;
  * per-cell log10(Da) field: rng(seed).uniform(-3, -1, (N, N)), float64;
  * finite-difference probe cells: rng(seed + 1).choice(N*N, 16, replace=False);
  * smooth perturbation direction of the log10(Da) field: rng(seed) normal
    coefficients of cos(pi a x) cos(pi b y), a, b in 0..2;
  * random population states (parity tests): rest weights times
    (1 + amp * standard normal), thermal weights times (T0 + amp_T * normal);
  * uniform population states: one such draw of the 9 + 5 populations,
    repeated at every node.
"""
import itertools

import numpy as np

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W5 = np.array([1 / 3] + [1 / 6] * 4)

SWEEP_N = (0.6, 0.8, 1.0)
SWEEP_DA = (1e-3, 1e-2, 1e-1)
SWEEP_RA = (1e3, 1e4, 1e5)
SWEEP_SIDES = (128, 192, 256, 384, 512)


def sweep_cases(seed=0):
    """The 27 (n, Da, Ra, N) cases of the parameter sweep."""
    rng = np.random.default_rng(seed)
    sides = rng.choice(SWEEP_SIDES, 27)
    combos = list(itertools.product(SWEEP_N, SWEEP_DA, SWEEP_RA))
    return [dict(n=n, Da=da, Ra=ra, N=int(s)) for (n, da, ra), s in zip(combos, sides)]


def logda_field(N, seed=0, lo=-3.0, hi=-1.0):
    return np.random.default_rng(seed).uniform(lo, hi, (N, N))


def fd_cells(N, seed=1, k=16):
    return np.random.default_rng(seed).choice(N * N, k, replace=False)


def random_state(nx, ny, seed, amp=0.05, T0=0.5, amp_T=0.2):
    """Random pre-collision populations f [9, ny, nx], g [5, ny, nx]."""
    rng = np.random.default_rng(seed)
    f = W9[:, None, None] * (1 + amp * rng.standard_normal((9, ny, nx)))
    g = W5[:, None, None] * (T0 + amp_T * rng.standard_normal((5, ny, nx)))
    return f, g


def smooth_direction(N, seed=5):
    """A smooth whole-field perturbation direction [N, N] for directional
    finite differences of the log10(Da) field: the nine products
    cos(pi a x) cos(pi b y), a, b in 0..2, x = i / N, y = j / N, with standard
    normal coefficients drawn in (a, b) row-major order."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:N, 0:N] / N
    w = np.zeros((N, N))
    for a in range(3):
        for b in range(3):
            w = w + rng.standard_normal() * np.cos(np.pi * a * x) * np.cos(np.pi * b * y)
    return w


def uniform_state(nx, ny, seed, amp=0.03, T0=0.5, amp_T=0.2):
    """One random node state (as random_state draws it) repeated at every
    node: f [9, ny, nx], g [5, ny, nx]."""
    rng = np.random.default_rng(seed)
    f = W9 * (1 + amp * rng.standard_normal(9))
    g = W5 * (T0 + amp_T * rng.standard_normal(5))
    return (np.repeat(np.repeat(f[:, None, None], ny, 1), nx, 2),
            np.repeat(np.repeat(g[:, None, None], ny, 1), nx, 2))
