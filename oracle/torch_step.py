"""Differentiable FP64 CPU re-implementation of the update in PyTorch, used as
the reference for the hand-written adjoint.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the tests use it to
check the GPU adjoint step against autograd.  It is written from the same
steps of the method as the C oracle (the paper's Eqs. (12)-(24) with the
readings documented there) but vectorised over all nodes with closed-form
moments, and is itself checked against the C oracle to round-off.  It shares
no code with the GPU library.

State layout: f [9, ny, nx], g [5, ny, nx] (pre-collision, absolute values),
velocity order of Eq. (14).  Parameters that can carry gradients: the per-cell
log10(Da) field, the power-law index n and the Rayleigh number Ra.
"""
import math

import torch

EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
W9 = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
W5 = [1 / 3] + [1 / 6] * 4

# moment basis (rho, e, eps, jx, qx, jy, qy, pxx, pxy) and its row norms
M9 = torch.tensor([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=torch.float64)
N5 = torch.tensor([[1, 1, 1, 1, 1], [0, 1, 0, -1, 0], [0, 0, 1, 0, -1], [-4, 1, 1, 1, 1],
                   [0, 1, -1, 1, -1]], dtype=torch.float64)


class Params:
    """Physical parameters (Step 0 mapping done here, in torch, so that n and
    Ra can carry gradients)."""

    def __init__(self, nx, ny, n, Ra, Pr=10.0, eps=0.6, Da=math.inf, mach=0.1, nu_lo=0.1,
                 nu_hi=10.0, forchheimer=True, s_e=1.4, s_eps=1.4, s_q=1.2, sT_e=1.0, sT_nu=1.0):
        self.nx, self.ny = nx, ny
        self.n = torch.as_tensor(n, dtype=torch.float64)
        self.Ra = torch.as_tensor(Ra, dtype=torch.float64)
        self.Pr, self.eps, self.Da = Pr, eps, Da
        self.U = mach / math.sqrt(3.0)
        self.nu_lo, self.nu_hi = nu_lo, nu_hi
        self.Feps = 1.75 / math.sqrt(150 * eps ** 3) if forchheimer else 0.0
        self.s_e, self.s_eps, self.s_q, self.sT_e, self.sT_nu = s_e, s_eps, s_q, sT_e, sT_nu

    def lattice(self):
        N = float(self.nx)
        nu0 = self.Pr / torch.sqrt(self.Ra) ** (2.0 - self.n) * self.U * N
        alpha = self.U * N / torch.sqrt(self.Ra)
        return dict(nu0=nu0, alpha=alpha, gbeta=self.Pr * self.U ** 2 / N, gscale=N / self.U,
                    Kscale=N * N)


def _viscosity(P, L, A, B):
    """nu = clamp(nu0 (gscale sqrt(A + B s^2))^(n-1), lo nu0, hi nu0),
    s = 1/(3 nu + 1/2): Newton's method in y = ln nu on the unclamped
    equation, safeguarded by bisection inside [ln(lo nu0), ln(hi nu0)]."""
    n, nu0 = P.n, L["nu0"]
    lo = torch.log(P.nu_lo * nu0) * torch.ones_like(A)
    hi = torch.log(P.nu_hi * nu0) * torch.ones_like(A)

    def G(y):
        nu = torch.exp(y)
        s = 1.0 / (3.0 * nu + 0.5)
        g2 = A + B * s * s
        Gy = y - torch.log(nu0) - (n - 1.0) * (math.log(L["gscale"]) + 0.5 * torch.log(g2))
        dG = 1.0 - (n - 1.0) * 0.5 * (2.0 * B * s * (-3.0 * nu * s * s)) / g2
        return Gy, dG

    Glo, _ = G(lo)
    Ghi, _ = G(hi)
    y = 0.5 * (lo + hi)
    a, b = lo, hi
    for _ in range(80):
        Gy, dG = G(y)
        a = torch.where(Gy < 0, y, a)
        b = torch.where(Gy < 0, b, y)
        yn = y - Gy / dG
        ok = (yn >= a) & (yn <= b)  # closed bracket: an exact root stays put
        y = torch.where(ok, yn, 0.5 * (a + b))
    y = torch.where(Glo >= 0, lo, torch.where(Ghi <= 0, hi, y))
    return torch.exp(y)


def collide(P, f, g, logda=None):
    """Steps 2-9 at every node; returns post-collision f*, g*."""
    L = P.lattice()
    eps, ex, ey = P.eps, torch.tensor(EX, dtype=torch.float64), torch.tensor(EY, dtype=torch.float64)
    rho = f.sum(0)
    jx = torch.einsum("q,qji->ji", ex, f)
    jy = torch.einsum("q,qji->ji", ey, f)
    T = g.sum(0)
    Gx = torch.zeros_like(T)
    Gy = L["gbeta"] * (T - 0.5)
    vx = jx / rho + 0.5 * eps * Gx
    vy = jy / rho + 0.5 * eps * Gy
    m = torch.einsum("kq,qji->kji", M9, f)
    v2 = vx * vx + vy * vy
    e_neq = m[1] - (-2 * rho + 3 * rho * v2 / eps)
    p_neq = m[7] - rho * (vx * vx - vy * vy) / eps
    q_neq = m[8] - rho * vx * vy / eps
    A = P.s_e ** 2 * e_neq ** 2 / (4 * rho ** 2)
    B = 9 * (p_neq ** 2 + 4 * q_neq ** 2) / (4 * rho ** 2)
    if not P.n.requires_grad and float(P.n) == 1.0:
        nu = L["nu0"] * torch.ones_like(rho)
    else:
        nu = _viscosity(P, L, A, B)
    if logda is not None:
        invK = 10.0 ** (-logda) / L["Kscale"]
    elif math.isinf(P.Da):
        invK = torch.zeros_like(rho)
    else:
        invK = torch.full_like(rho, 1.0 / (P.Da * L["Kscale"]))
    invsK = torch.sqrt(invK)
    c0 = 0.5 * (1 + 0.5 * eps * nu * invK)
    c1 = 0.5 * eps * P.Feps * invsK
    den = c0 + torch.sqrt(c0 * c0 + c1 * torch.sqrt(v2))
    ux, uy = vx / den, vy / den
    um = torch.sqrt(ux * ux + uy * uy)
    Fx = -eps * nu * invK * ux - eps * P.Feps * invsK * um * ux + eps * Gx
    Fy = -eps * nu * invK * uy - eps * P.Feps * invsK * um * uy + eps * Gy
    uu = ux * ux + uy * uy
    uF = ux * Fx + uy * Fy
    meq = torch.stack([rho, -2 * rho + 3 * rho * uu / eps, rho - 3 * rho * uu / eps, rho * ux, -rho * ux,
                       rho * uy, -rho * uy, rho * (ux * ux - uy * uy) / eps, rho * ux * uy / eps])
    Fm = rho * torch.stack([torch.zeros_like(rho), 6 * uF / eps, -6 * uF / eps, Fx, -Fx, Fy, -Fy,
                            2 * (ux * Fx - uy * Fy) / eps, (ux * Fy + uy * Fx) / eps])
    snu = 1.0 / (3 * nu + 0.5)
    one = torch.ones_like(rho)
    S = torch.stack([one, P.s_e * one, P.s_eps * one, one, P.s_q * one, one, P.s_q * one, snu, snu])
    ms = m - S * (m - meq) + (1 - 0.5 * S) * Fm
    D = torch.tensor([9, 36, 36, 6, 12, 6, 12, 4, 4], dtype=torch.float64)
    fo = torch.einsum("kq,kji->qji", M9, ms / D[:, None, None])
    # thermal
    nT = torch.einsum("kq,qji->kji", N5, g)
    sg = 1.0 / (3 * L["alpha"] + 0.5)
    neq = torch.stack([T, ux * T, uy * T, -2 * T / 3, torch.zeros_like(T)])
    ST = torch.stack([one, sg * one, sg * one, P.sT_e * one, P.sT_nu * one])
    ns = nT - ST * (nT - neq)
    D5 = torch.tensor([5, 2, 2, 20, 4], dtype=torch.float64)
    go = torch.einsum("kq,kji->qji", N5, ns / D5[:, None, None])
    return fo, go, dict(rho=rho, ux=ux, uy=uy, T=T, nu=nu)


def stream(P, fo, go, T_hot=1.0, T_cold=0.0):
    """Streaming with halfway bounce-back (flow), anti-bounce-back at x = 0, nx
    and bounce-back at y = 0, ny (thermal); cavity walls on every side."""
    ny, nx = P.ny, P.nx
    f = []
    for q in range(9):
        src = torch.roll(fo[q], shifts=(EY[q], EX[q]), dims=(0, 1))
        mask = torch.ones(ny, nx, dtype=torch.bool)
        if EX[q] == 1:
            mask[:, 0] = False
        if EX[q] == -1:
            mask[:, -1] = False
        if EY[q] == 1:
            mask[0, :] = False
        if EY[q] == -1:
            mask[-1, :] = False
        f.append(torch.where(mask, src, fo[OPP[q]]))
    g = []
    for q in range(5):
        src = torch.roll(go[q], shifts=(EY[q], EX[q]), dims=(0, 1))
        out = go[OPP[q]]
        if q == 1:  # incoming across x = 0 (hot)
            mask = torch.ones(ny, nx, dtype=torch.bool)
            mask[:, 0] = False
            out = -go[3] + 2 * W5[1] * T_hot
        elif q == 3:  # incoming across x = nx (cold)
            mask = torch.ones(ny, nx, dtype=torch.bool)
            mask[:, -1] = False
            out = -go[1] + 2 * W5[3] * T_cold
        else:
            mask = torch.ones(ny, nx, dtype=torch.bool)
            if EY[q] == 1:
                mask[0, :] = False
            if EY[q] == -1:
                mask[-1, :] = False
        g.append(torch.where(mask, src, out))
    return torch.stack(f), torch.stack(g)


def step(P, f, g, logda=None):
    fo, go, _ = collide(P, f, g, logda)
    return stream(P, fo, go)


def rest_state(P, T_init=0.5):
    f = torch.tensor(W9, dtype=torch.float64)[:, None, None].expand(9, P.ny, P.nx).clone()
    g = (torch.tensor(W5, dtype=torch.float64) * T_init)[:, None, None].expand(5, P.ny, P.nx).clone()
    return f, g


def nu_bar(P, g):
    """Eq. (24) with the one-sided quadratic wall gradient (theta_w = 1)."""
    T = g.sum(0)
    return (P.nx * (8.0 - 9.0 * T[:, 0] + T[:, 1]) / 3.0).mean()
