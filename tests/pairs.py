"""Helpers that run the same configuration through the GPU library and the
oracle and measure the agreement (used by the GPU tests)."""
import numpy as np

import oracle as O

ORACLE_KEYS = {"n", "Da", "Ra", "Pr", "eps", "mach", "nu_lo", "nu_hi", "clamp_mode",
               "forchheimer", "s_e", "s_eps", "s_q", "sT_e", "sT_nu", "gx", "gy", "T_init",
               "periodic_x", "periodic_y"}


def oracle_for(nx, ny=None, logda=None, **kw):
    phys = {k: v for k, v in kw.items() if k in ORACLE_KEYS}
    return O.Oracle.from_physics(O.physics(nx, ny, **phys), logda=logda)


def gpu_for(nx, ny=None, dtype="fp64", logda=None, **kw):
    import paper_2011_15073_amd as P
    return P.Cavity(nx, ny, dtype=dtype, logda=logda, **kw)


def rel_err(a, b):
    """max |a - b| / max |b| (the field error measure)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def gpu_fields(cav):
    import torch
    return [t.cpu().numpy() for t in cav.fields(torch.float64)]


def compare_fields(cav, orc):
    Ug, Vg, Tg = gpu_fields(cav)
    Ur, Vr, Tr = orc.fields()
    return dict(U=rel_err(Ug, Ur), V=rel_err(Vg, Vr), theta=rel_err(Tg, Tr))


def compare_nu(cav, orc):
    a, b = cav.nu(), orc.nu_bar()
    return abs(a - b) / abs(b)
