"""Writes tests/golden/cfg4_tangent_growth.json: growth of a perturbation of the
state under the linearised update (the tangent-linear model), on the CPU, with
the oracle package only.

Workload: the 256 x 256 gradient workload (porous cavity from rest, Pr = 10,
eps = 0.6, Ra = 1e4, n = 0.7, per-cell log10(Da) field uniform on [-3, -1],
seed 0), with the [0.1, 10] nu0 viscosity clamp and, as a control, the
[0.1, 2] clamp.  The FP64 C oracle runs 4900 steps from rest; from that
state, forward-mode differentiation (torch.func.jvp) of the torch
re-implementation of the update carries a random unit perturbation of all
14 population planes (standard normal, seed 3, scaled to max-norm 1) through
100 more steps.  Stored per step: the max-norm and the 2-norm of the
perturbation, and where the max-norm sits.

Run from the repository root:  python tests/golden/make_cfg4_tangent.py
(about ten minutes per clamp on one core).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "cfg4_tangent_growth.json")
N, T0, K = 256, 4900, 100
BASE = dict(n=0.7, Ra=1e4, Pr=10.0, eps=0.6)


def inputs():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "pm_inputs", os.path.join(ROOT, "paper_2011_15073_amd", "inputs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def growth(nu_hi):
    import torch
    from torch.func import jvp
    import oracle as O
    from oracle import torch_step as TS
    inp = inputs()
    ld = inp.logda_field(N, seed=0)
    t0 = time.time()
    orc = O.Oracle.from_physics(O.physics(N, nu_hi=nu_hi, **BASE), logda=ld)
    orc.step(T0)
    f, g = orc.state()
    print(f"  nu_hi {nu_hi}: oracle at step {T0} ({time.time() - t0:.0f} s)", flush=True)
    P = TS.Params(N, N, nu_hi=nu_hi, **BASE)
    ldt = torch.from_numpy(ld)
    f, g = torch.from_numpy(f), torch.from_numpy(g)
    rng = np.random.default_rng(3)
    tf = torch.from_numpy(rng.standard_normal((9, N, N)))
    tg = torch.from_numpy(rng.standard_normal((5, N, N)))
    scale = max(float(tf.abs().max()), float(tg.abs().max()))
    tf, tg = tf / scale, tg / scale
    out = []
    for k in range(1, K + 1):
        (f, g), (tf, tg) = jvp(lambda a, b: TS.step(P, a, b, ldt), (f, g), (tf, tg))
        t = torch.cat([tf, tg])
        amax = int(t.abs().argmax())
        q, rem = divmod(amax, N * N)
        j, i = divmod(rem, N)
        out.append(dict(step=T0 + k, max_norm=float(t.abs().max()), two_norm=float(t.norm()),
                        argmax=dict(q=q, i=i, j=j, logDa=float(ld[j, i]))))
        if k % 10 == 0:
            print(f"  nu_hi {nu_hi}: step {T0 + k}: max|d| {out[-1]['max_norm']:.3e}, "
                  f"|d|_2 {out[-1]['two_norm']:.3e} ({time.time() - t0:.0f} s)", flush=True)
    return out


def main():
    data = dict(workload=f"{N}x{N} porous cavity, n=0.7, Ra=1e4, Pr=10, eps=0.6, log10 Da ~ U[-3,-1] (seed 0); "
                         f"oracle to step {T0}, then the tangent-linear model of the torch re-implementation "
                         f"for {K} steps from a random unit perturbation (seed 3)",
                initial=dict(max_norm=1.0), runs={})
    for nu_hi in (10.0, 2.0):
        data["runs"][f"clamp_0.1_{nu_hi:g}"] = growth(nu_hi)
        with open(OUT + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(OUT + ".tmp", OUT)
    print(f"written {OUT}", flush=True)


if __name__ == "__main__":
    main()
