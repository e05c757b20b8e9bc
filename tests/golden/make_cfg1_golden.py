"""Writes tests/golden/cfg1_256_oracle.npz with the FP64 oracle only.

Workload: 256 x 256 porous cavity, modified power law n = 0.6 with the
viscosity clamped to [0.1, 10] nu0, Da = 1e-3, Ra = 1e5, Pr = 10, eps = 0.6,
from rest, run until max |dT| over 1000 steps < 1e-8 (checked every 1000
steps).  Stored: the stopping step S*, the final residual, the hot-wall
Nusselt number (Eq. 24), max |U|, max |V| over the whole field, the
nondimensional fields U, V, theta at every node (FP64), and, as before,
U, V, theta on every 4th node in each direction and on the two hot-wall
columns.

Run from the repository root:  python tests/golden/make_cfg1_golden.py [out.npz]
(about 85 minutes on 8 threads; the default output is the path above).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402

PHYS = dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6, nu_lo=0.1, nu_hi=10.0)
N = 256


def main():
    t0 = time.time()
    orc = O.Oracle.from_physics(O.physics(N, **PHYS))
    # run_to_steady in slices of 20 000 steps: each slice takes its first
    # snapshot at its start, which is the previous 1000-step check, so the
    # stopping step is that of one long call; a line per slice shows progress
    steps, r = 0, float("inf")
    while steps < 2_000_000:
        r, done = orc.run_to_steady(tol=1e-8, check_every=1000, max_steps=20_000)
        steps += done
        print(f"  {steps} steps, residual {r:.3e}, {time.time() - t0:.0f} s", flush=True)
        if r < 1e-8 or r != r or done < 20_000:
            break
    U, V, th = orc.fields()
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "tests", "golden", "cfg1_256_oracle.npz")
    np.savez_compressed(out, steps=steps, residual=r, nu_bar=orc.nu_bar(),
                        maxU=np.abs(U).max(), maxV=np.abs(V).max(), maxT=np.abs(th).max(),
                        U=U, V=V, T=th,
                        U4=U[::4, ::4], V4=V[::4, ::4], T4=th[::4, ::4],
                        Uw=U[:, :2], Vw=V[:, :2], Tw=th[:, :2],
                        phys=np.array(str(PHYS)))
    print(f"S* = {steps}, r = {r:.3e}, Nu = {orc.nu_bar():.12f}, {time.time() - t0:.0f} s -> {out}")


if __name__ == "__main__":
    main()
