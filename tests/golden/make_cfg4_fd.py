"""Writes tests/golden/cfg4_oracle_fd.json: central finite differences of the
hot-wall Nusselt number (Eq. 24) after 5000 steps, computed with the FP64
oracle only.

Workload: 256 x 256 porous cavity from rest, Pr = 10, eps = 0.6, Ra = 1e4,
per-cell log10(Da) field uniform on [-3, -1] (seed 0), J = Nu_bar after
T = 5000 steps.  Four variants:
  * "n1.0", "n1.4": n = 1.0 and 1.4 with the [0.1, 10] nu0 viscosity clamp;
  * "n0.7-clamp2":  n = 0.7 with a [0.1, 2] nu0 clamp;
  * "n0.7":         n = 0.7 with the [0.1, 10] nu0 clamp (the gradient
                    workload as stated).
Differences, each (J(p + h) - J(p - h)) / (2 h) in the parameter's units:
  * the 16 seeded probe cells (seed 1) of the log10(Da) field, h = 1e-2;
  * n and Ra, h = 1e-4 relative (h = 1e-4 * n, 1e-4 * Ra);
and, for "n0.7" only, a step-size study: n and Ra at relative h = 1e-2,
1e-3, 1e-4, the first two probe cells at h = 1e-2, 1e-3, 1e-4, and the
smooth whole-field direction w (seed 5) at h = 1e-2 and 1e-3.
Every J+ and J- is stored with its difference, so a reader can re-derive
any quotient.

Run from the repository root:
    python tests/golden/make_cfg4_fd.py [variant ...] [--procs P]
Each oracle run takes about 7 minutes on one core; runs go to P single-threaded
worker processes (default: the machine's CPU count).  Variants already in
the output file are kept; a variant is written as soon as it is complete.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
OUT = os.path.join(ROOT, "tests", "golden", "cfg4_oracle_fd.json")

N, T = 256, 5000
BASE = dict(Pr=10.0, eps=0.6, Ra=1e4)
VARIANTS = {
    "n1.0": dict(n=1.0),
    "n1.4": dict(n=1.4),
    "n0.7-clamp2": dict(n=0.7, nu_hi=2.0),
    "n0.7": dict(n=0.7),
}
H_CELL, H_REL = 1e-2, 1e-4
STUDY_H = (1e-2, 1e-3, 1e-4)
STUDY_DIR_H = (1e-2, 1e-3)


def _inputs():
    # the seeded generators, loaded by path (no package import, no GPU library)
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "pm_inputs", os.path.join(ROOT, "paper_2011_15073_amd", "inputs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def run_one(job):
    """One oracle run: (key, J) for the perturbation described by job."""
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import oracle as O
    inp = _inputs()
    key, variant, what, h = job
    phys = dict(BASE, **VARIANTS[variant])
    ld = inp.logda_field(N, seed=0)
    if what.startswith("cell:"):
        c = int(what[5:])
        j, i = divmod(c, N)
        ld = ld.copy()
        ld[j, i] += h
    elif what == "dir":
        ld = ld + h * inp.smooth_direction(N, seed=5)
    elif what == "n":
        phys["n"] = phys["n"] * (1.0 + h)
    elif what == "Ra":
        phys["Ra"] = phys["Ra"] * (1.0 + h)
    elif what != "base":
        raise ValueError(what)
    t0 = time.time()
    orc = O.Oracle.from_physics(O.physics(N, **phys), logda=ld)
    orc.step(T)
    return key, orc.nu_bar(), time.time() - t0


def jobs_for(variant, cells):
    """(key, variant, what, signed h) for every run of a variant."""
    out = [(f"{variant}|base|0", variant, "base", 0.0)]

    def pm(what, h):
        for s in (+1, -1):
            out.append((f"{variant}|{what}|{s * h:+.0e}", variant, what, s * h))

    for c in cells:
        pm(f"cell:{int(c)}", H_CELL)
    pm("n", H_REL)
    pm("Ra", H_REL)
    if variant == "n0.7":
        for h in STUDY_H:
            if h != H_REL:
                pm("n", h)
                pm("Ra", h)
            for c in cells[:2]:
                if h != H_CELL:
                    pm(f"cell:{int(c)}", h)
        for h in STUDY_DIR_H:
            pm("dir", h)
    return out


def summarise(variant, runs, cells):
    """Central differences from the J values of one variant."""
    def fd(what, h):
        jp, jm = runs[f"{variant}|{what}|{h:+.0e}"], runs[f"{variant}|{what}|{-h:+.0e}"]
        return dict(h=h, J_plus=jp, J_minus=jm, fd=(jp - jm) / (2.0 * h))

    phys = dict(BASE, **VARIANTS[variant])
    res = dict(params=dict(N=N, T=T, **phys), J=runs[f"{variant}|base|0"],
               cells=[int(c) for c in cells],
               cell_fd=[fd(f"cell:{int(c)}", H_CELL) for c in cells])
    # n and Ra perturbed relatively: divide by the absolute step as well
    for p in ("n", "Ra"):
        hs = [H_REL] + ([h for h in STUDY_H if h != H_REL] if variant == "n0.7" else [])
        entries = []
        for h in sorted(hs, reverse=True):
            e = fd(p, h)
            e["fd"] = e["fd"] / phys[p]
            e["h_abs"] = h * phys[p]
            entries.append(e)
        res[f"{p}_fd"] = entries
    if variant == "n0.7":
        res["cell_study"] = [[fd(f"cell:{int(c)}", h) for h in STUDY_H] for c in cells[:2]]
        res["dir_study"] = [fd("dir", h) for h in STUDY_DIR_H]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("variants", nargs="*", default=["n0.7", "n0.7-clamp2", "n1.0", "n1.4"])
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    inp = _inputs()
    cells = [int(c) for c in inp.fd_cells(N, seed=1, k=16)]
    data = {}
    if os.path.exists(a.out):
        with open(a.out) as fh:
            data = json.load(fh)
    data.setdefault("workload", "256x256 porous cavity from rest, Pr=10, eps=0.6, Ra=1e4, log10 Da ~ U[-3,-1] "
                                "(seed 0), J = Nu_bar (Eq. 24) after 5000 steps; FP64 oracle")
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=a.procs) as pool:
        for variant in a.variants:
            if variant in data.get("variants", {}):
                print(f"{variant}: already stored", flush=True)
                continue
            jobs = jobs_for(variant, cells)
            runs = {}
            for k, (key, J, dt) in enumerate(pool.map(run_one, jobs)):
                runs[key] = J
                print(f"  {variant} {k + 1}/{len(jobs)} {key}: J = {J:.15f} ({dt:.0f} s; {time.time() - t0:.0f} s)",
                      flush=True)
            data.setdefault("variants", {})[variant] = summarise(variant, runs, cells)
            with open(a.out + ".tmp", "w") as fh:
                json.dump(data, fh, indent=1)
            os.replace(a.out + ".tmp", a.out)
            print(f"{variant}: written to {a.out}", flush=True)


if __name__ == "__main__":
    main()
