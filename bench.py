"""Throughput benchmark of the fused lattice Boltzmann update on one MI355X.

Workload: the 4096 x 4096 porous cavity (FP32 storage and arithmetic, AA
pattern), power-law n = 0.8, Da = 1e-2, Ra = 1e5, Pr = 10, eps = 0.6, from
rest.  One step = one fused stream + collide of all nodes for both the D2Q9
flow and D2Q5 thermal populations; the reductions (hot-wall Nusselt number
and the max |dT| residual) run on device every 1000 steps, as in a
run-to-steady loop.  W untimed warm-up steps, then K timed steps between two
synchronisations.

Metric: MLUPS (million node updates per second, flow + thermal).  Also
reported, for the dominant kernel (the two-step kernel, which advances every
node by two steps per launch, at 4096^2 FP32):
  * roofline.achieved / frac: the kernel's algorithmic bytes per launch --
    one read and one write of the whole state, 112 B per node (9 + 5 FP32
    populations), for either step kernel -- over the HIP-event-timed launch,
    against the 8 TB/s HBM peak;
  * alg_equiv_GBps / alg_equiv_frac: the method's 112 B per node update times
    the 2 N^2 updates of a launch over the same time (the single-pass
    roofline of the method, which the two-step kernel can pass);
  * traffic / hbm_GBps / hbm_frac / copy_frac: the HBM bytes the kernel
    really moves per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, committed
    with a hash of the kernel code) over the launch time, against the peak
    and against the measured streaming-copy ceiling;
  * counters: VALU instructions per node update, the share of the CU's
    VALU issue rate they take and the share of wave time spent waiting
    (rocprofv3 SQ counters, committed with the same hash) -- what the kernel
    is bound by besides HBM;
and the other FP32 rounding mode, the adjoint/forward cost of the gradient
workload, a capped comparison of the 27-case sweep with sequential runs, and
the FP64 CPU oracle timed on a bounded sample of the same workload on this
host (all cores and one core), with its rates on the other parity workloads.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
       python bench.py --sweep | --adjoint | --paper-tables | --stream-function | --oracle-table
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 4096
PHYS = dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)
BYTES_PER_NODE = 112  # 14 FP32 populations, each read once and written once per step
HBM_PEAK_GBS = 8000.0
CHECK_EVERY = 1000
DEFAULT_ROUNDING = "stochastic"  # the library's default for FP32 (PM_ROUND_AUTO)
CSRC = os.path.join(ROOT, "paper_2011_15073_amd", "csrc")
# The step kernels the benchmark can time (--step-kernel; the default "auto"
# takes the two-step kernel at 4096^2), each with its committed counter
# summary and the code that decides what it computes and moves: the per-node
# device code and parameters (whole files), the kernel and its launcher, and
# the host's launch-shape choice.
KERNELS = {
    "pair": dict(
        name="k_step2 (two fused stream+collide steps per launch, LDS row rings)", steps_per_launch=2,
        traffic_file=os.path.join(ROOT, "profiles", "k_step2_fp32_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"// ---- two time steps in one pass.*?(?=// ---- )"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step2\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int pair_rows_for\(.*?\n}\n")]),
    "pair_sr": dict(
        name="k_step2 SR (two fused steps per launch, stochastically rounded updates)", steps_per_launch=2,
        traffic_file=os.path.join(ROOT, "profiles", "k_step2_fp32sr_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"// ---- two time steps in one pass.*?(?=// ---- )"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step2\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int pair_rows_for\(.*?\n}\n")]),
    "single_sr": dict(
        name="k_step SR (one fused stream+collide step per launch, stochastically rounded updates)",
        steps_per_launch=1,
        traffic_file=os.path.join(ROOT, "profiles", "k_step_fp32sr_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"void k_step\(KParams<T, S> p.*?\n}\n"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int step_width_for\(.*?\n}\n")]),
    "single_fp16": dict(
        name="k_step FP16 storage (one fused stream+collide step per launch, half-precision populations, "
             "FP32 arithmetic, stochastically rounded stores)", steps_per_launch=1,
        traffic_file=os.path.join(ROOT, "profiles", "k_step_fp16_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"void k_step\(KParams<T, S> p.*?\n}\n"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int step_width_for\(.*?\n}\n")]),
    "single_fp64": dict(
        name="k_step FP64 (one fused stream+collide step per launch, AA pattern in place)", steps_per_launch=1,
        traffic_file=os.path.join(ROOT, "profiles", "k_step_fp64_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"void k_step\(KParams<T, S> p.*?\n}\n"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int step_width_for\(.*?\n}\n")]),
    "single": dict(
        name="k_step (one fused stream+collide step per launch, AA pattern in place)", steps_per_launch=1,
        traffic_file=os.path.join(ROOT, "profiles", "k_step_fp32_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"void k_step\(KParams<T, S> p.*?\n}\n"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int step_width_for\(.*?\n}\n")]),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(kind="pair"):
    """sha256[:16] of a step kernel's code (KERNELS[kind]["srcs"]: whole
    files or the part a pattern selects), comments removed and runs of
    whitespace collapsed: editing a comment or another kernel keeps the
    committed counter summary, any change to this kernel's code orphans it."""
    h = hashlib.sha256()
    for src in KERNELS[kind]["srcs"]:
        path, pattern = src if isinstance(src, tuple) else (src, None)
        with open(path, encoding="utf-8") as fh:
            text = fh.read()
        if pattern is not None:
            m = re.search(pattern, text, flags=re.S)
            if m is None:
                raise RuntimeError(f"kernel_hash: {pattern!r} not found in {path}")
            text = m.group(0)
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def read_traffic(kind="pair"):
    """HBM bytes per launch of a step kernel from its committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when absent or taken on different kernel code."""
    path = KERNELS[kind]["traffic_file"]
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash(kind):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SQ_COUNTERS = os.path.join(ROOT, "profiles", "step_kernels_4096_sq_counters.txt")


def read_counters(kind="pair"):
    """VALU instructions per node update, VALU issue share and wait share of
    a step kernel from the committed SQ counter summary, or None when absent
    or taken on different kernel code (the summary records the code hash of
    each kernel family)."""
    if not os.path.exists(SQ_COUNTERS):
        return None
    family = "pair" if kind.startswith("pair") else "single"
    text = open(SQ_COUNTERS).read()
    m = re.search(r"bench\.kernel_hash\('%s'\) = ([0-9a-f]+)" % family, text)
    if m is None or m.group(1) != kernel_hash(kind):
        return None
    m = re.search(r"^%s: (.*)$" % re.escape(kind), text, flags=re.M)
    if m is None:
        return None
    vals = dict(kv.split(" = ") for kv in m.group(1).split(", "))
    try:
        return {"valu_per_node_update": float(vals["valu_per_node_update"]),
                "valu_issue_share": float(vals["valu_issue_share"]),
                "wait_share": float(vals["wait_share"])}
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_sample(budget_s):
    """Oracle MLUPS on the 4096^2 workload: one warm-up step, then as many
    steps as fit in about budget_s seconds (at least one)."""
    import oracle as O
    orc = O.Oracle.from_physics(O.physics(N, **PHYS))
    t0 = time.perf_counter()
    orc.step(1)
    per = time.perf_counter() - t0
    k = max(1, min(50, int(budget_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    orc.step(k)
    dt = time.perf_counter() - t0
    return N * N * k / dt / 1e6, k, dt


def cpu_baseline(budget_s=15.0, one_core=True):
    """The FP64 oracle on the same 4096^2 workload, on all the host's cores
    (OpenMP over rows), and on one core in a child process (one step, which
    takes about 20-30 s there)."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    mlups, k, dt = _oracle_sample(budget_s)
    out = {"value": round(mlups, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{k} steps of the 4096x4096 workload after 1 warm-up step, FP64, {dt:.1f} s, "
                     f"{threads} OpenMP threads"}
    if one_core:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        code = ("import sys, json; sys.path.insert(0, %r); import bench; "
                "m, k, dt = bench._oracle_sample(0.0); print(json.dumps([m, k, dt]))" % ROOT)
        try:
            r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                               timeout=300, check=True)
            m1, k1, dt1 = json.loads(r.stdout.strip().splitlines()[-1])
            out["value_1core"] = round(m1, 4)
            out["sample_1core"] = f"{k1} step(s) of the same workload after 1 warm-up step, 1 thread, {dt1:.1f} s"
        except (subprocess.SubprocessError, ValueError, IndexError) as e:
            out["value_1core"] = None
            out["sample_1core"] = f"not measured: {type(e).__name__}"
    return out


# The oracle's rate on each parity workload: (name, side, physics, log-Da
# field?, steps of the whole run, sampled steps on all cores, sampled steps on
# one core).  The steady-state run's 331 000 steps are the oracle's own stop
# (max|dT| over 1000 steps < 1e-8, tests/golden/cfg1_256_oracle.npz); the
# 27 sweep cases are sampled one after another and reported at 5000 steps each.
ORACLE_WORKLOADS = [
    ("64x64 Newtonian cavity, n=1 Da=0.1 Ra=1e3, 20000 steps", 64,
     dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6), False, 20000, 20000, 2000),
    ("256x256 power-law cavity to steady state, n=0.6 Da=1e-3 Ra=1e5, 331000 steps", 256,
     dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6), False, 331000, 1000, 100),
    ("27 sweep cases (sides 128-512), 5000 steps each", None, None, False, 5000, 60, 6),
    ("256x256 gradient workload forward, n=0.7 Ra=1e4, log10 Da ~ U[-3,-1], 5000 steps", 256,
     dict(n=0.7, Ra=1e4, Pr=10.0, eps=0.6), True, 5000, 500, 50),
]


def _oracle_rates(one_core):
    """Oracle MLUPS on each of ORACLE_WORKLOADS (sampled steps after one
    warm-up step per grid)."""
    import oracle as O
    from paper_2011_15073_amd import inputs
    out = []
    for name, side, phys, logda, full, s_all, s_one in ORACLE_WORKLOADS:
        k = s_one if one_core else s_all
        if side is None:
            runs = [(c["N"], dict(n=c["n"], Da=c["Da"], Ra=c["Ra"], Pr=10.0, eps=0.6), None)
                    for c in inputs.sweep_cases(0)]
        else:
            runs = [(side, phys, inputs.logda_field(side, seed=0) if logda else None)]
        upd, dt = 0, 0.0
        for nx, ph, ld in runs:
            orc = O.Oracle.from_physics(O.physics(nx, **ph), logda=ld)
            orc.step(1)
            t0 = time.perf_counter()
            orc.step(k)
            dt += time.perf_counter() - t0
            upd += nx * nx * k
        m = upd / dt / 1e6
        out.append(dict(workload=name, steps_sampled=k, seconds=round(dt, 2), mlups=round(m, 3),
                        est_full_run_s=round(upd / k * full / (m * 1e6), 1)))
    return out


def oracle_table():
    """The FP64 oracle's throughput on the parity workloads, on all the
    host's cores and on one core (a child process), with the wall time a
    whole run would take at that rate (about 25 s of CPU time in all)."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    log(f"oracle table: {threads} threads")
    rows = _oracle_rates(one_core=False)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, json; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench._oracle_rates(True)))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600, check=True)
    one = json.loads(r.stdout.strip().splitlines()[-1])
    for a, b in zip(rows, one):
        a["cores"] = threads
        a.update({k + "_1core": b[k] for k in ("steps_sampled", "seconds", "mlups", "est_full_run_s")})
        log(f"oracle table: {a['workload']}: {a['mlups']} MLUPS on {threads} threads, "
            f"{a['mlups_1core']} on one core")
    return rows, threads


def oracle_table_main(args):
    rows, threads = oracle_table()
    print(json.dumps({"metric": "oracle MLUPS", "unit": "MLUPS", "kind": "oracle", "dtype": "f64",
                      "cpu_model": cpu_model(), "cores": threads, "workloads": rows}), flush=True)


def sweep_main(args):
    """The 27-case (n, Da, Ra) sweep with seeded uneven grid sides: one batched
    sweep (tuned schedule, graph-replayed chunks) against the same cases run one
    after another with the single-case solver; cases/s for both, and a bitwise
    comparison of every case's final populations."""
    import torch
    import paper_2011_15073_amd as P
    from paper_2011_15073_amd import inputs

    dt = args.sweep_dtype
    cs = inputs.sweep_cases(0)
    cases = [dict(nx=c["N"], n=c["n"], Da=c["Da"], Ra=c["Ra"], Pr=10.0, eps=0.6, dtype=dt) for c in cs]
    log(f"sweep: {len(cases)} cases, sides {[c['N'] for c in cs]}, {dt}, tol {args.sweep_tol}")
    sched, times = P.tune(cases)
    log(f"sweep: schedule {sched} ({ {k: round(v, 1) for k, v in times.items()} } us/step)")
    sw = P.Sweep(cases, **sched)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, res = sw.run(tol=args.sweep_tol, check_every=1000, max_steps=args.sweep_cap,
                        progress=lambda nl, st: log(f"sweep: batched, {nl} live, max steps {max(st)}"))
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    nupd = sum(s_ * c["N"] ** 2 for s_, c in zip(steps, cs))
    log(f"sweep: batched {t_batched:.2f} s, {nupd / t_batched / 1e6:.0f} MLUPS")
    t_seq, same = 0.0, 0
    tdt = torch.float64 if dt == "fp64" else torch.float32
    for i, (kw, c) in enumerate(zip(cases, cs) if not args.sweep_no_sequential else []):
        kw = dict(kw)
        nx = kw.pop("nx")
        cav = P.Cavity(nx, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, st = cav.run_to_steady(tol=args.sweep_tol, check_every=1000, max_steps=args.sweep_cap)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        fa, ga = cav.populations(tdt)
        fb, gb = sw.case(i).populations(tdt)
        eq = st == steps[i] and torch.equal(fa, fb) and torch.equal(ga, gb)
        same += int(eq)
        log(f"sweep: case {i} N={c['N']} n={c['n']} Da={c['Da']:.0e} Ra={c['Ra']:.0e}: "
            f"{st} steps, r {r:.2e}, Nu {cav.nu():.6f}, bitwise equal {eq}")
        del cav
    print(json.dumps({
        "metric": "sweep cases/s", "value": round(len(cases) / t_batched, 4), "unit": "cases/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64" if dt == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "27-case sweep n in {0.6,0.8,1.0} x Da in {1e-3,1e-2,1e-1} x "
                               "Ra in {1e3,1e4,1e5}, eps=0.6, Pr=10, sides drawn from "
                               "{128,192,256,384,512} (seed 0)", "tol": args.sweep_tol,
                   "check_every": 1000, "max_steps": args.sweep_cap,
                   "schedule": {"order": sched["order"], "tile": list(sched["tile"])}},
        "batched_s": round(t_batched, 3), "sequential_s": round(t_seq, 3) if t_seq else None,
        "sequential_cases_per_s": round(len(cases) / t_seq, 4) if t_seq else None,
        "speedup_vs_sequential": round(t_seq / t_batched, 3) if t_seq else None,
        "node_updates": nupd, "batched_MLUPS": round(nupd / t_batched / 1e6, 1),
        "cases_bitwise_equal_to_sequential": f"{same}/{len(cases)}",
        "steps_per_case": steps}), flush=True)


# The paper's own runs and printed Nusselt numbers: its validation table
# (clear power-law fluid, Ra = 1e5, Pr = 100) and its parametric table
# (160 x 160, Pr = 6.2; n, Da and Ra varied in turn).  Read literally: the
# paper's equations have the Darcy term only, so eps = 1 and no Forchheimer
# term; the validation runs are a clear fluid (Da = inf).
PAPER_TABLES = os.path.join(ROOT, "tests", "golden", "paper_nu_tables.json")


PAPER_CLAMPS = {
    # the [0.1, 10] nu0 viscosity clamp of the 256^2 power-law workload
    "nu": dict(clamp_mode=0, nu_lo=0.1, nu_hi=10.0),
    # the paper's own modified power law, Eq. (21): gamma* clamped to [0.01, 1e6]
    "gamma": dict(clamp_mode=1, nu_lo=0.01, nu_hi=1e6),
}


def paper_cases(N, clamp="nu", mach=0.1):
    """(sweep case, label dict, paper Nu) for every row of both tables."""
    tab = json.load(open(PAPER_TABLES))
    extra = dict(PAPER_CLAMPS[clamp], mach=mach)
    out = []
    for r in tab["validation"]:
        out.append((dict(nx=N, n=r["n"], Ra=r["Ra"], Pr=r["Pr"], eps=1.0, forchheimer=0, dtype="fp64", **extra),
                    dict(table="validation", n=r["n"], Da=None, Ra=r["Ra"], Pr=r["Pr"]), r["nu"]))
    for r in tab["parametric"]:
        out.append((dict(nx=N, n=r["n"], Da=r["Da"], Ra=r["Ra"], Pr=r["Pr"], eps=1.0, forchheimer=0,
                         dtype="fp64", **extra),
                    dict(table="parametric", n=r["n"], Da=r["Da"], Ra=r["Ra"], Pr=r["Pr"]), r["nu"]))
    return out


def paper_main(args):
    """Both of the paper's tables run to steady state as one batched sweep
    (FP64, max|dT| over 1000 steps < tol); prints our Nu beside the paper's."""
    import torch
    import paper_2011_15073_amd as P

    N = args.paper_side
    rows_in = paper_cases(N, args.paper_clamp, args.paper_mach)
    cases = [c for c, _, _ in rows_in]
    sw = P.Sweep(cases)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, res = sw.run(tol=args.sweep_tol, check_every=1000, max_steps=args.sweep_cap,
                        progress=lambda nl, st: log(f"paper: {nl} live, max steps {max(st)}"))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rows = []
    for i, (_, par, nu_p) in enumerate(rows_in):
        nu = sw.case(i).nu()
        rows.append(dict(**par, steps=steps[i], residual=res[i], nu=round(nu, 6),
                         nu_paper=nu_p, rel_diff=round(nu / nu_p - 1.0, 4)))
        log(f"paper: {par}: Nu {nu:.6f} (paper {nu_p}), {steps[i]} steps, r {res[i]:.1e}")
    print(json.dumps({"metric": "paper tables: Nu", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"the paper's validation and parametric cases, {N}x{N}, "
                                             f"eps=1, Darcy drag only, Ma={args.paper_mach}, "
                                             f"viscosity clamp {args.paper_clamp} {PAPER_CLAMPS[args.paper_clamp]}",
                                 "tol": args.sweep_tol,
                                 "max_steps": args.sweep_cap},
                      "wall_s": round(wall, 2), "cases": rows}), flush=True)


def adjoint_main(args):
    """Cost of the gradient of Nu_bar on the 256 x 256 cavity (or --adjoint-side; FP32 forward
    state, FP64 adjoint, n = 0.7, Ra = 1e4, per-cell log10 Da ~ U[-3, -1]
    seed 0, T = 5000 steps, checkpoints every ceil(sqrt(T)) steps): forward
    with checkpoints vs backward (segment replay + adjoint steps).  With the
    [0.1, 10] viscosity clamp the exact adjoint of this workload grows without
    bound (low-shear regions amplify perturbations), so the gradient is taken
    with the shear floor gamma* = --adjoint-shear-floor; the work per step is
    the same either way.  --adjoint-lambda fp32 stores the adjoint state in
    FP32 between steps (FP64 arithmetic)."""
    import torch
    import paper_2011_15073_amd as P
    from paper_2011_15073_amd import inputs

    N, T = args.adjoint_side, args.adjoint_steps
    ld = torch.from_numpy(inputs.logda_field(N, seed=0))
    times = []
    for rep in range(2):
        cav = P.Cavity(N, dtype="fp32", logda=ld, n=0.7, Ra=1e4, Pr=10.0, eps=0.6)
        adj = P.Adjoint(cav, T, shear_floor=args.adjoint_shear_floor, lambda_dtype=args.adjoint_lambda)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = adj.forward()
        t1 = time.perf_counter()
        gld, gn, gRa = adj.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
        log(f"adjoint: rep {rep}: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s, J {J:.8f}")
        adj.close()
        del adj, cav
    fwd, bwd = times[-1]
    print(json.dumps({
        "metric": "adjoint/forward cost", "value": round(bwd / fwd, 3), "unit": "x",
        "n_gpus": 1, "higher_is_better": False,
        "dtype": "f32 forward / f64 adjoint" + (", f32 adjoint state" if args.adjoint_lambda == "fp32" else ""),
        "data": "synthetic",
        "config": {"workload": f"{N}x{N} porous cavity, n=0.7, Ra=1e4, Pr=10, eps=0.6, per-cell "
                               "log10 Da ~ U[-3,-1] (seed 0), J = Nu_bar after T steps",
                   "T": T, "checkpoint_every": math.ceil(math.sqrt(T)),
                   "shear_floor": args.adjoint_shear_floor},
        "forward_s": round(fwd, 4), "backward_s": round(bwd, 4), "J": J,
        "dJ_dn": gn, "dJ_dRa": gRa, "max_abs_dJ_dlogDa": float(gld.abs().max())}), flush=True)


def psi_main(args):
    """Stream function of the 4096^2 workload (FP32 state after the warm-up
    steps, FP64 psi): one pm_stream_function call = the porous-velocity field
    kernel (reads the 14 populations, writes U) and the three-pass blocked
    column scan.  Algorithmic bytes per node: 56 (populations) + 8 (U) + 8
    (U, block sums) + 16 (U read, psi written) = 88."""
    import torch
    import paper_2011_15073_amd as P

    cav = P.Cavity(N, dtype="fp32", device="cuda:0", **PHYS)
    cav.step(args.warmup)
    psi = cav.stream_function()
    torch.cuda.synchronize()
    reps = 20
    with torch.cuda.stream(cav.stream):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(cav.stream)
        for _ in range(reps):
            cav.stream_function(out=psi)
        e1.record(cav.stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    alg = 88 * N * N
    log(f"psi: {us:.1f} us per call, {alg / us / 1e3:.0f} GB/s algorithmic")
    print(json.dumps({
        "metric": "stream function time", "value": round(us, 2), "unit": "us", "n_gpus": 1,
        "higher_is_better": False, "dtype": "f32 state / f64 psi", "data": "synthetic",
        "config": {"workload": f"stream function of the porous power-law cavity {N}x{N} after "
                               f"{args.warmup} steps (n=0.8 Da=1e-2 Ra=1e5 Pr=10 eps=0.6)"},
        "roofline": {"bound": "hbm", "achieved": round(alg / us / 1e3, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(alg / us / 1e3 / 8000.0, 4), "traffic": None,
                     "algorithmic_bytes_per_call": alg}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-kernel", default="auto", choices=["auto", "single", "pair"],
                    help="step kernel of the cavity (auto: the two-step kernel at 4096^2)")
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64", "fp16"],
                    help="storage and arithmetic of the timed cavity (fp64: the single-step kernel, 224 B per "
                         "node update; fp16: half-precision population storage with FP32 arithmetic, the "
                         "single-step kernel, 56 B per node update)")
    ap.add_argument("--rounding", default=None, choices=["nearest", "stochastic"],
                    help="rounding of the FP32 population updates (PM_ROUND_*; default: the library's)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other rounding mode, the adjoint cost, the capped sweep and the oracle's "
                         "rates on the other parity workloads")
    ap.add_argument("--sweep-extra-cap", type=int, default=10000,
                    help="step cap of the capped 27-case sweep comparison in the default run")
    ap.add_argument("--roofline-steps", type=int, default=400)
    ap.add_argument("--side", type=int, default=N,
                    help="grid side of the timed cavity (default 4096, the benchmark workload; other sides "
                         "report no counter traffic and no CPU baseline)")
    ap.add_argument("--sweep", action="store_true",
                    help="run the 27-case batched-sweep benchmark instead")
    ap.add_argument("--sweep-dtype", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--sweep-tol", type=float, default=1e-8)
    ap.add_argument("--sweep-cap", type=int, default=3_000_000)
    ap.add_argument("--sweep-no-sequential", action="store_true",
                    help="time only the batched sweep (no sequential runs, no bitwise comparison)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="run the paper's validation and parametric cases and print Nu beside its values")
    ap.add_argument("--paper-side", type=int, default=160)
    ap.add_argument("--paper-clamp", default="gamma", choices=sorted(PAPER_CLAMPS),
                    help="viscosity bounds of the paper's runs: the [0.1, 10] nu0 clamp, or Eq. (21)'s shear-rate "
                         "thresholds 0.01 and 1e6")
    ap.add_argument("--paper-mach", type=float, default=0.05, help="lattice Mach number of the paper's runs")
    ap.add_argument("--stream-function", action="store_true",
                    help="time the stream function of the 4096^2 workload")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the gradient of Nu (forward with checkpoints vs backward)")
    ap.add_argument("--oracle-table", action="store_true",
                    help="time the FP64 CPU oracle on the parity workloads (all cores and one core); no GPU")
    ap.add_argument("--adjoint-steps", type=int, default=5000)
    ap.add_argument("--adjoint-side", type=int, default=256,
                    help="grid side of the adjoint benchmark (default 256, the gradient workload)")
    ap.add_argument("--adjoint-shear-floor", type=float, default=0.1,
                    help="nondimensional shear floor of the regularised adjoint (0: exact)")
    ap.add_argument("--adjoint-lambda", choices=("fp64", "fp32"), default="fp64",
                    help="storage of the adjoint state between steps (FP64 arithmetic either way)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the step is measured on one GPU's share of the grid; a multi-GPU slab split is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    if args.oracle_table:
        oracle_table_main(args)
        return
    if args.sweep:
        sweep_main(args)
        return
    if args.paper_tables:
        return paper_main(args)
    if args.adjoint:
        adjoint_main(args)
        return
    if args.stream_function:
        psi_main(args)
        return

    import torch
    import paper_2011_15073_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S, dt = args.side, args.dtype
    rounding = args.rounding or ("stochastic" if dt in ("fp32", "fp16") and DEFAULT_ROUNDING == "stochastic"
                                 else "nearest")
    kind, K = kernel_kind(P, S, dt, args.step_kernel, rounding)
    spl = K["steps_per_launch"]
    bpn = bytes_per_node(dt)
    log(f"bench: {S}x{S} {dt} {PHYS}, warmup {args.warmup}, steps {args.steps}, step kernel {args.step_kernel} "
        f"({K['name'].split()[0]}), rounding {rounding}")
    run = time_cavity(P, S, dt, rounding, args.step_kernel, args.warmup, args.steps, args.roofline_steps)
    mlups, ms_per_step, launch_s = run["mlups"], run["ms_per_step"], run["per_step_s"] * spl
    # algorithmic bytes of one launch of either step kernel: the launch reads
    # the whole state once and writes it once (the two-step kernel keeps its
    # intermediate step on chip), 112 B (FP32) / 224 B (FP64) / 56 B (FP16
    # storage) per node
    alg_launch = bpn * S * S
    achieved = alg_launch / launch_s / 1e9
    alg_equiv = bpn * S * S * spl / launch_s / 1e9  # the method's bytes per node update (112 B in FP32)
    log(f"bench: {K['name'].split()[0]} {launch_s * 1e6:.1f} us/launch, {achieved:.0f} GB/s kernel-algorithmic, "
        f"{alg_equiv:.0f} GB/s at {bpn} B per node update")
    copy_gbs = copy_ceiling(P, dev)
    log(f"bench: copy ceiling {copy_gbs:.0f} GB/s")

    # counters were taken at 4096^2 on the kernel code the hash names
    traffic = read_traffic(kind) if S == N else None
    hbm = traffic / launch_s / 1e9 if traffic else None
    result = {
        "metric": "MLUPS (flow+thermal)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dt == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"porous power-law cavity {S}x{S}, D2Q9 MRT + D2Q5 MRT, "
                               f"{dt.upper()} {'storage (FP32 arithmetic) ' if dt == 'fp16' else ''}"
                               "AA layout, n=0.8 Da=1e-2 Ra=1e5 Pr=10 eps=0.6, "
                               "Nu + residual on device every 1000 steps",
                   "nodes": S * S, "steps_timed": args.steps, "step_kernel": args.step_kernel,
                   "rounding": rounding},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "hbm_GBps": round(hbm, 1) if hbm else None,
                     "hbm_frac": round(hbm / HBM_PEAK_GBS, 4) if hbm else None,
                     "copy_frac": round(hbm / copy_gbs, 4) if hbm else None,
                     "counters": read_counters(kind),
                     "alg_equiv_GBps": round(alg_equiv, 1),
                     "alg_equiv_frac": round(alg_equiv / HBM_PEAK_GBS, 4),
                     "kernel": K["name"],
                     "steps_per_launch": spl,
                     "us_per_launch": round(launch_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": alg_launch,
                     "copy_ceiling_GBps": round(copy_gbs, 1)},
        "nu_bar": run["nu"],
    }
    del run
    torch.cuda.empty_cache()
    if dt in ("fp32", "fp16") and not args.no_extras:
        other = "nearest" if rounding == "stochastic" else "stochastic"
        kind_o, K_o = kernel_kind(P, S, dt, args.step_kernel, other)
        o = time_cavity(P, S, dt, other, args.step_kernel, args.warmup, args.steps, args.roofline_steps)
        result["other_rounding"] = {"rounding": other, "mlups": round(o["mlups"], 1),
                                    "ms_per_step": round(o["ms_per_step"], 5),
                                    "us_per_launch": round(o["per_step_s"] * K_o["steps_per_launch"] * 1e6, 2),
                                    "kernel": K_o["name"]}
        log(f"bench: {other} rounding: {o['mlups']:.1f} MLUPS")
        del o
        torch.cuda.empty_cache()
    if not args.no_extras:
        result["adjoint"] = adjoint_cost(P, 5000, args.adjoint_shear_floor)
        result["sweep_capped"] = sweep_capped(P, args.sweep_extra_cap)
    if not args.no_cpu_baseline and S == N:
        torch.cuda.empty_cache()
        log("bench: timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline()
        if not args.no_extras:
            try:
                result["cpu_baseline"]["workloads"] = oracle_table()[0]
            except Exception as e:  # a failed CPU sample must not cost the GPU line
                log(f"bench: oracle table not measured: {type(e).__name__}: {e}")
    print(json.dumps(result), flush=True)


def bytes_per_node(dt):
    """Algorithmic bytes per node update: 14 populations read once and written
    once, 4 B each in FP32, 8 B in FP64, 2 B with FP16 storage."""
    return {"fp32": BYTES_PER_NODE, "fp64": 2 * BYTES_PER_NODE, "fp16": BYTES_PER_NODE // 2}[dt]


def kernel_kind(P, S, dt, step_kernel, rounding):
    """The step kernel the library will run (only the two-step kernel needs a
    second population region) and its entry in KERNELS."""
    pair = (P.workspace_bytes(P.make_params(S, dtype=dt, step_kernel=step_kernel, **PHYS)) >
            P.workspace_bytes(P.make_params(S, dtype=dt, step_kernel="single", **PHYS)))
    kind = ("pair" if pair else "single") + {"fp64": "_fp64", "fp16": "_fp16"}.get(dt, "")
    if rounding == "stochastic" and kind + "_sr" in KERNELS:
        kind += "_sr"
    return kind, KERNELS[kind]


def time_cavity(P, S, dt, rounding, step_kernel, warmup, steps, roofline_steps):
    """The timed run: warm-up, then `steps` steps with the on-device Nu and
    residual every CHECK_EVERY steps between two synchronisations; then the
    step time from HIP events on the context's stream around
    roofline_steps steps (a multiple of 4: whole two-step pairs)."""
    import torch
    cav = P.Cavity(S, dtype=dt, device="cuda:0", step_kernel=step_kernel, rounding=rounding, **PHYS)
    stream = cav.stream
    cav.step(warmup)  # also builds the step graphs
    cav.nu()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left, nus = steps, []
    while left > 0:
        k = min(CHECK_EVERY, left)
        cav.step(k)
        left -= k
        if k == CHECK_EVERY:
            nus.append(cav.nu())
            cav.residual()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nu = nus[-1] if nus else cav.nu()
    log(f"bench: {rounding}: {S * S * steps / elapsed / 1e6:.1f} MLUPS, {elapsed * 1e3 / steps:.4f} ms/step, "
        f"Nu {nu:.6f}")
    rs = roofline_steps - roofline_steps % 4
    with torch.cuda.stream(stream):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cav.step(rs)
        e1.record(stream)
    e1.synchronize()
    out = {"mlups": S * S * steps / elapsed / 1e6, "ms_per_step": elapsed * 1e3 / steps, "nu": nu,
           "per_step_s": e0.elapsed_time(e1) / 1e3 / rs}
    del cav
    return out


def copy_ceiling(P, dev):
    """Streaming copy of 1 GiB (read + write) with the library's copy kernel."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream(dev)
    for _ in range(3):
        P.copy_probe(src, dst, stream)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        P.copy_probe(src, dst, stream)
    c1.record(stream)
    c1.synchronize()
    return 2 * nbytes * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9


def adjoint_cost(P, T, shear_floor):
    """The gradient workload (256^2, FP32 forward state, n = 0.7, Ra = 1e4,
    per-cell log10 Da seed 0, J = Nu_bar after T steps): backward (segment
    replays + adjoint steps) over forward (with checkpoints), wall clock,
    second of two repetitions; then once more with the adjoint state stored
    in FP32 between steps (pm_adjoint_set_lambda_dtype)."""
    import torch
    from paper_2011_15073_amd import inputs
    ld = torch.from_numpy(inputs.logda_field(256, seed=0))
    times = {}
    for lam in ("fp64", "fp64", "fp32"):
        cav = P.Cavity(256, dtype="fp32", logda=ld, n=0.7, Ra=1e4, Pr=10.0, eps=0.6)
        adj = P.Adjoint(cav, T, shear_floor=shear_floor, lambda_dtype=lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = adj.forward()
        t1 = time.perf_counter()
        adj.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times[lam] = (t1 - t0, t2 - t1)
        adj.close()
        del adj, cav
    (f64, b64), (f32, b32) = times["fp64"], times["fp32"]
    log(f"bench: adjoint {T} steps: forward {f64:.4f} s, backward {b64:.4f} s (FP32 adjoint state: {b32:.4f} s)")
    return {"adjoint_over_forward": round(b64 / f64, 3), "forward_s": round(f64, 4),
            "backward_s": round(b64, 4),
            "adjoint_over_forward_fp32_adjoint_state": round(b32 / f32, 3),
            "T": T, "J": J, "shear_floor": shear_floor,
            "workload": "256x256, n=0.7, Ra=1e4, Pr=10, eps=0.6, log10 Da ~ U[-3,-1] (seed 0), FP32 forward / "
                        "FP64 adjoint, checkpoints every ceil(sqrt(T)) steps"}


def sweep_capped(P, cap, dtype="fp64"):
    """The 27-case sweep with every case capped at `cap` steps (tol 1e-8,
    checks every 1000 steps; few cases stop before the cap): one batched
    sweep with the tuned schedule against the cases run one after another,
    wall clock, and whether every case ends bitwise equal."""
    import torch
    from paper_2011_15073_amd import inputs
    cs = inputs.sweep_cases(0)
    cases = [dict(nx=c["N"], n=c["n"], Da=c["Da"], Ra=c["Ra"], Pr=10.0, eps=0.6, dtype=dtype) for c in cs]
    sched, _ = P.tune(cases)
    sw = P.Sweep(cases, **sched)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, _ = sw.run(tol=1e-8, check_every=1000, max_steps=cap)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    t_s, same = 0.0, 0
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    for i, kw in enumerate(cases):
        kw = dict(kw)
        cav = P.Cavity(kw.pop("nx"), **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, st = cav.run_to_steady(tol=1e-8, check_every=1000, max_steps=cap)
        torch.cuda.synchronize()
        t_s += time.perf_counter() - t0
        fa, ga = cav.populations(tdt)
        fb, gb = sw.case(i).populations(tdt)
        same += int(st == steps[i] and torch.equal(fa, fb) and torch.equal(ga, gb))
        del cav
    sw.close()
    log(f"bench: sweep capped at {cap}: batched {t_b:.2f} s, sequential {t_s:.2f} s, {same}/27 bitwise")
    nupd = sum(st * c["N"] ** 2 for st, c in zip(steps, cs))
    return {"speedup_vs_sequential": round(t_s / t_b, 3), "batched_s": round(t_b, 3),
            "sequential_s": round(t_s, 3), "batched_MLUPS": round(nupd / t_b / 1e6, 1),
            "cases_per_s": round(len(cases) / t_b, 2), "sequential_cases_per_s": round(len(cases) / t_s, 2),
            "cases_bitwise_equal": f"{same}/{len(cases)}", "cap": cap, "dtype": dtype,
            "schedule": {"order": sched["order"], "tile": list(sched["tile"])},
            "workload": "27 cases n x Da x Ra, eps=0.6, Pr=10, sides from {128,...,512} (seed 0), "
                        f"tol 1e-8 every 1000 steps, capped at {cap} steps"}


if __name__ == "__main__":
    main()
