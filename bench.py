"""Throughput benchmark of the fused lattice Boltzmann update on one MI355X.

Workload: the 4096 x 4096 porous cavity (FP32 storage and arithmetic, AA
pattern), power-law n = 0.8, Da = 1e-2, Ra = 1e5, Pr = 10, eps = 0.6, from
rest.  One step = one fused stream + collide of all nodes for both the D2Q9
flow and D2Q5 thermal populations; the reductions (hot-wall Nusselt number
and the max |dT| residual) run on device every 1000 steps, as in a
run-to-steady loop.  W untimed warm-up steps, then K timed steps between two
synchronisations.

Metric: MLUPS (million node updates per second, flow + thermal).  Also
reported: the roofline of the dominant kernel -- the two-step kernel, which
advances every node by two steps per launch -- from HIP-event-timed launches
against the 8 TB/s HBM peak, with 112 algorithmic bytes per node update (9 +
5 FP32 populations read once and written once per step) times the 2 N^2
updates of a launch; the kernel keeps the intermediate step on chip, so it
moves about half of those bytes (see `traffic`).  Also the measured ceiling
of a plain streaming copy, and the FP64 CPU oracle timed on a bounded sample
of the same workload on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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
    "single_fp64": dict(
        name="k_step FP64 (one fused stream+collide step per launch, AA pattern in place)", steps_per_launch=1,
        traffic_file=os.path.join(ROOT, "profiles", "k_step_fp64_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"void k_step\(KParams<T> p.*?\n}\n"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"hipError_t launch_step\(.*?\n}\n"),
              (os.path.join(CSRC, "pm_api.hip"), r"int step_width_for\(.*?\n}\n")]),
    "single": dict(
        name="k_step (one fused stream+collide step per launch, AA pattern in place)", steps_per_launch=1,
        traffic_file=os.path.join(ROOT, "profiles", "k_step_fp32_4096_traffic.txt"),
        srcs=[os.path.join(CSRC, "pm_device.h"), os.path.join(CSRC, "pm_internal.h"),
              (os.path.join(CSRC, "pm_kernels.hip"), r"void k_step\(KParams<T> p.*?\n}\n"),
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


def cpu_baseline(budget_s=15.0):
    """The FP64 oracle on the same 4096^2 workload: one warm-up step, then as
    many steps as fit in about budget_s seconds (at least one)."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    orc = O.Oracle.from_physics(O.physics(N, **PHYS))
    t0 = time.perf_counter()
    orc.step(1)
    t1 = time.perf_counter()
    per = t1 - t0
    k = max(1, min(50, int(budget_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    orc.step(k)
    dt = time.perf_counter() - t0
    del orc
    return {"value": round(N * N * k / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{k} steps of the 4096x4096 workload after 1 warm-up step, FP64, "
                      f"{dt:.1f} s"}


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
    for i, (kw, c) in enumerate(zip(cases, cs)):
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
        "batched_s": round(t_batched, 3), "sequential_s": round(t_seq, 3),
        "sequential_cases_per_s": round(len(cases) / t_seq, 4),
        "speedup_vs_sequential": round(t_seq / t_batched, 3),
        "node_updates": nupd, "batched_MLUPS": round(nupd / t_batched / 1e6, 1),
        "cases_bitwise_equal_to_sequential": f"{same}/{len(cases)}",
        "steps_per_case": steps}), flush=True)


# The paper's own runs and printed Nusselt numbers: its validation table
# (clear power-law fluid, Ra = 1e5, Pr = 100) and its parametric table
# (160 x 160, Pr = 6.2; n, Da and Ra varied in turn).  Read literally: the
# paper's equations have the Darcy term only, so eps = 1 and no Forchheimer
# term; the validation runs are a clear fluid (Da = inf).
PAPER_TABLES = os.path.join(ROOT, "tests", "golden", "paper_nu_tables.json")


def paper_cases(N):
    """(sweep case, label dict, paper Nu) for every row of both tables."""
    tab = json.load(open(PAPER_TABLES))
    out = []
    for r in tab["validation"]:
        out.append((dict(nx=N, n=r["n"], Ra=r["Ra"], Pr=r["Pr"], eps=1.0, forchheimer=0, dtype="fp64"),
                    dict(table="validation", n=r["n"], Da=None, Ra=r["Ra"], Pr=r["Pr"]), r["nu"]))
    for r in tab["parametric"]:
        out.append((dict(nx=N, n=r["n"], Da=r["Da"], Ra=r["Ra"], Pr=r["Pr"], eps=1.0, forchheimer=0,
                         dtype="fp64"),
                    dict(table="parametric", n=r["n"], Da=r["Da"], Ra=r["Ra"], Pr=r["Pr"]), r["nu"]))
    return out


def paper_main(args):
    """Both of the paper's tables run to steady state as one batched sweep
    (FP64, max|dT| over 1000 steps < tol); prints our Nu beside the paper's."""
    import torch
    import paper_2011_15073_amd as P

    N = args.paper_side
    rows_in = paper_cases(N)
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
                                             "eps=1, Darcy drag only, Ma=0.1", "tol": args.sweep_tol,
                                 "max_steps": args.sweep_cap},
                      "wall_s": round(wall, 2), "cases": rows}), flush=True)


def adjoint_main(args):
    """Cost of the gradient of Nu_bar on the 256 x 256 cavity (FP32 forward
    state, FP64 adjoint, n = 0.7, Ra = 1e4, per-cell log10 Da ~ U[-3, -1]
    seed 0, T = 5000 steps, checkpoints every ceil(sqrt(T)) steps): forward
    with checkpoints vs backward (segment replay + adjoint steps).  With the
    [0.1, 10] viscosity clamp the exact adjoint of this workload grows without
    bound (low-shear regions amplify perturbations), so the gradient is taken
    with the shear floor gamma* = --adjoint-shear-floor; the work per step is
    the same either way."""
    import torch
    import paper_2011_15073_amd as P
    from paper_2011_15073_amd import inputs

    N, T = 256, args.adjoint_steps
    ld = torch.from_numpy(inputs.logda_field(N, seed=0))
    times = []
    for rep in range(2):
        cav = P.Cavity(N, dtype="fp32", logda=ld, n=0.7, Ra=1e4, Pr=10.0, eps=0.6)
        adj = P.Adjoint(cav, T, shear_floor=args.adjoint_shear_floor)
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
        "n_gpus": 1, "higher_is_better": False, "dtype": "f32 forward / f64 adjoint",
        "data": "synthetic",
        "config": {"workload": "256x256 porous cavity, n=0.7, Ra=1e4, Pr=10, eps=0.6, per-cell "
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
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "fp64"],
                    help="storage and arithmetic of the timed cavity (fp64: the single-step kernel, 224 B per "
                         "node update)")
    ap.add_argument("--rounding", default="nearest", choices=["nearest", "stochastic"],
                    help="rounding of the FP32 population updates (PM_ROUND_*)")
    ap.add_argument("--roofline-steps", type=int, default=400)
    ap.add_argument("--side", type=int, default=N,
                    help="grid side of the timed cavity (default 4096, the benchmark workload; other sides "
                         "report no counter traffic and no CPU baseline)")
    ap.add_argument("--sweep", action="store_true",
                    help="run the 27-case batched-sweep benchmark instead")
    ap.add_argument("--sweep-dtype", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--sweep-tol", type=float, default=1e-8)
    ap.add_argument("--sweep-cap", type=int, default=3_000_000)
    ap.add_argument("--paper-tables", action="store_true",
                    help="run the paper's validation and parametric cases and print Nu beside its values")
    ap.add_argument("--paper-side", type=int, default=160)
    ap.add_argument("--stream-function", action="store_true",
                    help="time the stream function of the 4096^2 workload")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the gradient of Nu (forward with checkpoints vs backward)")
    ap.add_argument("--adjoint-steps", type=int, default=5000)
    ap.add_argument("--adjoint-shear-floor", type=float, default=0.1,
                    help="nondimensional shear floor of the regularised adjoint (0: exact)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the step is measured on one GPU's share of the grid; a multi-GPU slab split is not implemented)",
              file=sys.stderr)
        sys.exit(2)

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
    # the step kernel the library will run: only the two-step kernel (FP32)
    # needs a second population region in the workspace
    pair = (P.workspace_bytes(P.make_params(S, dtype=dt, step_kernel=args.step_kernel, **PHYS)) >
            P.workspace_bytes(P.make_params(S, dtype=dt, step_kernel="single", **PHYS)))
    kind = ("pair" if pair else "single") + ("_fp64" if dt == "fp64" else "")
    if args.rounding == "stochastic" and kind + "_sr" in KERNELS:
        kind += "_sr"
    K = KERNELS[kind]
    spl = K["steps_per_launch"]
    bpn = BYTES_PER_NODE * (2 if dt == "fp64" else 1)
    log(f"bench: {S}x{S} {dt} {PHYS}, warmup {args.warmup}, steps {args.steps}, step kernel {args.step_kernel} "
        f"({K['name'].split()[0]}), rounding {args.rounding}")
    cav = P.Cavity(S, dtype=dt, device="cuda:0", step_kernel=args.step_kernel, rounding=args.rounding,
                   **PHYS)
    stream = cav.stream

    # warm-up (also builds the step graphs)
    cav.step(args.warmup)
    cav.nu()
    torch.cuda.synchronize()
    log("bench: warm-up done")

    # timed region: K steps with the on-device reductions every CHECK_EVERY steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = args.steps
    nus = []
    while left > 0:
        k = min(CHECK_EVERY, left)
        cav.step(k)
        left -= k
        if k == CHECK_EVERY:
            nus.append(cav.nu())
            cav.residual()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    mlups = S * S * args.steps / elapsed / 1e6
    log(f"bench: {mlups:.1f} MLUPS, {ms_per_step:.4f} ms/step, Nu {nus[-1] if nus else cav.nu():.6f}")

    # roofline of the step kernel: back-to-back launches (for the two-step
    # kernel rs steps from an even step count: rs / 2 launches) bracketed by
    # HIP events on the context's stream
    rs = args.roofline_steps - args.roofline_steps % 4
    with torch.cuda.stream(stream):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cav.step(rs)
        e1.record(stream)
    e1.synchronize()
    per_step_s = e0.elapsed_time(e1) / 1e3 / rs
    launch_s = spl * per_step_s
    achieved = bpn * S * S * spl / launch_s / 1e9
    log(f"bench: {K['name'].split()[0]} {launch_s * 1e6:.1f} us/launch ({per_step_s * 1e6:.1f} us/step), "
        f"{achieved:.0f} GB/s algorithmic")

    # measured streaming-copy ceiling (read + write of 1 GiB)
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        P.copy_probe(src, dst, stream)
    with torch.cuda.stream(stream):
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(10):
            P.copy_probe(src, dst, stream)
        c1.record(stream)
    c1.synchronize()
    copy_gbs = 2 * nbytes * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    log(f"bench: copy ceiling {copy_gbs:.0f} GB/s")

    # counters were taken at 4096^2, with nearest rounding unless the kernel entry is a stochastic one
    traffic = read_traffic(kind) if S == N and (args.rounding == "nearest" or kind.endswith("_sr")) else None
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
                               f"{dt.upper()} AA layout, n=0.8 Da=1e-2 Ra=1e5 Pr=10 eps=0.6, "
                               "Nu + residual on device every 1000 steps",
                   "nodes": S * S, "steps_timed": args.steps, "step_kernel": args.step_kernel,
                   "rounding": args.rounding},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": K["name"],
                     "steps_per_launch": spl,
                     "us_per_launch": round(launch_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": bpn * S * S * spl,
                     "copy_ceiling_GBps": round(copy_gbs, 1)},
        "nu_bar": nus[-1] if nus else None,
    }
    if not args.no_cpu_baseline and S == N:
        del cav
        torch.cuda.empty_cache()
        log("bench: timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
