"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the hash of a
step kernel's code, and the rule that counter traffic is reported only for
the kernel code it was measured on."""
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_algorithmic_bytes_per_node_update():
    # 9 + 5 FP32 populations, each read once and written once
    assert bench.BYTES_PER_NODE == (9 + 5) * 4 * 2


def _recorded(kind):
    vals = {}
    for line in open(bench.KERNELS[kind]["traffic_file"]):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    return vals


@pytest.mark.parametrize("kind", sorted(bench.KERNELS))
def test_traffic_only_for_the_measured_kernel_code(kind, monkeypatch):
    vals = _recorded(kind)
    monkeypatch.setattr(bench, "kernel_hash", lambda k="pair": vals["kernel_source_sha256_16"])
    t = bench.read_traffic(kind)
    assert t == float(vals["hbm_bytes_per_launch"]) and t > 0
    monkeypatch.setattr(bench, "kernel_hash", lambda k="pair": "0" * 16)
    assert bench.read_traffic(kind) is None


@pytest.mark.parametrize("kind", ["pair", "pair_sr", "single_sr", "single_fp16"])
def test_counters_only_for_the_measured_kernel_code(kind, monkeypatch):
    text = open(bench.SQ_COUNTERS).read()
    fam = "pair" if kind.startswith("pair") else "single"
    recorded = text.split(f"bench.kernel_hash('{fam}') = ")[1][:16]
    monkeypatch.setattr(bench, "kernel_hash", lambda k="pair": recorded)
    c = bench.read_counters(kind)
    assert c is not None and 0 < c["valu_issue_share"] <= 1 and 0 <= c["wait_share"] <= 1
    assert c["valu_per_node_update"] > 100
    monkeypatch.setattr(bench, "kernel_hash", lambda k="pair": "0" * 16)
    assert bench.read_counters(kind) is None


@pytest.mark.parametrize("kind", sorted(bench.KERNELS))
def test_kernel_hash_follows_code_not_comments(kind, tmp_path, monkeypatch):
    srcs = []
    for src in bench.KERNELS[kind]["srcs"]:
        path, pattern = src if isinstance(src, tuple) else (src, None)
        dst = tmp_path / os.path.basename(path)
        if not dst.exists():
            shutil.copy(path, dst)
        srcs.append((str(dst), pattern) if pattern else str(dst))
    monkeypatch.setitem(bench.KERNELS, kind, dict(bench.KERNELS[kind], srcs=srcs))
    h0 = bench.kernel_hash(kind)
    assert len(h0) == 16 and int(h0, 16) >= 0
    dev = tmp_path / "pm_device.h"
    text = dev.read_text()
    dev.write_text("// a comment line\n" + text.replace("\n", "\n  ", 3) + "/* another */\n")
    assert bench.kernel_hash(kind) == h0
    dev.write_text(text.replace("T(0.5)", "T(0.25)", 1))
    assert bench.kernel_hash(kind) != h0


def test_oracle_table_rates(monkeypatch):
    """The oracle-timing table (bench.py --oracle-table) on one-step samples:
    every workload timed, its whole-run estimate the sampled rate scaled to
    the run's node updates."""
    small = [w[:5] + (1, 1) for w in bench.ORACLE_WORKLOADS if w[1] is not None]
    monkeypatch.setattr(bench, "ORACLE_WORKLOADS", small)
    rows = bench._oracle_rates(one_core=True)
    assert len(rows) == len(small) == 3
    for (name, side, _, _, full, _, _), r in zip(small, rows):
        assert r["workload"] == name and r["steps_sampled"] == 1 and r["mlups"] > 0
        assert r["est_full_run_s"] == pytest.approx(side * side * full / (r["mlups"] * 1e6), rel=2e-2, abs=0.2)
