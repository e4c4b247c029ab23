"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
work counts behind the whole-HVP ceiling, the roofline record and the stored
traffic lines."""

import hashlib
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_separable_transform_counts():
    """Band 32^3 to the 48^3 padded grid: 8 (M K K K + M M K K) + 4 M M M K
    flops (two complex stages, a real last stage); to the 128^3 grid the
    same form."""
    assert bench.separable_flops((32, 32, 32), (48, 48, 48)) == 8 * (48 * 32**3 + 48**2 * 32**2) + 4 * 48**3 * 32
    assert abs(bench.separable_flops((32, 32, 32), (48, 48, 48)) - 45.6e6) < 0.05e6
    assert abs(bench.separable_flops((32, 32, 32), (128, 128, 128)) - 436.2e6) < 0.1e6


def test_whole_hvp_ceiling():
    """The ceiling is priced at the work the kernels perform (the library's
    per-launch counts summed over one product) against 157.3 TFLOP/s, or its
    kernels' traffic against 8 TB/s when that takes longer (19.8 GFLOP is
    126 us, 1.9 GB is 238 us: traffic-bound); the full-spectrum count of the
    separable algorithm (600 padded-grid and 33 image-grid transforms at
    nt = 10, 41.8 GFLOP) is reported beside it."""
    prob = types.SimpleNamespace(band=(32, 32, 32), grid=(128, 128, 128), time_steps=10)
    work = (19.8e9, 1.9e9, {})
    c = bench.hvp_ceiling(prob, work, res_value=900.0, hvp_only=1200.0)
    assert c["flops_per_hvp"] == 19.8e9 and c["kernel_bytes_per_hvp"] == 1.9e9
    assert c["bound"] == "hbm"
    t_cmp, t_mem = 19.8e9 / 157.3e12, 1.9e9 / 8000e9
    assert abs(c["ceiling_hvp_per_s"] - 1.0 / max(t_cmp, t_mem)) < 1e-6
    assert abs(c["full_spectrum_flops_per_hvp"] - 41.76e9) < 0.01e9
    assert abs(c["frac_registration"] - 900.0 / c["ceiling_hvp_per_s"]) < 1e-12
    assert abs(c["frac_back_to_back"] - 1200.0 / c["ceiling_hvp_per_s"]) < 1e-12
    assert bench.hvp_ceiling(prob, work, 900.0, None)["frac_back_to_back"] is None
    # compute-bound when the flops take longer than the bytes
    assert bench.hvp_ceiling(prob, (19.8e9, 0.5e9, {}), 900.0, None)["bound"] == "mfma"


def test_roofline_record_picks_the_binding_fraction():
    # 1 ms for 10 launches of 10 GFLOP and 1 GB: 10 TFLOP/s (6.4 %) against 1000 GB/s (12.5 %)
    r = bench.roofline(5, "k_colstep", 10, 1.0, 10e9, 1e9, None)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["frac"] - 1000.0 / bench.PEAK_GBS_HBM) < 1e-12
    r = bench.roofline(5, "k_colstep", 10, 1.0, 100e9, 1e9, 123.0)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["traffic"] == 123.0
    assert abs(r["achieved"] - 100.0) < 1e-9 and abs(r["avg_us"] - 100.0) < 1e-9
    assert bench.roofline(3, "k_sl", 10, 1.0, 100e9, 1e9, None)["bound"] == "alu"


def test_stored_traffic_follows_the_kernel_source():
    src = os.path.join(ROOT, "paper_1807_11560_amd", "csrc", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    lines = [ln for ln in open(os.path.join(ROOT, "profiles", "traffic.md")) if ln.startswith("| traffic |")]
    assert lines, "profiles/traffic.md has no machine-readable lines"
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        expect = float(cells[2]) if cells[3] == digest else None
        assert bench.stored_traffic(cells[1]) == expect
    assert bench.stored_traffic("no_such_kernel") is None
