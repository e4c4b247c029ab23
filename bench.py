#!/usr/bin/env python3
"""Benchmark: Hessian-vector products/s and registrations/min of band-limited
Jacobi PDE-EPDiff LDDMM (Gauss-Newton-Krylov) on one MI355X.

Workload: the 128^3 synthetic tissue phantom, band 32^3 (padded grid 48^3),
L = (Id - 0.0025 Laplacian)^3, sigma = 0.03, 10 Euler steps; the target is
the phantom warped by a random band-limited geodesic of 8 voxels maximal
displacement.  One step = one full registration from v0 = 0: 10 Gauss-Newton
iterations, each with the gradient, 20 CG iterations (one Hessian-vector
product each) and the Armijo line search.  Inputs are resident in HBM before
the timed region.

``--state deformation`` registers the same images subject to the deformation
state equation (paper §3.3) instead of the image state (paper §3.2).
``--batch N`` measures instead the atlas-serving batch: N independent pairs of
different sizes in one lddmm_register_batch call (aggregate HVP/s), all
driven from one host thread; ``--graphs`` replays each pair's captured
sequences.  Before the timed region the tile autotuner (lddmm_autotune)
picks the launch shapes of each problem shape, or ``--tiles FILE`` loads a
table (``--no-autotune``: the built-in rule); the choice is in the JSON line.

Prints one JSON line on stdout (everything else goes to stderr).
"""

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hessian-vector products/s + registrations/min, 128³ band 32³, FP32/BF16 vs FP64"
CONFIG = 3
PEAK_TFLOPS_FP32 = 157.3   # MI355X dense FP32 (MFMA); also the packed-FP32 vector peak
PEAK_GBS_HBM = 8000.0
TIMER_EVERY = 16           # the timed region brackets one launch in 16 of the dominant kernel (on average)
# kernels whose contractions run on the matrix cores
MFMA_KERNELS = {1, 2, 5}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=0,
                    help="measure the atlas-serving batch of this many pairs (lddmm_register_batch) instead")
    ap.add_argument("--concurrency", type=int, default=0, help="pairs running at a time in --batch (0: default)")
    ap.add_argument("--graphs", action="store_true", help="graph replay of the registration loops' sequences")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the tile autotuner before the timed region (built-in launch shapes)")
    ap.add_argument("--tiles", default=None, help="load this tile table (JSON) instead of autotuning")
    ap.add_argument("--tiles-out", default=None, help="write the tile table used to this JSON file")
    ap.add_argument("--band", type=int, default=0,
                    help="register with this band size instead of 32 (the band sweep of the paper's experiment; "
                         "the target stays the one made with band 32)")
    ap.add_argument("--state", choices=("image", "deformation"), default="image",
                    help="constraint of the registered problem: the image state (paper §3.2, the "
                         "default) or the deformation state (paper §3.3)")
    ap.add_argument("--hvp-loop", type=int, default=50, help="extra pure hessvec calls timed")
    ap.add_argument("--precision", choices=("fp32", "bf16x3"), default="fp32",
                    help="arithmetic of the matrix-core contractions of the timed registrations: FP32, or "
                         "compensated BF16 (hi/lo split, three products, FP32 accumulation)")
    ap.add_argument("--no-second-precision", action="store_true",
                    help="skip the shorter measurement of the other precision mode")
    return ap.parse_args()


def roofline(fam, name, launches, ms, flops, nbytes, traffic):
    t = ms * 1e-3
    tf = flops / t / 1e12
    gbs = nbytes / t / 1e9
    f_cmp = tf / PEAK_TFLOPS_FP32
    f_hbm = gbs / PEAK_GBS_HBM
    common = {"kernel": name, "timed_launches": launches, "avg_us": 1e3 * ms / max(launches, 1),
              "flops_per_launch": flops / max(launches, 1), "bytes_per_launch": nbytes / max(launches, 1)}
    if f_hbm > f_cmp:
        return dict({"bound": "hbm", "achieved": gbs, "peak": PEAK_GBS_HBM, "unit": "GB/s", "frac": f_hbm,
                     "traffic": traffic, "tflops": tf}, **common)
    return dict({"bound": "mfma" if fam in MFMA_KERNELS else "alu", "achieved": tf, "peak": PEAK_TFLOPS_FP32,
                 "unit": "TFLOP/s", "frac": f_cmp, "traffic": traffic, "gbs": gbs}, **common)


def stored_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration),
    or None if there is none or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.md")
    src = os.path.join(ROOT, "paper_1807_11560_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] == "traffic" and cells[1] == kernel_name:
            if cells[3] != digest:
                log(f"traffic: {kernel_name} changed since its counters were taken")
                return None
            return float(cells[2])
    return None


def stored_trace(kernel_name):
    """Average duration (us) per launch of `kernel_name` in the committed
    rocprofv3 kernel trace of the measured workload, or None if there is
    none or the kernel source changed since the trace was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "kernels_register_128cubed_band32.md")
    src = os.path.join(ROOT, "paper_1807_11560_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] == "trace" and cells[1] == kernel_name:
            if cells[3] != digest:
                log(f"trace: {kernel_name} changed since the kernel trace was taken")
                return None
            return float(cells[2])
    return None


def _cpu_model():
    """CPU model name of the host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:  # pragma: no cover
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def _blas_threads():
    try:
        import threadpoolctl
        return max(i["num_threads"] for i in threadpoolctl.threadpool_info()) or os.cpu_count()
    except Exception:  # pragma: no cover
        return os.cpu_count()


def _timed(fn, reps):
    """Median wall-clock seconds of `reps` calls of fn (and the last result)."""
    ts, out = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), out


def cpu_baseline(w, state="image", band=None, counts=None):
    """The FP64 oracle on the host cores, on a bounded sample of the measured
    workload: one Euler step of the band EPDiff, one gradient, one
    Hessian-vector product and one line-search trial (a forward shooting and
    transport plus the energy) at v0 = v*/2, medians of 3 where the sample
    allows, on all BLAS threads and (one step and one product) on one thread;
    and the registration time these give, n_grad t_grad + n_hvp t_hvp +
    n_trial t_trial with the counts of the GPU registration.  Also returns the
    oracle results the GPU is checked against."""
    import threadpoolctl
    from oracle import Params
    from oracle.epdiff import shoot
    from oracle.jacobi import energy, forward
    from paper_1807_11560_amd import synth
    if state == "image":
        from oracle.jacobi import gradient, hessvec
        fwd = forward
    else:
        from oracle import deformation as D
        gradient, hessvec, fwd = D.gradient, D.hessvec, D.forward
    cores = int(_blas_threads())
    pp = w["params"]
    p = Params(grid=pp["grid"], band=pp["band"], nt=pp["nt"], alpha=pp["alpha"], s=pp["s"], sigma=pp["sigma"])
    I0, vstar = w["I0"], w["v_star"]
    # the target is the phantom warped by the image-state model in both cases
    I1 = forward(vstar, I0, p)[2][-1]
    at = "v0 = v*/2"
    v0 = 0.5 * vstar
    if band and tuple(band) != tuple(pp["band"]):
        # register with another band: the same target, v0 = 0
        p = dataclasses.replace(p, band=tuple(band), spectral=None)
        v0 = np.zeros((3,) + tuple(band), dtype=np.complex128)
        at = "v0 = 0"
    d = synth.random_direction(4242, p.band, s=pp["s"])
    p1 = dataclasses.replace(p, nt=1)
    t_step, _ = _timed(lambda: shoot(p.dt * v0, p1), 3)
    t_grad, (g, E, cache) = _timed(lambda: gradient(v0, I0, I1, p), 1)
    t_hvp, h = _timed(lambda: hessvec(cache, d, p, "R1"), 3)

    def trial():
        m1 = fwd(v0, I0, p)[2]
        return energy(v0, m1[-1] if state == "image" else m1, I1, p)

    t_trial, _ = _timed(trial, 1)
    with threadpoolctl.threadpool_limits(1):
        t_step1, _ = _timed(lambda: shoot(p.dt * v0, p1), 1)
        t_hvp1, _ = _timed(lambda: hessvec(cache, d, p, "R1"), 1)
    out = {"value": 1.0 / t_hvp, "unit": "HVP/s", "cores": cores, "kind": "oracle",
           "sample": f"128^3 / band {p.band[0]}^3 problem ({state} state) at {at}, FP64 NumPy: one Euler step "
                     f"of the band EPDiff (median of 3), one gradient, one Hessian-vector product (median of "
                     f"3), one line-search trial on {cores} threads; one step and one product on 1 thread",
           "cpu_model": _cpu_model(), "numpy": np.__version__,
           "seconds": {"euler_step": t_step, "gradient": t_grad, "hvp": t_hvp, "line_search_trial": t_trial,
                       "euler_step_1_thread": t_step1, "hvp_1_thread": t_hvp1},
           "hvp_per_s_1_thread": 1.0 / t_hvp1}
    if counts:
        t_reg = counts["gradients"] * t_grad + counts["hvps"] * t_hvp + counts["trials"] * t_trial
        out["registration_seconds_extrapolated"] = t_reg
        out["registrations_per_min_extrapolated"] = 60.0 / t_reg
        out["extrapolation"] = (f"{counts['gradients']} gradients x {t_grad:.2f} s + {counts['hvps']} products x "
                                f"{t_hvp:.2f} s + {counts['trials']} trials x {t_trial:.2f} s (counts of the GPU "
                                "registration; the oracle registration itself is not run)")
    refs = {"I1": I1, "v0": v0, "direction": d, "gradient": g, "energy": E, "hvp": h, "params": p}
    return out, refs


def gpu_accuracy(L, prob, refs, dev):
    """Relative errors of the library against the FP64 oracle on the sample
    of cpu_baseline: energy, gradient and the Hessian-vector product (the
    timed operation) at the same v0 and direction, on the oracle's target."""
    import torch
    ws = L.Workspace(prob, dev)
    I0 = refs["I0"]
    g, e3 = L.gradient(prob, I0, torch.from_numpy(refs["I1"]).float().to(dev),
                       torch.from_numpy(refs["v0"]).to(torch.complex64).to(dev), ws)
    h = L.hessvec(prob, torch.from_numpy(refs["direction"]).to(torch.complex64).to(dev), ws)
    torch.cuda.synchronize()

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    e3 = e3.cpu().numpy()
    return {"hvp_rel_l2": rel(h.cpu().numpy().astype(np.complex128), refs["hvp"]),
            "gradient_rel_l2": rel(g.cpu().numpy().astype(np.complex128), refs["gradient"]),
            "energy_rel": float(abs(e3[0] - refs["energy"][0]) / abs(refs["energy"][0])),
            "against": "FP64 oracle, same inputs (v0 = v*/2 or 0, one random direction)"}


def separable_flops(K, G):
    """Flops of one band <-> grid transform of a scalar field by separable
    partial DFTs over the full spectrum: two complex stages, then a real
    last stage (the count of the method's separable algorithm before any
    Hermitian saving)."""
    return 8.0 * (G[0] * K[0] * K[1] * K[2] + G[0] * G[1] * K[1] * K[2]) + 4.0 * G[0] * G[1] * G[2] * K[2]


def hvp_work(L, prob, ws, d):
    """Flops and HBM bytes one Hessian-vector product performs: the library's
    per-launch work counts (the half-spectrum contractions, products,
    interpolation and every launch's inputs and outputs, each read or written
    once) summed over every kernel family, one family timed per product."""
    import torch
    fl = by = 0.0
    per = {}
    for fam in L.KERNEL_FAMILIES:
        L.kernel_timer(fam, 1)
        L.hessvec(prob, d, ws)
        torch.cuda.synchronize()
        _, _, f, b = L.kernel_timer_read()
        per[L.KERNEL_FAMILIES[fam]] = {"gflop": f / 1e9, "mb": b / 1e6}
        fl += f
        by += b
    L.kernel_timer(0)
    return fl, by, per


def hvp_ceiling(prob, work, res_value, hvp_only):
    """The whole-HVP roofline: the performed flops against the FP32 matrix
    peak and the performed kernel traffic against HBM, whichever is longer;
    the measured rates as fractions of it.  The full-spectrum count of the
    separable algorithm (60 padded-grid and 3.3 image-grid transforms per time
    step) is given beside it."""
    flops, nbytes, per = work
    K = prob.band
    M = tuple(3 * k // 2 for k in K)
    nt = prob.time_steps
    full = 60.0 * nt * separable_flops(K, M) + 3.3 * nt * separable_flops(K, prob.grid)
    t_cmp = flops / (PEAK_TFLOPS_FP32 * 1e12)
    t_mem = nbytes / (PEAK_GBS_HBM * 1e9)
    ceiling = 1.0 / max(t_cmp, t_mem)
    return {"flops_per_hvp": flops, "kernel_bytes_per_hvp": nbytes,
            "bound": "mfma" if t_cmp >= t_mem else "hbm",
            "ceiling_hvp_per_s": ceiling, "frac_registration": res_value / ceiling,
            "frac_back_to_back": (hvp_only / ceiling) if hvp_only else None,
            "full_spectrum_flops_per_hvp": full, "per_kernel": per}


def dominant_family(L, run):
    """The kernel family with the largest summed duration over one run."""
    fam_ms = {}
    for fam in L.KERNEL_FAMILIES:
        L.kernel_timer(fam, 1)
        run()
        fam_ms[fam] = L.kernel_timer_read()[1]
    L.kernel_timer(0)
    log("ms per run by kernel: " + ", ".join(f"{L.KERNEL_FAMILIES[f]} {fam_ms[f]:.2f}" for f in fam_ms))
    return max(fam_ms, key=fam_ms.get)


def select_tiles(args, L, jobs):
    """The launch shapes of the timed region: the tile table loaded from
    --tiles, else the autotuner's choice for each problem shape (one untimed
    tuning run per shape, on its first job: (problem, I0, I1, v0, ws)), else
    the built-in rule.  Returns what was chosen, per shape."""
    out = {}
    if args.tiles:
        L.tiles_load(args.tiles)
        for prob, *_ in jobs:
            out["x".join(map(str, prob.grid)) + f"/{prob.band[0]}"] = {"chosen": L.tiles_get(prob),
                                                                       "from": args.tiles}
    elif not args.no_autotune:
        seen = set()
        for prob, I0, I1, v0, ws in jobs:
            key = (prob.grid, prob.band, prob.precision)
            if key in seen:
                continue
            seen.add(key)
            best, ms_b, ms_d = L.autotune(prob, I0, I1, v0, ws, reps=10)
            name = "x".join(map(str, prob.grid)) + f"/{prob.band[0]}"
            log(f"autotune {name}: {best}, {ms_b:.3f} ms per product (built-in rule {ms_d:.3f} ms)")
            out[name] = {"chosen": best, "ms_per_hvp": ms_b, "built_in_ms_per_hvp": ms_d}
    if args.tiles_out:
        L.tiles_save(args.tiles_out)
    return out or None


def batch_main(args):
    """The atlas-serving batch: independent registrations of different sizes
    in one lddmm_register_batch call."""
    import torch
    from paper_1807_11560_amd import lddmm as L
    from paper_1807_11560_amd import synth

    dev = torch.device("cuda:0")
    work = synth.batch_workload(pairs=args.batch)
    probs, I0s, I1s = [], [], []
    for w in work:
        pp = w["params"]
        prob = L.Problem(grid=pp["grid"], band=pp["band"], time_steps=pp["nt"], alpha=pp["alpha"], s=pp["s"],
                         sigma=pp["sigma"], hessian=L.GN_PAPER)
        I0 = torch.from_numpy(w["I0"]).float().to(dev)
        I1 = L.shoot(prob, I0, torch.from_numpy(w["v_star"]).to(torch.complex64).to(dev), L.Workspace(prob, dev))
        probs.append(prob)
        I0s.append(I0)
        I1s.append(I1)
    gn, pcg = synth.BATCH["gn"], synth.BATCH["pcg"]
    tune = []
    for w, prob, I0, I1 in zip(work, probs, I0s, I1s):
        if any(q.grid == prob.grid and q.band == prob.band for q, *_ in tune):
            continue
        v0 = torch.from_numpy(0.5 * w["v_star"]).to(torch.complex64).to(dev)
        tune.append((prob, I0, I1, v0, L.Workspace(prob, dev)))
    tiles = select_tiles(args, L, tune)
    del tune
    ws = L.BatchWorkspace(probs, dev)
    torch.cuda.synchronize()
    log(f"batch ready: {len(probs)} pairs, workspace {ws.nbytes / 2**30:.2f} GiB")
    L.use_graphs(bool(args.graphs))

    def run():
        return L.register_batch(probs, I0s, I1s, ws, gn_iters=gn, pcg_iters=pcg, concurrency=args.concurrency)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    dominant = dominant_family(L, run)
    L.kernel_timer(dominant, TIMER_EVERY)
    hvps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, stats, status, hv, rc = run()
        hvps += sum(hv)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    launches, kms, kfl, kby = L.kernel_timer_read()
    L.kernel_timer(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hvps_u = 0
    for _ in range(args.steps):
        hvps_u += sum(run()[3])
    torch.cuda.synchronize()
    T_u = time.perf_counter() - t0
    log(f"timed {args.steps} batches in {T:.3f} s, {hvps} HVPs; status {rc}")
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline_pair(work[0])
        log(f"oracle: {cpu['seconds']:.1f} s per HVP on {cpu['cores']} threads")
    name = L.KERNEL_FAMILIES[dominant]
    res = {
        "metric": METRIC,
        "value": hvps / T,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"atlas serving batch: {len(probs)} tissue-phantom pairs, grids from 96^3 to "
                        "160x192x160, bands 24^3 / 32^3, geodesics of 4-10 voxels, s=3, nt=10, "
                        f"{gn} Gauss-Newton x {pcg} CG iterations each, lddmm_register_batch",
            "pairs": [[list(q.grid), q.band[0]] for q in probs],
            "concurrency": args.concurrency or 8,
            "driver": "one host thread resuming every pair's loop" + (", graph replay" if args.graphs else ""),
        },
        "tiles": tiles,
        "registrations_per_min": 60.0 * args.steps * len(probs) / T,
        "value_without_timer_events": hvps_u / T_u,
        "final_mse_rel_mean": float(np.mean([s[-1]["mse_rel"] for s in stats])),
        "pair_status": [int(x) for x in status],
        "pair_hvps": [int(x) for x in hv],
        "workspace_mib": ws.nbytes / 2**20,
        "roofline": roofline(dominant, name, launches, kms, kfl, kby, None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def cpu_baseline_pair(w):
    """The FP64 oracle on the host: one Hessian-vector product of one pair of
    the batch at v0 = v*/2, after an untimed oracle gradient."""
    from oracle import Params
    from oracle.jacobi import forward, gradient, hessvec
    from paper_1807_11560_amd import synth
    try:
        import threadpoolctl
        cores = max(i["num_threads"] for i in threadpoolctl.threadpool_info()) or os.cpu_count()
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    pp = w["params"]
    p = Params(grid=pp["grid"], band=pp["band"], nt=pp["nt"], alpha=pp["alpha"], s=pp["s"], sigma=pp["sigma"])
    I0, vstar = w["I0"], w["v_star"]
    I1 = forward(vstar, I0, p)[2][-1]
    _, _, cache = gradient(0.5 * vstar, I0, I1, p)
    d = synth.random_direction(4242, p.band, s=pp["s"])
    t0 = time.perf_counter()
    hessvec(cache, d, p, "R1")
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "HVP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one Hessian-vector product of the first pair ({'x'.join(map(str, pp['grid']))}, band "
                      f"{pp['band'][0]}^3) at v0 = v*/2 (FP64 NumPy, after an untimed oracle gradient)",
            "seconds": t}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    if args.batch:
        batch_main(args)
        return

    import torch
    from paper_1807_11560_amd import lddmm as L
    from paper_1807_11560_amd import synth

    w = synth.workload(CONFIG)
    pp = w["params"]
    # the target is the phantom warped by the image-state model in both cases
    prob_img = L.Problem(grid=pp["grid"], band=pp["band"], time_steps=pp["nt"], alpha=pp["alpha"], s=pp["s"],
                         sigma=pp["sigma"], hessian=L.GN_PAPER)
    band = (args.band,) * 3 if args.band else tuple(pp["band"])
    prec = L.FP32 if args.precision == "fp32" else L.FP32_BF16X3
    prob = dataclasses.replace(prob_img, band=band, precision=prec,
                               state=L.STATE_IMAGE if args.state == "image" else L.STATE_DEFORMATION)
    gn, pcg = pp["gn"], pp["pcg"]
    dev = torch.device("cuda:0")
    ws = L.Workspace(prob, dev)
    I0 = torch.from_numpy(w["I0"]).float().to(dev)
    vstar = torch.from_numpy(w["v_star"]).to(torch.complex64).to(dev)
    # the target is made by the FP32 image-state shooting in every mode
    I1 = L.shoot(prob_img, I0, vstar, L.Workspace(prob_img, dev))
    torch.cuda.synchronize()
    log(f"workload ready: grid {prob.grid} band {prob.band} ws {ws.nbytes / 2**20:.0f} MiB")
    tiles = select_tiles(args, L, [(prob, I0, I1, 0.5 * vstar, ws)])
    L.use_graphs(bool(args.graphs))

    def registration():
        return L.register(prob, I0, I1, ws, gn_iters=gn, pcg_iters=pcg)

    for _ in range(args.warmup):
        registration()
    torch.cuda.synchronize()

    # dominant kernel: the largest summed duration over one registration
    fam_ms = {}
    for fam in L.KERNEL_FAMILIES:
        L.kernel_timer(fam, 1)
        registration()
        fam_ms[fam] = L.kernel_timer_read()[1]
    L.kernel_timer(0)
    dominant = max(fam_ms, key=fam_ms.get)
    log("ms per registration by kernel: " + ", ".join(f"{L.KERNEL_FAMILIES[f]} {fam_ms[f]:.2f}" for f in fam_ms))

    # timed region: K registrations, about one launch in TIMER_EVERY of the dominant kernel bracketed by events
    L.kernel_timer(dominant, TIMER_EVERY)
    hvps = 0
    stats = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        v, stats, rc, n = registration()
        hvps += n
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    launches, kms, kfl, kby = L.kernel_timer_read()
    L.kernel_timer(0)
    log(f"timed {args.steps} registrations in {T:.3f} s, {hvps} HVPs; last status {rc}")
    for i, s in enumerate(stats):
        log(f"  GN {i}: E {s['energy']:.5f} MSE_rel {s['mse_rel']:.3f} |g|rel {s['grad_inf_rel']:.4f} "
            f"eps {s['step']} pcg {s['pcg_iters']}")

    # the same registrations without the timing events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hvps_u = 0
    for _ in range(args.steps):
        hvps_u += registration()[3]
    torch.cuda.synchronize()
    T_u = time.perf_counter() - t0

    # pure Hessian-vector product rate (same problem, last iterate)
    hvp_only = hvp_med = cold_ms = work = hvp_enqueue_ms = None
    if args.hvp_loop > 0:
        L.gradient(prob, I0, I1, v, ws)
        d = torch.from_numpy(synth.random_direction(1, prob.band, s=pp["s"])).to(torch.complex64).to(dev)
        out = torch.empty_like(d)
        for _ in range(3):
            L.hessvec(prob, d, ws, out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.hvp_loop):
            L.hessvec(prob, d, ws, out=out)
        t_enq = time.perf_counter()
        torch.cuda.synchronize()
        hvp_only = args.hvp_loop / (time.perf_counter() - t1)
        # host time to enqueue one product (its launches, event records and waits)
        hvp_enqueue_ms = 1e3 * (t_enq - t1) / args.hvp_loop
        # per-call durations (events on the stream the library runs on) and the cold product
        # (gradient with its trajectories recomputed, then the product)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        for e0, e1 in evs:
            e0.record()
            L.hessvec(prob, d, ws, out=out)
            e1.record()
        torch.cuda.synchronize()
        hvp_med = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
        t1 = time.perf_counter()
        for _ in range(5):
            L.gradient(prob, I0, I1, v, ws)
            L.hessvec(prob, d, ws, out=out)
        torch.cuda.synchronize()
        cold_ms = 1e3 * (time.perf_counter() - t1) / 5
        work = hvp_work(L, prob, ws, d)

    # plain copy of known size: the calibration for the FETCH_SIZE / WRITE_SIZE counters
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    # the configured 20 CG iterations: classical Gauss-Newton (definite), whose
    # CG is not cut short by the curvature guard
    prob_cl = dataclasses.replace(prob, hessian=L.GN_CLASSICAL)
    ws_cl = L.Workspace(prob_cl, dev)
    L.register(prob_cl, I0, I1, ws_cl, gn_iters=gn, pcg_iters=pcg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st_cl, _, n_cl = L.register(prob_cl, I0, I1, ws_cl, gn_iters=gn, pcg_iters=pcg)
    torch.cuda.synchronize()
    T_cl = time.perf_counter() - t0
    del ws_cl
    classical = {"registrations_per_min": 60.0 / T_cl, "hvps_per_registration": n_cl, "hvp_per_s": n_cl / T_cl,
                 "final_mse_rel": st_cl[-1]["mse_rel"] if st_cl else None,
                 "what": "one registration with classical Gauss-Newton (coupling terms dropped)"}

    # the other precision mode, shorter: one registration and back-to-back products
    other = None
    if not args.no_second_precision:
        prob_o = dataclasses.replace(prob, precision=L.FP32_BF16X3 if prec == L.FP32 else L.FP32)
        ws_o = L.Workspace(prob_o, dev)
        L.register(prob_o, I0, I1, ws_o, gn_iters=gn, pcg_iters=pcg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v_o, st_o, _, n_o = L.register(prob_o, I0, I1, ws_o, gn_iters=gn, pcg_iters=pcg)
        torch.cuda.synchronize()
        T_o = time.perf_counter() - t0
        L.gradient(prob_o, I0, I1, v_o, ws_o)
        d_o = torch.from_numpy(synth.random_direction(1, prob.band, s=pp["s"])).to(torch.complex64).to(dev)
        out_o = torch.empty_like(d_o)
        for _ in range(3):
            L.hessvec(prob_o, d_o, ws_o, out=out_o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.hvp_loop or 20):
            L.hessvec(prob_o, d_o, ws_o, out=out_o)
        torch.cuda.synchronize()
        other = {"dtype": "bf16x3" if prob_o.precision == L.FP32_BF16X3 else "f32",
                 "value": n_o / T_o, "unit": "HVP/s", "registrations_per_min": 60.0 / T_o,
                 "hvps_per_registration": n_o,
                 "hvp_only_per_s": (args.hvp_loop or 20) / (time.perf_counter() - t1),
                 "final_mse_rel": st_o[-1]["mse_rel"] if st_o else None,
                 "what": "one registration and back-to-back products of the same workload"}
        del ws_o

    cpu = accuracy = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        counts = {"gradients": len(stats), "hvps": int(round(hvps / args.steps)),
                  "trials": int(sum(s["trials"] for s in stats))}
        cpu, refs = cpu_baseline(w, args.state, band, counts)
        log(f"oracle: {cpu['seconds']}")
        refs["I0"] = I0
        accuracy = gpu_accuracy(L, prob, refs, dev)
        log(f"accuracy against the oracle: {accuracy}")
        if other is not None:
            other["accuracy_vs_fp64"] = gpu_accuracy(L, prob_o, refs, dev)
            log(f"{other['dtype']} accuracy against the oracle: {other['accuracy_vs_fp64']}")

    name = L.KERNEL_FAMILIES[dominant]
    res = {
        "metric": METRIC,
        "value": hvps / T,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.FP32 else "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": "tissue phantom 128^3 registered to its warp by a random band-limited geodesic "
                        "(8 voxels), band 32^3, padded grid 48^3, s=3, alpha=0.0025, sigma=0.03, nt=10, "
                        "10 Gauss-Newton x 20 CG iterations, paper Gauss-Newton reading"
                        + ("" if args.state == "image" else ", subject to the deformation state equation")
                        + ("" if band == tuple(pp["band"]) else f", registered with band {band[0]}^3 "
                           f"(padded grid {3 * band[0] // 2}^3)"),
            "state": args.state, "precision": args.precision,
            "grid": list(prob.grid), "band": list(prob.band), "time_steps": prob.time_steps,
            "gn_iters": gn, "pcg_iters": pcg,
        },
        "registrations_per_min": 60.0 * args.steps / T,
        "hvps_per_registration": hvps / args.steps,
        "value_without_timer_events": hvps_u / T_u,
        "hvp_only_per_s": hvp_only,
        "hvp_ms_median": hvp_med,
        "hvp_enqueue_ms": hvp_enqueue_ms,
        "cold_hvp_ms": cold_ms,
        "hvp_roofline": hvp_ceiling(prob, work, res_value=hvps / T, hvp_only=hvp_only) if work else None,
        "gn_classical": classical,
        "other_precision": other,
        "accuracy_vs_fp64": accuracy,
        "final_mse_rel": stats[-1]["mse_rel"] if stats else None,
        "final_grad_inf_rel": stats[-1]["grad_inf_rel"] if stats else None,
        "workspace_mib": ws.nbytes / 2**20,
        "tiles": tiles,
        "graphs": bool(args.graphs),
        "roofline": roofline(dominant, name, launches, kms, kfl, kby, stored_traffic(name)),
        "cpu_baseline": cpu,
    }
    # the same kernel's average duration in the committed kernel trace of this workload (the
    # events of a timed launch also span the command processor's work around it)
    default_workload = (args.state == "image" and band == tuple(pp["band"]) and prec == L.FP32)
    tr = stored_trace(name) if default_workload else None
    if tr:
        rl = res["roofline"]
        rl["trace_avg_us"] = tr
        per = rl["bytes_per_launch"] if rl["bound"] == "hbm" else rl["flops_per_launch"]
        scale = 1e-9 if rl["bound"] == "hbm" else 1e-12
        rl["frac_trace"] = per / (tr * 1e-6) * scale / rl["peak"]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
