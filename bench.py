"""Benchmark of the SPGR multi-parameter-mapping hot path on one MI355X.

One step = the whole hot path over the whole-brain synthetic volume
(192 x 240 x 256 voxels, 8/8/6 echoes of PDw/T1w/MTw, B1 in [0.8, 1.2]):
  1. ML fit, 20 Newton-like steps per voxel (default initialisation);
  2. JTV-MAP fit, 10 IRLS loops x 8 Newton-like steps x 32 CG iterations;
  3. Laplace posterior variance (+ log-normal moments of R1 / T1) at the MAP maps.
Echoes are simulated on the GPU from seeded ground-truth maps and seeded noise
before the clock starts, so the timed region starts with every input resident
in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--dtype f32|f16|bf16] [--no-cpu-baseline]

Other workloads (one JSON line each; not the headline step):
    --hires       JTV-MAP + variance on 416 x 384 x 320 voxels with FP16 echoes
    --projected   the MAP fit with two contrasts acquired on moved grids (Sec. 2.4)
    --e1          the convergence experiment of Sec. 3.1 at scale (1 M voxels, a
                  protocol each, 10,000 steps) and its rate / time representation
                  comparison
    --noise       the noise estimation of Sec. 2.7 on the whole-brain volume in air
    --serving     the continuous-batching queue on a mix of 64 ML and MAP requests
    --autotune    mpm_autotune's CG sweep times per workgroup count on the serving sizes
    --counters    a short workload for rocprofv3 counter runs (with --projected or
                  --e1: theirs)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# Per-voxel byte model of the planned hot path (compulsory HBM bytes): CG
# sweep A reads z, the previous direction, w and the 10-entry Hessian and
# writes p and q (16 + 16 + 4 + 40 + 16 + 16); sweep B reads the solution,
# residual, p, q, the Hessian and the stencil diagonal and writes the solution,
# residual and z (156).  The kernels' own byte counts differ (sweep A writes no
# q and carries the deferred solution update; sweep B recomputes q) and are
# reported beside these.
MODEL_BYTES_PER_VOXEL = {"cg_a": 108.0, "cg_b": 156.0}
# The whole step per voxel: ML fit 108 B; 80 MAP Newton steps of 8772 B
# (likelihood pass 168, CG start 108, 32 x (108 + 156), update 48); the Laplace
# variance pass 164 B (echoes 88, b1 4, maps 16, w 4, 20 for the weights
# pass, variance 16, moments 16).
STEP_MODEL_BYTES_PER_VOXEL = 108.0 + 80 * 8772.0 + 164.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2102_01604_amd", "csrc", f)
                  for f in ("k_map.hip", "mpm_map.h", "mpm_device.h", "mpm_kernels.h", "mpm_tune.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_map_brain.txt")
# the oracle's full 10 x 8 x 32 MAP fit of the whole-brain volume, stored once
# with its wall time by tests/golden/make_whole_brain_map.py
ORACLE_FULL_FIT = os.path.join(ROOT, "tests", "golden", "whole_brain_map_10x8x32.json")
VALU_SOURCES = [os.path.join(ROOT, "paper_2102_01604_amd", "csrc", f)
                for f in ("k_voxel.hip", "mpm_voxelwise.h", "mpm_device.h")]
VALU_FILE = os.path.join(ROOT, "profiles", "valu_ml_fit_pv_e1.txt")
ML_VALU_FILE = os.path.join(ROOT, "profiles", "valu_ml_fit_brain.txt")
NOISE_SOURCES = [os.path.join(ROOT, "paper_2102_01604_amd", "csrc", f)
                 for f in ("k_noise.hip", "mpm_noise.h", "mpm_device.h")]
NOISE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_noise_hist_brain.txt")
# Published FP32 vector peak 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 FMA lanes
# per clock: 2 wave64 VALU instructions per clock per CU, 78.6 T lane-instructions/s.
VALU_PEAK_T = 256 * 2.4e9 * 128 / 1e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel, path=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch measured by rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy-kernel calibration), recorded together with
    the hash of the kernel sources they were taken on; None if absent or stale."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_hash(sources) or kv.get("kernel") != kernel:
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_ml_valu():
    """VALU lane-instructions per voxel evaluation of the whole-brain ML kernel
    from the committed counter summary; None if absent or taken on other sources."""
    if not os.path.exists(ML_VALU_FILE):
        return None
    kv = {}
    for line in open(ML_VALU_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_hash(VALU_SOURCES):
        return None
    try:
        return float(kv["SQ_INSTS_VALU_dispatch0_lanes_per_voxel_eval"])
    except KeyError:
        return None


def read_valu_counts():
    """VALU lane-instructions per voxel evaluation of the voxelwise ML kernel,
    per loading (dispatch order Proposed, Proposed+, Gauss-Newton, then the
    rate and time representations with Proposed+), from the committed counter
    summary; None if absent or taken on other sources."""
    if not os.path.exists(VALU_FILE):
        return None
    kv = {}
    for line in open(VALU_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_hash(VALU_SOURCES):
        return None
    try:
        out = {load: float(kv[f"SQ_INSTS_VALU_dispatch{d}_lanes_per_voxel_eval"])
               for d, load in enumerate(("proposed", "plus", "gn"))}
    except KeyError:
        return None
    for d, basis in ((3, "rate"), (4, "time")):
        v = kv.get(f"SQ_INSTS_VALU_dispatch{d}_lanes_per_voxel_eval")
        if v is not None:
            out[basis] = float(v)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving-leg", dest="serving_leg", action="store_false",
                    help="skip the serving leg (64 requests of four sizes in one burst, schedule seed 4000, "
                         "continuous batching against serial fits)")
    ap.add_argument("--profile-every", type=int, default=7,
                    help="bracket one in this many launches of each kernel with HIP events")
    ap.add_argument("--dims", default="192,240,256")
    ap.add_argument("--serving", action="store_true",
                    help="serving benchmark instead: 64 fit requests of uneven sizes (ML or MAP), Poisson "
                         "arrivals, continuous-batching server against serial plain fits; one JSON line")
    ap.add_argument("--hires", action="store_true",
                    help="high-resolution workload instead: 416 x 384 x 320 voxels, FP16 echo storage, B1 in "
                         "[0.7, 1.3], sigma 2%% of mean PD, JTV-MAP 10 x 8 x 32 then the Laplace variance")
    ap.add_argument("--projected", action="store_true",
                    help="spatially projected workload instead: T1w and MTw on rigidly moved grids, JTV-MAP "
                         "10 x 8 x 32 then the Laplace variance on the 192 x 240 x 256 reconstruction grid "
                         "(with --counters: a 2 x 1 x 32 projected fit and the copy calibration, then exit)")
    ap.add_argument("--e1", action="store_true",
                    help="the paper's convergence experiment at scale instead: a random protocol per voxel, ML "
                         "steps with the Proposed, Proposed+ and Gauss-Newton loadings")
    ap.add_argument("--noise", action="store_true",
                    help="the noise estimation of Sec. 2.7 (histogram + Rician mixture per image) on the "
                         "whole-brain volume placed in air")
    ap.add_argument("--batch", action="store_true",
                    help="batched JTV-MAP fits (mpm_fit_batch) against the same fits one after another: 16 volumes "
                         "of 64^3 and 4 of 96 x 128 x 128, 10 x 8 x 32 each; one JSON line")
    ap.add_argument("--oracle-full", action="store_true",
                    help="CPU only: the FP64 oracle on the whole benchmark volume (ML 20 GN, MAP 10 x 8 x 32, "
                         "variance), each stage timed; one JSON line (tens of minutes)")
    ap.add_argument("--autotune", action="store_true",
                    help="mpm_autotune on the four serving volume sizes: the CG sweep A time per workgroup count")
    ap.add_argument("--e1-voxels", type=int, default=1 << 20)
    ap.add_argument("--e1-iters", type=int, default=10000)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=2.0, help="serving: arrivals per second")
    ap.add_argument("--schedule-seeds", default="4000",
                    help="serving: comma-separated seeds of the arrival schedules (request mix and gaps)")
    ap.add_argument("--budget-gib", type=float, default=16.0, help="serving: HBM budget of the server (GiB)")
    ap.add_argument("--no-groups", action="store_true",
                    help="serving: the server runs every fit on its own stream (no batched groups)")
    ap.add_argument("--serve-classes", default="0,1,2,3",
                    help="serving: the size classes requests are drawn from (indices into the four sizes)")
    ap.add_argument("--ml-counters", action="store_true",
                    help="for hardware-counter runs: the whole-brain ML fit (20 Newton steps, default "
                         "initialisation) once, then exit")
    ap.add_argument("--counters", action="store_true",
                    help="for hardware-counter runs: two outer loops of one Newton step each of the MAP fit "
                         "(2 x 1 x 32; the second loop has JTV weights, so its 32 CG iterations all run, as in "
                         "the timed fit) on the same volume and a plain 1 GiB device copy as the byte-count "
                         "calibration, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the fits are single-GPU; "
              "a z-slab decomposition across GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    if args.oracle_full:
        oracle_full(args)
        return

    import torch

    from paper_2102_01604_amd import _lib, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.serving:
        serving(args, torch, _lib, synth, dev)
        return
    if args.hires:
        hires(torch, _lib, synth, dev)
        return
    if args.projected:
        projected(args, torch, _lib, synth, dev)
        return
    if args.e1:
        convergence_experiment(args, torch, _lib, synth, dev)
        return
    if args.noise:
        noise_estimation(args, torch, _lib, synth, dev)
        return
    if args.batch:
        batch_bench(torch, _lib, synth, dev)
        return
    if args.autotune:
        out = {"metric": "CG sweep A time per workgroup count (mpm_autotune)", "sizes": {}}
        for dims in SERVE_SIZES:
            r = _lib.mpm_autotune(dims, reps=10)
            out["sizes"]["x".join(str(v) for v in dims)] = r
            log(f"autotune {dims}: chose {r['workgroups'][r['chosen']]} workgroups "
                f"({r['planes_per_run'][r['chosen']]} planes each), {r['ms'][r['chosen']] * 1e3:.1f} us")
        print(json.dumps(out), flush=True)
        return
    dims = tuple(int(v) for v in args.dims.split(","))
    t0 = time.time()
    case = synth.make_case("map_brain", dims=dims)
    N = int(np.prod(dims))
    I = int(sum(case["proto"]["n_echoes"]))
    log(f"generated {dims} x {I} echoes in {time.time() - t0:.1f}s")

    truth = torch.from_numpy(case["truth"].astype(np.float32)).to(dev)
    b1 = torch.from_numpy(case["b1"].astype(np.float32)).to(dev)
    eps = torch.from_numpy(case["eps"]).to(dev)
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    X = torch.empty((I, N), dtype=tdt, device=dev)
    _lib.mpm_simulate(case["proto"], dims, truth, b1, eps, X)
    del eps
    torch.cuda.synchronize()
    log("echoes simulated on the GPU")

    lam = case["lam"]
    if args.ml_counters:
        maps = torch.empty((4, N), dtype=torch.float32, device=dev)
        _lib.mpm_fit(case["proto"], dims, X, b1, {"mode": "ml", "n_gn": 20}, maps)
        torch.cuda.synchronize()
        log("counter workload done: ML 20 GN")
        return
    if args.counters:
        maps = torch.empty((4, N), dtype=torch.float32, device=dev)
        _lib.mpm_fit(case["proto"], dims, X, b1, {"mode": "map", "n_outer": 2, "n_gn": 1, "n_cg": 32,
                                                   "max_halvings": 4, "lam": lam}, maps)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("counter workload done: MAP 2x1x32 + one 1 GiB copy")
        return
    ml_opts = {"mode": "ml", "n_gn": 20, "init": "default"}
    map_opts = {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32, "max_halvings": 4, "lam": lam,
                "init": "default"}
    maps_ml = torch.empty((4, N), dtype=torch.float32, device=dev)
    maps_map = torch.empty((4, N), dtype=torch.float32, device=dev)
    var = torch.empty((4, N), dtype=torch.float32, device=dev)
    mom = torch.empty((4, N), dtype=torch.float32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    parts = {"ml": [], "map": [], "unc": []}
    reports = {}

    def step(record):
        ev[0].record(stream)
        reports["ml"] = _lib.mpm_fit(case["proto"], dims, X, b1, ml_opts, maps_ml, stream=stream)[0]
        ev[1].record(stream)
        reports["map"] = _lib.mpm_fit(case["proto"], dims, X, b1, map_opts, maps_map, stream=stream)[0]
        ev[2].record(stream)
        _lib.mpm_uncertainty(case["proto"], dims, X, b1, map_opts, maps_map, var, mom, stream=stream)
        ev[3].record(stream)
        if record:
            ev[3].synchronize()
            parts["ml"].append(ev[0].elapsed_time(ev[1]))
            parts["map"].append(ev[1].elapsed_time(ev[2]))
            parts["unc"].append(ev[2].elapsed_time(ev[3]))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("warmup done")
    _lib.mpm_profile_reset()
    _lib.mpm_profile_enable(args.profile_every)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(True)
        log(f"step {k}: ml {parts['ml'][-1]:.1f} ms, map {parts['map'][-1]:.1f} ms, unc {parts['unc'][-1]:.1f} ms")
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    _lib.mpm_profile_enable(0)
    stats = _lib.mpm_profile_read()
    # the same MAP fit with FP16 echo storage and per-image offsets (outside the timed steps)
    f16 = None
    if args.dtype == "f32":
        X16 = torch.empty(X.shape, dtype=torch.float16, device=dev)
        off16 = _lib.mpm_pack_echoes(X, X16, stream=stream)
        o16 = dict(map_opts, echo_offset=off16)
        m16 = torch.empty((4, N), dtype=torch.float32, device=dev)
        _lib.mpm_fit(case["proto"], dims, X16, b1, dict(o16, n_outer=1, n_gn=1, n_cg=1), m16, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rep16 = _lib.mpm_fit(case["proto"], dims, X16, b1, o16, m16, stream=stream)[0]
        e1.record(stream)
        e1.synchronize()
        ms16 = e0.elapsed_time(e1)
        d16 = (m16 - maps_map).abs().amax(dim=1) / maps_map.abs().amax(dim=1)
        f16 = {"map_fit_ms": round(ms16, 3), "map_voxel_gn_iters_per_s": round(N * 80 / (ms16 * 1e-3), 1),
               "storage": "FP16 of each image minus its mean (mpm_pack_echoes)",
               "max_rel_diff_vs_f32_storage": [float(v) for v in d16.cpu()],
               "objective": rep16["objective"]}
        del X16, m16
        log(f"f16 storage MAP fit {ms16:.1f} ms")

    # achievable copy rate of a buffer the size of CG sweep A's working set, on
    # the same stream (reads + writes of a device-to-device copy)
    cg_ws = int(N * 124)
    ca = torch.empty(cg_ws // 4, dtype=torch.float32, device=dev)
    ca.fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        cb.copy_(ca)
    e1.record(stream)
    e1.synchronize()
    copy_gbps = 2.0 * cg_ws * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    torch.cuda.empty_cache()
    log(f"device copy of {cg_ws / 1e9:.2f} GB: {copy_gbps:.0f} GB/s")

    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    ml_ms, map_ms, unc_ms = (float(np.median(parts[k])) for k in ("ml", "map", "unc"))
    gn_iters = N * (ml_opts["n_gn"] + map_opts["n_outer"] * map_opts["n_gn"])
    value = gn_iters / (ms_per_step / 1e3)

    # dominant kernel: largest estimated total time (launches x mean timed duration)
    best, best_t = None, -1.0
    for name, s in stats.items():
        if s["timed"] > 0 and name != "fin":
            tot = s["launches"] * s["timed_ms"] / s["timed"]
            if tot > best_t:
                best, best_t = name, tot
    roof = None
    kernels = {}
    kernel_bytes = 0.0
    for name, s in stats.items():
        kernel_bytes += s["bytes"]
        if s["timed"] > 0:
            avg = s["timed_ms"] / s["timed"]
            bpl = s["bytes"] / max(s["launches"], 1)
            kernels[name] = {"launches": s["launches"], "avg_ms": round(avg, 5),
                             "alg_GBps": round(bpl / (avg * 1e-3) / 1e9, 1) if bpl > 0 else None}
    if best is not None:
        s = stats[best]
        avg_s = s["timed_ms"] / s["timed"] * 1e-3
        own = s["bytes"] / s["launches"]
        # byte model of one CG sweep A per voxel as planned: z, the previous
        # direction, w and the 10-entry Hessian in, p and q out (108 B); the
        # kernel itself writes no q and carries the deferred solution update
        model = MODEL_BYTES_PER_VOXEL.get(best)
        bpl = N * model if model else own
        achieved = bpl / avg_s / 1e9
        traffic = read_traffic(best)
        roof = {"bound": "hbm", "kernel": best, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": traffic, "alg_bytes_per_launch": bpl, "bytes_per_voxel_model": model,
                "kernel_bytes_per_launch": own, "achieved_on_kernel_bytes": round(own / avg_s / 1e9, 1),
                "frac_on_kernel_bytes": round(own / avg_s / 1e9 / HBM_PEAK_GBPS, 4),
                "avg_ms": round(avg_s * 1e3, 5),
                "copy_GBps_same_size": round(copy_gbps, 1),
                "frac_of_copy_rate": round(achieved / copy_gbps, 4)}
    # the ML kernel against the VALU roofline: executed lane-instructions (from
    # the committed counter summary) over its measured launch time
    ml_valu = None
    lanes = read_ml_valu()
    if lanes is not None and "ml_fit" in stats and stats["ml_fit"]["timed"] > 0:
        s_ = stats["ml_fit"]
        t_ml = s_["timed_ms"] / s_["timed"] * 1e-3
        evals = N * (ml_opts["n_gn"] + 1)
        ach = lanes * evals / t_ml / 1e12
        ml_valu = {"bound": "alu", "kernel": "ml_fit", "lanes_per_voxel_eval": lanes,
                   "achieved": round(ach, 2), "peak": round(VALU_PEAK_T, 2), "unit": "T lane-instructions/s",
                   "frac": round(ach / VALU_PEAK_T, 4), "avg_ms": round(t_ml * 1e3, 4)}
    # step level: the byte model of the whole step over the measured step time
    step_model = N * STEP_MODEL_BYTES_PER_VOXEL
    step_hbm = {"model_bytes_per_step": step_model,
                "model_GBps": round(step_model / (ms_per_step * 1e-3) / 1e9, 1),
                "model_frac": round(step_model / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "kernel_bytes_per_step": kernel_bytes / args.steps,
                "kernel_GBps": round(kernel_bytes / args.steps / (ms_per_step * 1e-3) / 1e9, 1),
                "model": "per voxel: ML 108 B; each of the 80 MAP Newton steps 8772 B (likelihood pass 168, "
                         "CG start 108, 32 CG iterations x 264, update 48); variance 164 B"}

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        cpu, cr = cpu_baseline(case, dims)
        parity = crop_parity(torch, _lib, case, cr, dev)
        log(f"crop parity vs the FP64 oracle: {parity}")

    serve = None
    if args.serving_leg:
        classes = np.arange(len(SERVE_SIZES))
        per_seed, n_map = serve_runs(torch, _lib, synth, dev, [4000], classes, 64, 2.0, 16 << 30,
                                     labels=("burst",))
        serve = {"schedule_seed": 4000, "requests": 64, "n_map": n_map[4000],
                 "sizes": [list(v) for v in SERVE_SIZES], "arrivals": "burst (all at t = 0)",
                 "max_active": 4, "hbm_budget_bytes": 16 << 30, **per_seed[4000]["burst"]}

    rm = reports["map"]
    out = {
        "metric": "voxel-iters/s (GN+JTV-CG)",
        "value": round(value, 1),
        "unit": "voxel-GN-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f32 (f16 echo storage)", "bf16": "f32 (bf16 echo storage)"}[args.dtype],
        "data": "synthetic",
        "config": {"workload": f"SPGR-ML 20 GN + SPGR+JTV-MAP 10x8x32 + Laplace variance, "
                               f"{dims[0]}x{dims[1]}x{dims[2]} grid, 8/8/6 echoes, B1 0.8-1.2",
                   "voxels": N, "echoes": I, "echo_storage": args.dtype, "ml_gn": 20,
                   "map_schedule": [10, 8, 32], "lambda": [round(v, 6) for v in lam]},
        "roofline": roof,
        "step_hbm": step_hbm,
        "ml_valu_roofline": ml_valu,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "serving_burst": serve,
        "breakdown_ms": {"ml_fit": round(ml_ms, 3), "map_fit": round(map_ms, 3), "uncertainty": round(unc_ms, 3)},
        "ml_voxel_iters_per_s": round(N * 20 / (ml_ms * 1e-3), 1),
        "map_voxel_gn_iters_per_s": round(N * 80 / (map_ms * 1e-3), 1),
        "map_voxel_cg_iters_per_s": round(N * rm["cg_done"] / (map_ms * 1e-3), 1),
        "map_report": {k: rm[k] for k in ("objective", "gn_done", "cg_done", "rejected", "degenerate_voxels",
                                          "nonfinite_voxels")},
        "map_f16_storage": f16,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


def hires(torch, _lib, synth, dev):
    """High-resolution JTV-MAP fit + Laplace variance on 51 M voxels (FP16 echoes)."""
    t0 = time.time()
    case = synth.make_case("map_hires")
    dims = case["dims"]
    N = int(np.prod(dims))
    log(f"generated {dims} in {time.time() - t0:.1f}s")
    truth = torch.from_numpy(case["truth"].astype(np.float32)).to(dev)
    b1 = torch.from_numpy(case["b1"].astype(np.float32)).to(dev)
    eps = torch.from_numpy(case["eps"]).to(dev)
    del case["eps"]
    X = torch.empty((22, N), dtype=torch.float16, device=dev)
    _lib.mpm_simulate(case["proto"], dims, truth, b1, eps, X)
    del eps
    opts = {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32, "max_halvings": 4, "lam": case["lam"]}
    maps = torch.empty((4, N), dtype=torch.float32, device=dev)
    var = torch.empty((4, N), dtype=torch.float32, device=dev)
    mom = torch.empty((4, N), dtype=torch.float32, device=dev)
    _lib.mpm_fit(case["proto"], dims, X, b1, dict(opts, n_outer=1, n_gn=1, n_cg=1), maps)  # warm-up
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    rep = _lib.mpm_fit(case["proto"], dims, X, b1, opts, maps)[0]
    ev[1].record()
    _lib.mpm_uncertainty(case["proto"], dims, X, b1, opts, maps, var, mom)
    ev[2].record()
    ev[2].synchronize()
    map_ms, unc_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    err = (maps - truth).float()
    rmse = err.pow(2).mean(dim=1).sqrt().cpu().tolist()
    sd = var.sqrt()
    out = {"metric": "voxel-iters/s (GN+JTV-CG), high-resolution MAP + uncertainty",
           "value": round(N * 80 / ((map_ms + unc_ms) * 1e-3), 1), "unit": "voxel-GN-iterations/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32 (f16 echo storage)", "data": "synthetic",
           "config": {"workload": "JTV-MAP 10x8x32 + Laplace variance, 416x384x320, 8/8/6 echoes, FP16 echoes, "
                                  "B1 0.7-1.3, sigma 2% of mean PD", "voxels": N},
           "map_fit_ms": round(map_ms, 2), "uncertainty_ms": round(unc_ms, 2),
           "map_voxel_cg_iters_per_s": round(N * rep["cg_done"] / (map_ms * 1e-3), 1),
           "report": rep, "rmse_vs_truth_log_maps": rmse,
           "median_sd_log_maps": sd.median(dim=1).values.cpu().tolist(),
           "device_footprint_GiB": round(_lib.mpm_footprint_bytes(case["proto"], dims, _lib.MPM_F16, _lib.MPM_MAP_JTV)
                                         / 2 ** 30, 2)}
    print(json.dumps(out), flush=True)


def projected(args, torch, _lib, synth, dev):
    """Spatially projected JTV-MAP fit + Laplace variance: the PDw contrast on
    the reconstruction grid, T1w and MTw acquired on grids moved by seeded
    rigid motions (up to 2 degrees and 1.5 voxels); echoes simulated on the GPU
    by reslicing the true maps into each space, plus seeded Gaussian noise."""
    t0 = time.time()
    case = synth.make_case("map_brain")
    dims = case["dims"]
    N = int(np.prod(dims))
    rng = np.random.default_rng(7102)
    spaces = [synth.identity_space(dims), synth.rigid_space(dims, dims, rng),
              synth.rigid_space(dims, (dims[0], dims[1], dims[2] - 8), rng)]
    log(f"generated {dims} in {time.time() - t0:.1f}s")
    truth = torch.from_numpy(case["truth"].astype(np.float32)).to(dev)
    b1 = torch.from_numpy(case["b1"].astype(np.float32)).to(dev)
    del case["eps"]
    ne = case["proto"]["n_echoes"]
    n_vals = sum(int(np.prod(sp["dims"])) * e for sp, e in zip(spaces, ne))
    gen = torch.Generator(device=dev)
    gen.manual_seed(7103)
    eps = torch.randn(n_vals, generator=gen, dtype=torch.float32, device=dev)
    X = torch.empty(n_vals, dtype=torch.float32, device=dev)
    _lib.mpm_simulate_projected(case["proto"], dims, spaces, truth, b1, eps, X)
    del eps
    opts = {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32, "max_halvings": 4, "lam": case["lam"]}
    maps = torch.empty((4, N), dtype=torch.float32, device=dev)
    var = torch.empty((4, N), dtype=torch.float32, device=dev)
    if args.counters:
        _lib.mpm_fit_projected(case["proto"], dims, spaces, X, b1, dict(opts, n_outer=2, n_gn=1), maps)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("counter workload done: projected MAP 2x1x32 + one 1 GiB copy")
        return
    _lib.mpm_fit_projected(case["proto"], dims, spaces, X, b1, dict(opts, n_outer=1, n_gn=1, n_cg=1), maps)
    torch.cuda.synchronize()
    _lib.mpm_profile_reset()
    _lib.mpm_profile_enable(7)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    rep = _lib.mpm_fit_projected(case["proto"], dims, spaces, X, b1, opts, maps)[0]
    ev[1].record()
    _lib.mpm_uncertainty_projected(case["proto"], dims, spaces, X, b1, opts, maps, var)
    ev[2].record()
    ev[2].synchronize()
    _lib.mpm_profile_enable(0)
    stats = _lib.mpm_profile_read()
    map_ms, unc_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    kernels = {}
    for name, s in stats.items():
        if s["timed"] > 0:
            avg = s["timed_ms"] / s["timed"]
            bpl = s["bytes"] / max(s["launches"], 1)
            kernels[name] = {"launches": s["launches"], "avg_ms": round(avg, 5),
                             "est_total_ms": round(avg * s["launches"], 2),
                             "alg_GBps": round(bpl / (avg * 1e-3) / 1e9, 1) if bpl > 0 else None}
    err = (maps - truth).float()
    inside = torch.isfinite(err).all(dim=0)
    rmse = err[:, inside].pow(2).mean(dim=1).sqrt().cpu().tolist()
    # dominant kernel (largest estimated total time, finalisers aside), as in the main workload
    best = max((k for k in kernels if k != "fin"), key=lambda k: kernels[k]["est_total_ms"])
    s_best = stats[best]
    bpl = s_best["bytes"] / s_best["launches"]
    avg_s = s_best["timed_ms"] / s_best["timed"] * 1e-3
    achieved = bpl / avg_s / 1e9
    roof = {"bound": "hbm", "kernel": best, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": read_traffic(best), "alg_bytes_per_launch": bpl,
            "avg_ms": round(avg_s * 1e3, 5)}
    out = {"metric": "voxel-iters/s (GN+JTV-CG), spatially projected MAP + uncertainty",
           "value": round(N * 80 / ((map_ms + unc_ms) * 1e-3), 1), "unit": "voxel-GN-iterations/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"projected JTV-MAP 10x8x32 + Laplace variance, recon {dims[0]}x{dims[1]}x{dims[2]}, "
                                  "8/8/6 echoes, T1w and MTw on rigidly moved grids (MTw 8 slices fewer)",
                      "voxels": N, "acquisition_voxels": [int(np.prod(sp["dims"])) for sp in spaces]},
           "map_fit_ms": round(map_ms, 2), "uncertainty_ms": round(unc_ms, 2),
           "report": rep, "rmse_vs_truth_log_maps": rmse, "roofline": roof, "kernels": kernels}
    print(json.dumps(out), flush=True)


def convergence_experiment(args, torch, _lib, synth, dev):
    """The paper's convergence experiment (Sec. 3.1) at scale: every voxel its
    own random protocol (3 contrasts x 5 echoes, the last with MT), sigma = 1,
    ML Newton-like steps from y = 0 with the Proposed, Proposed+ and plain
    Gauss-Newton loadings; per loading the time and the fraction of voxels whose
    NLL rose at some step."""
    N, its = args.e1_voxels, args.e1_iters
    rng = np.random.default_rng(2102)
    y, tr, flip, te = synth.e1_problems(N, rng)
    noise = rng.standard_normal((15, N), dtype=np.float32)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    Y, TR, FL, TE, NZ = f(y), f(tr), f(flip), f(te), f(noise)
    shape = {"n_echoes": [5, 5, 5], "mt": [0, 0, 1], "sigma": [1.0] * 15}
    X = torch.empty((15, N), dtype=torch.float32, device=dev)
    _lib.mpm_simulate_voxelwise(shape, TR, FL, TE, Y, NZ, X)
    del NZ
    maps = torch.empty((4, N), dtype=torch.float32, device=dev)
    inc = torch.empty(N, dtype=torch.int32, device=dev)
    nll = torch.empty(N, dtype=torch.float32, device=dev)
    res = {}
    if args.counters:  # one fit each, no warm-up: dispatches proposed, plus, gn, rate (plus), time (plus)
        for load in ("proposed", "plus", "gn"):
            _lib.mpm_fit_voxelwise(shape, TR, FL, TE, X, {"mode": "ml", "n_gn": its, "init": "const",
                                                          "init_const": [0.0] * 4, "loading": load}, maps, inc, nll)
        for basis in ("rate", "time"):
            _lib.mpm_fit_voxelwise(shape, TR, FL, TE, X, {"mode": "ml", "n_gn": its, "init": "const",
                                                          "init_const": [1.0, 1.0, 1.0, 0.5], "loading": "plus",
                                                          "basis": basis}, maps, inc, nll)
        torch.cuda.synchronize()
        log("counter workload done: five voxelwise fits")
        return
    for load in ("proposed", "plus", "gn"):
        opts = {"mode": "ml", "n_gn": its, "init": "const", "init_const": [0.0] * 4, "loading": load}
        _lib.mpm_fit_voxelwise(shape, TR, FL, TE, X, dict(opts, n_gn=1), maps, inc, nll)  # warm-up
        torch.cuda.synchronize()
        e0, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rep = _lib.mpm_fit_voxelwise(shape, TR, FL, TE, X, opts, maps, inc, nll)
        e1_.record()
        e1_.synchronize()
        ms = e0.elapsed_time(e1_)
        rose = (inc > 0).float().mean().item()
        res[load] = {"ms": round(ms, 2), "voxel_iters_per_s": round(N * its / (ms * 1e-3), 1),
                     "frac_voxels_nll_rose": round(rose, 5), "mean_rises_per_voxel": round(rep["nll_increases"] / N, 3),
                     "frac_nonfinite": round(rep["nonfinite_voxels"] / N, 5)}
        log(f"e1 {load}: {ms:.1f} ms, NLL rose in {100 * rose:.2f}% of voxels")
    reps = representation_comparison(args, torch, _lib, shape, TR, FL, TE, X, maps, inc, nll)
    counts = read_valu_counts()
    for b, key in (("log", "plus"), ("rate", "rate"), ("time", "time")):
        if counts is not None and key in counts:
            evals = N * (its + len(reps[b]["steps"]))  # each call evaluates its steps + 1 times
            ach = counts[key] * evals / (reps[b]["ms"] * 1e-3) / 1e12
            reps[b]["roofline"] = {"bound": "alu", "achieved": round(ach, 2), "peak": round(VALU_PEAK_T, 2),
                                   "unit": "T VALU lane-instructions/s", "frac": round(ach / VALU_PEAK_T, 4),
                                   "valu_per_voxel_iteration": counts[key]}
    cpu = None
    if not args.no_cpu_baseline:
        # the FP64 oracle on the first 32768 voxels of the same problems, 8000 steps, Proposed loading
        import oracle
        n_s, it_s = 32768, 8000
        xs = X[:, :n_s].cpu().numpy().astype(np.float64)
        t = time.perf_counter()
        with np.errstate(all="ignore"):
            oracle.fit_voxelwise(shape, tr[:, :n_s].astype(np.float32), flip[:, :n_s].astype(np.float32),
                                 te[:, :n_s].astype(np.float32), xs, {"n_gn": it_s, "init": "const",
                                                                      "init_const": [0.0] * 4})
        dt = time.perf_counter() - t
        cpu = {"value": round(n_s * it_s / dt, 1), "unit": "voxel-iterations/s", "cores": oracle.num_threads(),
               "kind": "oracle", "seconds": round(dt, 2),
               "sample": f"the first {n_s} voxels of the same problems, {it_s} steps, Proposed loading, FP64"}
    roof = None
    if counts is not None:
        ach = counts["proposed"] * N * (its + 1) / (res["proposed"]["ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "ml_fit_pv", "achieved": round(ach, 2), "peak": round(VALU_PEAK_T, 2),
                "unit": "T VALU lane-instructions/s", "frac": round(ach / VALU_PEAK_T, 4), "traffic": None,
                "valu_per_voxel_iteration": counts["proposed"]}
    out = {"metric": "voxel-iterations/s (ML, a protocol per voxel: the Sec. 3.1 convergence experiment)",
           "value": res["proposed"]["voxel_iters_per_s"], "unit": "voxel-iterations/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{N} voxels, each with its own random protocol (3 contrasts x 5 echoes, MT on the "
                                  f"last; log TR, log TE, log-parameters ~ U[-5, 5], flips ~ U[0, pi/4]), sigma 1, "
                                  f"{its} ML steps from 0", "voxels": N, "iterations": its},
           "loadings": res, "representations": reps, "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def representation_comparison(args, torch, _lib, shape, TR, FL, TE, X, maps, inc, nll):
    """Sec. 3.1 representation comparison on the same problems: the steps act
    on the log/logit parameters, on (A, R1, R2*, MTsat) or on (A, T1, T2*,
    MTsat), all with the |H| 1 (Proposed+) loading and from the point
    log-parameters 0 give; the NLL of every voxel is read after 100, 1000 and
    all steps (the fit continues from its maps), and compared with the lowest
    final NLL any basis reached for that voxel."""
    its = args.e1_iters
    marks = [m for m in (100, 1000) if m < its] + [its]
    finals, out = {}, {}
    for basis, start in (("log", [0.0] * 4), ("rate", [1.0, 1.0, 1.0, 0.5]), ("time", [1.0, 1.0, 1.0, 0.5])):
        base = {"mode": "ml", "loading": "plus", "basis": basis}
        _lib.mpm_fit_voxelwise(shape, TR, FL, TE, X, dict(base, n_gn=1, init="const", init_const=start), maps, inc,
                               nll)  # warm-up
        torch.cuda.synchronize()
        done, ms, rows = 0, 0.0, []
        for m in marks:
            o = dict(base, n_gn=m - done, **({"init": "const", "init_const": start} if done == 0 else {"init": "maps"}))
            e0, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _lib.mpm_fit_voxelwise(shape, TR, FL, TE, X, o, maps, inc, nll)
            e1_.record()
            e1_.synchronize()
            ms += e0.elapsed_time(e1_)
            rows.append(nll.double().clone())
            done = m
        finals[basis] = rows
        th = maps
        fin = torch.isfinite(th).all(dim=0)
        entry = {"ms": round(ms, 2), "voxel_iters_per_s": round(X.shape[1] * its / (ms * 1e-3), 1),
                 "frac_finite": round(fin.double().mean().item(), 5)}
        if basis != "log":
            # the closed domain: repeated halving ends exactly on a boundary in FP32 (A = 0, MTsat = 1)
            inside = (th[:3] >= 0).all(dim=0) & (th[3] >= 0) & (th[3] <= 1)
            at_edge = (th[:3] == 0).any(dim=0) | (th[3] == 0) | (th[3] == 1)
            entry["closed_domain_kept"] = bool((inside | ~fin).all().item())
            entry["frac_on_boundary"] = round(at_edge.double().mean().item(), 5)
        out[basis] = entry
    best = torch.stack([finals[b][-1] for b in finals]).min(dim=0).values
    for b in finals:
        ex = [((r - best) / best.abs()) for r in finals[b]]
        out[b]["steps"] = marks
        out[b]["median_rel_nll_excess"] = [float(f"{e.nanmedian().item():.3e}") for e in ex]
        out[b]["frac_within_1e-6_of_best"] = round((ex[-1] <= 1e-6).double().mean().item(), 4)
        log(f"e1 basis {b}: {out[b]['ms']:.1f} ms, median NLL excess {out[b]['median_rel_nll_excess']}")
    return out


def noise_estimation(args, torch, _lib, synth, dev):
    """Sec. 2.7 noise estimation on the whole-brain volume (192 x 240 x 256,
    8/8/6 echoes, FP32) placed in air: the head an ellipsoid over 80% of each
    axis, no signal outside, magnitudes |s + sigma (e1 + i e2)| with sigma 2%
    of the head's mean PD (complex Gaussian noise drawn on the GPU, seeded).
    A step is one mpm_estimate_noise call (1024 bins, 200 EM iterations)."""
    dims = (192, 240, 256)
    c = synth.make_case("map_brain", dims=dims)
    N, I = int(np.prod(dims)), int(sum(c["proto"]["n_echoes"]))
    mask_np = synth.head_mask(dims)
    sigma = 0.02 * float(np.exp(c["truth"][0][mask_np]).mean())
    truth = torch.from_numpy(c["truth"].astype(np.float32)).to(dev)
    b1 = torch.from_numpy(c["b1"].astype(np.float32)).to(dev)
    mask = torch.from_numpy(mask_np).to(dev)
    X = torch.empty((I, N), dtype=torch.float32, device=dev)
    _lib.mpm_simulate(c["proto"], dims, truth, b1, None, X)
    g = torch.Generator(device=dev).manual_seed(2107)
    for i in range(I):  # input synthesis (plumbing): Rician magnitudes, image by image
        e1 = torch.randn(N, generator=g, device=dev)
        e2 = torch.randn(N, generator=g, device=dev)
        X[i] = torch.hypot(torch.where(mask, X[i], 0.0) + sigma * e1, sigma * e2)
    del e1, e2, truth
    torch.cuda.synchronize()
    log(f"noise workload: {dims} x {I} magnitude images in air, sigma {sigma:.3f}")
    if args.counters:  # one estimate, then a plain 1 GiB device copy as the byte-count calibration
        _lib.mpm_estimate_noise(c["proto"], dims, X, b1)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("counter workload done: one noise estimate and a 1 GiB copy")
        return
    for _ in range(args.warmup):
        _lib.mpm_estimate_noise(c["proto"], dims, X, b1)
    torch.cuda.synchronize()
    _lib.mpm_profile_reset()
    _lib.mpm_profile_enable(1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        est = _lib.mpm_estimate_noise(c["proto"], dims, X, b1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.mpm_profile_enable(0)
    stats = _lib.mpm_profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    kern = {k: {"launches": v["launches"], "avg_ms": round(v["timed_ms"] / max(v["timed"], 1), 5),
                "alg_GBps": round(v["bytes"] / v["launches"] / (v["timed_ms"] / v["timed"] * 1e-3) / 1e9, 1)
                if v["bytes"] > 0 and v["timed"] else None}
            for k, v in stats.items()}
    dom = max(("image_max", "image_hist"), key=lambda k: kern[k]["avg_ms"])
    alg = float(N) * I * 4.0
    ach = alg / (kern[dom]["avg_ms"] * 1e-3) / 1e9
    traffic = read_traffic(dom, NOISE_TRAFFIC_FILE, NOISE_SOURCES)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(ach / 8000.0, 4), "traffic": traffic, "alg_bytes_per_launch": alg,
            "avg_ms": kern[dom]["avg_ms"],
            "note": "the streaming pass over the echoes; the EM (rice_em) is a chain of dependent iterations, "
                    "one workgroup per image, bound by its FP64 latency on 22 CUs, not by a roofline"}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        z = 64  # a slab of 64 planes of the same volume (all 22 images)
        xs = X[:, : dims[0] * dims[1] * z].cpu().numpy().astype(np.float64)
        b1s = c["b1"][: dims[0] * dims[1] * z].astype(np.float32).astype(np.float64)
        t = time.perf_counter()
        oracle.estimate_noise(c["proto"], xs, b1s)
        dt = time.perf_counter() - t
        cpu = {"value": round(xs.size / dt, 1), "unit": "image-voxels/s", "cores": 1, "kind": "oracle",
               "seconds": round(dt, 2), "sample": f"the first {z} planes of the same volume ({xs.shape[1]} voxels "
                                                  f"x {I} images), 1024 bins, 200 EM iterations, FP64"}
    out = {"metric": "image-voxels/s (noise estimation: histogram + two-class Rician mixture per image)",
           "value": round(N * I / (ms * 1e-3), 1), "unit": "image-voxels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "dtype": "f32 / f64 EM",
           "data": "synthetic",
           "config": {"workload": "192x240x256 whole-brain volume in air (ellipsoid head), 8/8/6 echoes, Rician "
                                  "noise 2% of the head's mean PD, 1024 bins, 200 EM iterations",
                      "voxels": N, "images": I},
           "sigma_true": sigma, "sigma_contrast": est["sigma_contrast"],
           "kernels": kern, "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


SERVE_SIZES = [(64, 64, 64), (96, 128, 128), (128, 160, 160), (192, 240, 256)]


def batch_bench(torch, _lib, synth, dev):
    """JTV-MAP fits of several small volumes (the serving sizes 64^3 and
    96 x 128 x 128, each its own seeded noise) one after another with mpm_fit
    and together with mpm_fit_batch; the maps must be identical."""
    res = {}
    for dims, n in (((64, 64, 64), 16), ((96, 128, 128), 4)):
        c = synth.make_case("map_brain", dims=dims, seed=4100)
        del c["eps"]
        N = int(np.prod(dims))
        truth = torch.from_numpy(c["truth"].astype(np.float32)).to(dev)
        b1 = torch.from_numpy(c["b1"].astype(np.float32)).to(dev)
        opts = {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32, "max_halvings": 4, "lam": c["lam"]}
        Xs = []
        for r in range(n):
            g = torch.Generator(device=dev).manual_seed(9000 + r)
            eps = torch.randn((22, N), generator=g, device=dev)
            X = torch.empty((22, N), dtype=torch.float32, device=dev)
            _lib.mpm_simulate(c["proto"], dims, truth, b1, eps, X)
            Xs.append(X)
        del eps
        warm = torch.empty((4, N), device=dev)
        _lib.mpm_fit(c["proto"], dims, Xs[0], b1, dict(opts, n_outer=1, n_gn=1, n_cg=2), warm)
        _lib.mpm_fit_batch([(c["proto"], dims, X, b1, dict(opts, n_outer=1, n_gn=1, n_cg=2), torch.empty((4, N), device=dev))
                            for X in Xs[:2]])
        torch.cuda.synchronize()
        serial = [torch.empty((4, N), device=dev) for _ in range(n)]
        t0 = time.perf_counter()
        for X, m in zip(Xs, serial):
            _lib.mpm_fit(c["proto"], dims, X, b1, opts, m)
        torch.cuda.synchronize()
        t_serial = time.perf_counter() - t0
        batched = [torch.empty((4, N), device=dev) for _ in range(n)]
        t0 = time.perf_counter()
        reps = _lib.mpm_fit_batch([(c["proto"], dims, X, b1, opts, m) for X, m in zip(Xs, batched)])
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        same = all(bool(torch.equal(a, b)) for a, b in zip(serial, batched))
        iters = n * N * 80
        key = "x".join(str(v) for v in dims)
        res[key] = {"fits": n, "serial_s": round(t_serial, 4), "batched_s": round(t_batch, 4),
                    "serial_voxel_gn_iters_per_s": round(iters / t_serial, 1),
                    "batched_voxel_gn_iters_per_s": round(iters / t_batch, 1),
                    "speedup": round(t_serial / t_batch, 3), "maps_identical": same,
                    "gn_done": [r[0]["gn_done"] for r in reps]}
        log(f"batch {key} x {n}: serial {t_serial:.3f} s, batched {t_batch:.3f} s, identical {same}")
        del Xs, serial, batched
        torch.cuda.empty_cache()
    out = {"metric": "batched JTV-MAP fits vs one at a time (voxel-GN-iterations/s)",
           "value": res["64x64x64"]["batched_voxel_gn_iters_per_s"], "unit": "voxel-GN-iterations/s",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "JTV-MAP 10x8x32 of 16 volumes of 64^3 and of 4 volumes of 96x128x128, 22 "
                                  "echoes, FP32 storage, each volume its own noise"},
           "batch": res}
    print(json.dumps(out), flush=True)


def serve_runs(torch, _lib, synth, dev, seeds, classes, n, rate, budget, labels=("poisson", "burst"),
               groups=True):
    """Continuous batching against serial plain fits on the same arrival
    schedules, for each schedule seed.  Each size class has one seeded tissue
    volume; each request draws its own noise (seeded) on the GPU; all inputs
    are resident in HBM before the clock starts.  Returns (per-seed results,
    MAP request count per seed)."""
    vols = {}
    for k, dims in enumerate(SERVE_SIZES):
        if k not in classes:
            continue
        c = synth.make_case("map_brain", dims=dims, seed=4100 + k)
        del c["eps"]
        vols[k] = {"case": c, "truth": torch.from_numpy(c["truth"].astype(np.float32)).to(dev),
                   "b1": torch.from_numpy(c["b1"].astype(np.float32)).to(dev)}
    log(f"serving: generated {len(vols)} volume classes")

    def make_requests(seed):
        rng = np.random.default_rng(seed)
        cls = classes[rng.integers(0, len(classes), n)]
        is_map = rng.random(n) < 0.5
        gaps = rng.exponential(1.0 / rate, n)
        arrive = np.cumsum(gaps) - gaps[0]
        reqs = []
        for r in range(n):
            v = vols[int(cls[r])]
            c = v["case"]
            dims = c["dims"]
            N = int(np.prod(dims))
            g = torch.Generator(device=dev).manual_seed(seed * 1000 + r)
            eps = torch.randn((22, N), generator=g, device=dev)
            X = torch.empty((22, N), dtype=torch.float32, device=dev)
            _lib.mpm_simulate(c["proto"], dims, v["truth"], v["b1"], eps, X)
            del eps
            opts = ({"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32, "max_halvings": 4, "lam": c["lam"]}
                    if is_map[r] else {"mode": "ml", "n_gn": 20})
            reqs.append({"proto": c["proto"], "dims": dims, "X": X, "b1": v["b1"], "opts": opts, "N": N,
                         "iters": N * (80 if is_map[r] else 20)})
        torch.cuda.synchronize()
        return reqs, arrive, int(is_map.sum())

    def run_serial(reqs, times):
        outs, done = [], np.zeros(n)
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            now = time.perf_counter() - t0
            if now < times[i]:
                time.sleep(times[i] - now)
            o = torch.empty((4, r["N"]), device=dev)
            _lib.mpm_fit(r["proto"], r["dims"], r["X"], r["b1"], r["opts"], o)
            done[i] = time.perf_counter() - t0
            outs.append(o)
        return outs, done

    def run_batched(reqs, times):
        outs = [torch.empty((4, r["N"]), device=dev) for r in reqs]
        done = np.full(n, np.nan)
        tickets = [None] * n
        srv = _lib.MpmServer(hbm_budget=budget, max_active=4, groups=groups)
        t0 = time.perf_counter()
        nxt = 0
        while np.isnan(done).any():
            now = time.perf_counter() - t0
            while nxt < n and times[nxt] <= now:
                r = reqs[nxt]
                tickets[nxt] = srv.submit(r["proto"], r["dims"], r["X"], r["b1"], r["opts"], outs[nxt])
                nxt += 1
            srv.step()
            now = time.perf_counter() - t0
            for i in range(nxt):
                if np.isnan(done[i]) and srv.poll(tickets[i]) is not None:
                    done[i] = now
            time.sleep(0.0002)
        srv.close()
        return outs, done

    nr = lambda v, q: float(np.sort(v)[max(0, int(np.ceil(q * len(v))) - 1)])  # nearest rank
    per_seed, n_map = {}, {}
    for seed in seeds:
        reqs, arrive, n_map[seed] = make_requests(seed)
        if seed == seeds[0]:  # warm-up: one small fit of each mode
            small = min(range(n), key=lambda i: reqs[i]["N"])
            for mode in ("ml", "map"):
                r = reqs[small]
                o = torch.empty((4, r["N"]), device=dev)
                _lib.mpm_fit(r["proto"], r["dims"], r["X"], r["b1"],
                             dict(r["opts"], mode=mode, lam=r["opts"].get("lam", [1e-3] * 4), n_outer=1, n_gn=1,
                                  n_cg=2), o)
            torch.cuda.synchronize()
        log(f"serving seed {seed}: {n} requests resident ({sum(r['N'] for r in reqs) / 1e6:.1f} M voxels)")
        res = {}
        for label in labels:
            times = arrive if label == "poisson" else np.zeros(n)
            so, sd = run_serial(reqs, times)
            torch.cuda.synchronize()
            bo, bd = run_batched(reqs, times)
            torch.cuda.synchronize()
            lat_s, lat_b = sd - times, bd - times
            diff = max(float((a - b).abs().max()) for a, b in zip(so, bo))
            iters = sum(r["iters"] for r in reqs)
            res[label] = {
                "serial": {"p50_s": round(nr(lat_s, 0.5), 3), "p99_s": round(nr(lat_s, 0.99), 3),
                           "makespan_s": round(float(sd.max()), 3),
                           "voxel_iters_per_s": round(iters / float(sd.max()), 1)},
                "batched": {"p50_s": round(nr(lat_b, 0.5), 3), "p99_s": round(nr(lat_b, 0.99), 3),
                            "makespan_s": round(float(bd.max()), 3),
                            "voxel_iters_per_s": round(iters / float(bd.max()), 1)},
                "throughput_batched_over_serial": round(float(sd.max()) / float(bd.max()), 3),
                "max_abs_map_diff_batched_vs_serial": diff,
            }
            log(f"serving seed {seed} {label}: {res[label]}")
            del so, bo
        per_seed[seed] = res
        del reqs
        torch.cuda.empty_cache()
    return per_seed, n_map


def serving(args, torch, _lib, synth, dev):
    """The serving benchmark: one JSON line over every schedule seed."""
    seeds = [int(v) for v in args.schedule_seeds.split(",")]
    n = args.requests
    classes = np.array([int(v) for v in args.serve_classes.split(",")])
    budget = int(args.budget_gib * (1 << 30))
    per_seed, n_map = serve_runs(torch, _lib, synth, dev, seeds, classes, n, args.rate, budget,
                                 groups=not args.no_groups)
    med = lambda f: round(float(np.median([f(per_seed[s_]) for s_ in seeds])), 3)
    summary = {lab: {kind: {q: med(lambda r, lab=lab, kind=kind, q=q: r[lab][kind][q])
                            for q in ("p50_s", "p99_s", "makespan_s")} for kind in ("serial", "batched")}
               for lab in ("poisson", "burst")}
    out = {"metric": "p50/p99 fit latency, batched vs plain (serving)",
           "value": summary["poisson"]["batched"]["p99_s"],
           "unit": "s (p99 latency, batched; median over schedules)", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic",
           "config": {"workload": f"{n} fit requests, sizes uniform over {[SERVE_SIZES[k] for k in classes]}, "
                                  f"22 echoes, ML (20 GN) or "
                                  f"JTV-MAP (10x8x32) with p=0.5, Poisson arrivals {args.rate}/s; burst = all at t=0",
                      "max_active": 4, "hbm_budget_bytes": budget, "schedule_seeds": seeds,
                      "n_map": n_map, "batched_groups": not args.no_groups},
           "serving_median_over_schedules": summary,
           "serving": {str(k): v for k, v in per_seed.items()}}
    print(json.dumps(out), flush=True)


def crop(case, dims, c):
    """The central c^3 crop of the volume as its own volume: (dims, voxel
    indices, echoes made by the oracle's forward model plus the case's noise
    (FP32 values, widened), b1 (FP32, widened), truth)."""
    import oracle
    nx, ny, nz = dims
    cx, cy, cz = (min(c, nx), min(c, ny), min(c, nz))
    x0, y0, z0 = (nx - cx) // 2, (ny - cy) // 2, (nz - cz) // 2
    idx = (np.arange(z0, z0 + cz)[:, None, None] * ny + np.arange(y0, y0 + cy)[None, :, None]) * nx \
        + np.arange(x0, x0 + cx)[None, None, :]
    idx = idx.reshape(-1)
    truth = case["truth"][:, idx]
    b1 = case["b1"][idx].astype(np.float32).astype(np.float64)
    s = oracle.simulate(case["proto"], truth, b1)
    x = (s + case["sigma"] * case["eps"][:, idx].astype(np.float64)).astype(np.float32).astype(np.float64)
    return (cx, cy, cz), idx, np.ascontiguousarray(x), b1, np.ascontiguousarray(truth)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_stages(case, cd, x, b1, lam):
    """The oracle's three stages on one volume; returns (seconds, ML maps, MAP maps)."""
    import oracle
    t = time.perf_counter()
    ml, _, _ = oracle.fit(case["proto"], cd, x, b1, {"mode": "ml", "n_gn": 20})
    maps, rep, _ = oracle.fit(case["proto"], cd, x, b1, {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32,
                                                        "max_halvings": 4, "lam": lam})
    oracle.uncertainty(case["proto"], cd, x, b1, {"mode": "map", "lam": lam}, maps, moments=True)
    return time.perf_counter() - t, ml, maps


def cpu_baseline(case, dims):
    """The FP64 oracle on a bounded sample of the same workload: the central
    40^3 crop fitted as its own volume with the same three stages on every
    host thread, and the central 20^3 crop on one thread.  Also returns the
    40^3 crop and the oracle's maps, for the GPU's parity leg."""
    import oracle
    lam = case["lam"]
    cd, idx, x, b1, truth = crop(case, dims, 40)
    threads = oracle.num_threads()
    dt, ml, mp = oracle_stages(case, cd, x, b1, lam)
    n = len(idx)
    cd1, idx1, x1, b11, _ = crop(case, dims, 20)
    oracle.set_num_threads(1)
    try:
        dt1, _, _ = oracle_stages(case, cd1, x1, b11, lam)
    finally:
        oracle.set_num_threads(threads)
    rec = {"value": round(n * 100 / dt, 1), "unit": "voxel-GN-iterations/s", "cores": threads,
           "kind": "oracle", "seconds": round(dt, 2), "cpu_model": cpu_model(),
           "sample": f"central {cd[0]}x{cd[1]}x{cd[2]} crop ({n} voxels) of the same volume, fitted as its own "
                     "volume: ML 20 GN + MAP 10x8x32 + variance, FP64",
           "one_thread": {"value": round(len(idx1) * 100 / dt1, 1), "unit": "voxel-GN-iterations/s", "cores": 1,
                          "seconds": round(dt1, 2),
                          "sample": f"central {cd1[0]}x{cd1[1]}x{cd1[2]} crop ({len(idx1)} voxels), "
                                    "the same three stages"}}
    if os.path.exists(ORACLE_FULL_FIT):
        g = json.load(open(ORACLE_FULL_FIT))
        if tuple(g["dims"]) == tuple(dims):
            nv = int(np.prod(dims))
            o = g["options"]
            rec["full_size_map_fit"] = {
                "value": round(nv * o["n_outer"] * o["n_gn"] / g["oracle_fit_seconds"], 1),
                "unit": "voxel-GN-iterations/s", "cores": g["oracle_threads"], "seconds": g["oracle_fit_seconds"],
                "sample": "the whole volume, MAP 10x8x32 alone, FP64, timed once on the host that wrote "
                          "tests/golden/whole_brain_map_10x8x32.json (not this one)"}
    return rec, {"dims": cd, "x": x, "b1": b1, "truth": truth, "ml": ml, "map": mp}


def oracle_full(args):
    """The FP64 oracle on the whole benchmark volume (the timed step's three
    stages, default initialisation), each stage timed: the CPU baseline at full
    size.  Runs on the host only."""
    import oracle
    from paper_2102_01604_amd import synth
    dims = tuple(int(v) for v in args.dims.split(","))
    case = synth.make_case("map_brain", dims=dims)
    N = int(np.prod(dims))
    log(f"oracle at full size: {dims}, {oracle.num_threads()} threads")
    b1 = case["b1"].astype(np.float32).astype(np.float64)
    x = np.empty((len(case["proto"]["te"]), N))
    step = 1 << 21
    for s0 in range(0, N, step):
        sl = slice(s0, min(N, s0 + step))
        sim = oracle.simulate(case["proto"], case["truth"][:, sl], b1[sl])
        x[:, sl] = (sim + case["sigma"] * case["eps"][:, sl].astype(np.float64)).astype(np.float32)
    del case["eps"]
    lam = case["lam"]
    t = {}
    t0 = time.perf_counter()
    oracle.fit(case["proto"], dims, x, b1, {"mode": "ml", "n_gn": 20})
    t["ml_s"] = time.perf_counter() - t0
    log(f"ML {t['ml_s']:.1f} s")
    t0 = time.perf_counter()
    maps, rep, _ = oracle.fit(case["proto"], dims, x, b1, {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32,
                                                          "max_halvings": 4, "lam": lam})
    t["map_s"] = time.perf_counter() - t0
    log(f"MAP {t['map_s']:.1f} s")
    t0 = time.perf_counter()
    oracle.uncertainty(case["proto"], dims, x, b1, {"mode": "map", "lam": lam}, maps, moments=True)
    t["var_s"] = time.perf_counter() - t0
    total = t["ml_s"] + t["map_s"] + t["var_s"]
    out = {"metric": "voxel-iters/s (GN+JTV-CG), FP64 oracle at full size", "value": round(N * 100 / total, 1),
           "unit": "voxel-GN-iterations/s", "cores": oracle.num_threads(), "cpu_model": cpu_model(),
           "kind": "oracle", "seconds": {k: round(v, 1) for k, v in t.items()}, "total_s": round(total, 1),
           "map_voxel_cg_iters_per_s": round(N * rep["cg_done"] / t["map_s"], 1), "map_report": rep,
           "config": {"workload": f"SPGR-ML 20 GN + SPGR+JTV-MAP 10x8x32 + Laplace variance, "
                                  f"{dims[0]}x{dims[1]}x{dims[2]} grid, 8/8/6 echoes, B1 0.8-1.2", "voxels": N}}
    print(json.dumps(out), flush=True)


def map_error(gpu, orc, truth):
    """max_n |gpu - orc| / max_n |orc| per map (relative on log maps), over all
    voxels and over the well-posed ones (oracle within 1 of the truth)."""
    gpu = np.asarray(gpu, np.float64)
    d = np.abs(gpu - orc)
    sc = np.maximum(np.abs(orc).max(axis=1), 1e-30)
    good = np.all(np.abs(orc - truth) < 1.0, axis=0)
    return {"all_voxels": [float(v) for v in d.max(axis=1) / sc],
            "well_posed": [float(v) for v in d[:, good].max(axis=1) / sc], "well_posed_frac": float(good.mean())}


def crop_parity(torch, _lib, case, cr, dev):
    """The GPU's fits of the oracle's crop (default initialisation, the
    benchmark's options) with FP32 echoes and with FP16 echoes stored with
    per-image offsets, against the oracle's FP64 maps of the unquantised data."""
    cd, x, b1, truth = cr["dims"], cr["x"], cr["b1"], cr["truth"]
    N = x.shape[1]
    X = torch.from_numpy(x.astype(np.float32)).to(dev)
    B1 = torch.from_numpy(b1.astype(np.float32)).to(dev)
    Q = torch.empty(X.shape, dtype=torch.float16, device=dev)
    off = _lib.mpm_pack_echoes(X, Q)
    ml_opts = {"mode": "ml", "n_gn": 20}
    map_opts = {"mode": "map", "n_outer": 10, "n_gn": 8, "n_cg": 32, "max_halvings": 4, "lam": case["lam"]}
    out = {}
    for name, E, extra in (("f32", X, {}), ("f16_offsets", Q, {"echo_offset": off})):
        m = torch.empty((4, N), dtype=torch.float32, device=dev)
        _lib.mpm_fit(case["proto"], cd, E, B1, dict(ml_opts, **extra), m)
        ml = m.cpu().numpy()
        _lib.mpm_fit(case["proto"], cd, E, B1, dict(map_opts, **extra), m)
        mp = m.cpu().numpy()
        out[name] = {"ml": map_error(ml, cr["ml"], truth), "map": map_error(mp, cr["map"], truth)}
    out["tolerance"] = {"f32": 1e-4, "f16_offsets": 1e-3}
    out["sample"] = f"the cpu_baseline crop {cd[0]}x{cd[1]}x{cd[2]}, default initialisation on both sides"
    return out


if __name__ == "__main__":
    main()
