"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2102_01604_amd.profile_summary trace <run_kernel_stats.csv>
    python -m paper_2102_01604_amd.profile_summary traffic <FETCH run_counter_collection.csv>
                                                   <WRITE run_counter_collection.csv> <kernel> <voxels> [last]

    python -m paper_2102_01604_amd.profile_summary valu <run_counter_collection.csv> <kernel> <voxels> <steps>
    python -m paper_2102_01604_amd.profile_summary counters <run_counter_collection.csv> <kernel> [last]

`trace` prints a markdown table of per-kernel call counts and durations.
`valu` prints the executed VALU instructions (SQ_INSTS_VALU, per wavefront,
so x 64 lanes) and transcendental ones (SQ_INSTS_VALU_TRANS_F32) per voxel
and evaluation, for each dispatch of a voxelwise kernel that evaluates the
likelihood steps + 1 times per voxel, tagged with the hash of the voxel
kernel sources.
`counters` prints the mean per dispatch of every counter a run collected for
one kernel.
`traffic` prints the HBM bytes per dispatch of one kernel (averaged over its
last `last` dispatches, default all): FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) scaled by what the same counters read for a
plain device-to-device copy of 1 GiB in the same run (the copy kernel whose
name contains "copyBuffer" with the largest FETCH_SIZE), in the key: value
format bench.py reads, tagged with the hash of the kernel's sources (the MAP
kernels', or the noise kernels' for image_hist / image_max).
"""
from __future__ import annotations

import csv
import hashlib
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("k_map.hip", "mpm_map.h", "mpm_device.h", "mpm_kernels.h", "mpm_tune.hip")]


def _short(name):
    return name.split("(")[0].replace("void ", "")


def trace(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for r in rows:
        print(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")


def _counter(path):
    out = {}
    for r in csv.DictReader(open(path)):
        out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


NOISE_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("k_noise.hip", "mpm_noise.h", "mpm_device.h")]
# kernels whose summaries are tagged with the hash of other sources than the MAP kernels'
SOURCES_BY_KERNEL = {"image_hist": NOISE_SOURCES, "image_max": NOISE_SOURCES}


def traffic(fetch_csv, write_csv, kernel, voxels, last=0):
    f, w = _counter(fetch_csv), _counter(write_csv)
    copy = [k for k in f if "copyBuffer" in k]
    cf = max((v for k in copy for v in f[k]))
    cw = max((v for k in copy for v in w[k]))
    gib_kib = 1024.0 * 1024.0
    fs, ws = gib_kib / cf, gib_kib / cw
    name = [k for k in f if k.endswith(kernel) or k.split("<")[0].endswith(kernel)][0]
    fv, wv = f[name][-last:] if last else f[name], w[name][-last:] if last else w[name]
    fk, wk = statistics.mean(fv), statistics.mean(wv)
    b = (fk * fs + wk * ws) * 1024.0
    h = hashlib.sha256()
    for p in SOURCES_BY_KERNEL.get(kernel, KERNEL_SOURCES):
        h.update(open(p, "rb").read())
    src = h.hexdigest()[:16]
    print(f"kernel: {kernel}")
    print(f"dispatches: {len(fv)} (of {len(f[name])})")
    print(f"fetch_kib_min_max: {min(fv):.1f} {max(fv):.1f}")
    print(f"fetch_kib_per_dispatch: {fk:.1f}")
    print(f"write_kib_per_dispatch: {wk:.1f}")
    print(f"copy_calibration_fetch_kib_for_1gib: {cf:.1f}")
    print(f"copy_calibration_write_kib_for_1gib: {cw:.1f}")
    print(f"fetch_scale: {fs:.4f}")
    print(f"write_scale: {ws:.4f}")
    print(f"bytes_per_launch: {b:.0f}")
    print(f"bytes_per_voxel: {b / voxels:.1f}")
    print(f"source_sha256_16: {src}")


VALU_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("k_voxel.hip", "mpm_voxelwise.h", "mpm_device.h")]


def valu(csv_path, kernel, voxels, steps):
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if _short(r["Kernel_Name"]).split("<")[0].endswith(kernel):
            per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    h = hashlib.sha256()
    for p in VALU_SOURCES:
        h.update(open(p, "rb").read())
    evals = float(voxels) * (steps + 1)
    print(f"kernel: {kernel}")
    print(f"dispatches: {len(next(iter(per.values())))}")
    for c in sorted(per):
        for d, v in enumerate(per[c]):
            print(f"{c}_dispatch{d}: {v:.6g}")
            if c.startswith("SQ_INSTS_VALU"):
                print(f"{c}_dispatch{d}_lanes_per_voxel_eval: {v * 64.0 / evals:.2f}")
    print(f"source_sha256_16: {h.hexdigest()[:16]}")


def counters(csv_path, kernel, last=0):
    """Mean value per dispatch of every counter of one kernel (its last `last`
    dispatches, default all)."""
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if _short(r["Kernel_Name"]).split("<")[0].endswith(kernel):
            per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    print(f"kernel: {kernel}")
    for c in sorted(per):
        v = per[c][-last:] if last else per[c]
        print(f"{c}_dispatches: {len(v)}")
        print(f"{c}_per_dispatch: {statistics.mean(v):.6g}")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif sys.argv[1] == "valu":
        valu(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5]))
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], int(sys.argv[4]) if len(sys.argv) > 4 else 0)
    else:
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]) if len(sys.argv) > 6 else 0)
