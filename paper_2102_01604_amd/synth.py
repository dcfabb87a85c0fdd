"""Seeded synthetic inputs shaped like the paper's multi-parameter mapping data.

This module only draws random numbers and arranges them; it contains none of
the fitting method's arithmetic (no signal equation, derivative or solve).  The
noise-free echoes are made by a forward model elsewhere: ``x = s(maps) +
sigma * eps`` where ``eps`` comes from here.

Stand-in for the paper's two 0.8 mm MPM datasets (Sec. 3.2), which are not
available: three SPGR contrasts (PDw 6 deg, T1w 21 deg, MTw 6 deg with an MT
pulse), TR = 25 ms, echoes at TE = 2.3 ms * (k + 1), a seeded ground truth,
seeded B1 transmit field and seeded Gaussian noise.

Parameter maps are returned in the log / logit coordinates the method works in
(Sec. 2.4): (log A, log R1, log R2*, logit MTsat), layout ``[4][N]`` with voxel
index ``n = x + nx*(y + ny*z)``.  Draw order is fixed: maps, then B1, then
noise in (image, z, y, x) order.
"""
from __future__ import annotations

import math
import os

import numpy as np

# cfg-1 style parameter ranges (units: A arbitrary, R1 and R2* in 1/s)
PD_RANGE = (500.0, 1000.0)
R1_RANGE = (0.5, 1.5)
R2_RANGE = (10.0, 40.0)
MT_RANGE = (0.005, 0.02)


def protocol(echoes=(8, 8, 6), flips_deg=(6.0, 21.0, 6.0), mt=(0, 0, 1), tr=0.025,
             te0=2.3e-3, dte=2.3e-3, sigma=1.0):
    """Plain-dict protocol: contrasts PDw / T1w / MTw by default (Sec. 3.2)."""
    te = []
    for e in echoes:
        te += [te0 + dte * k for k in range(e)]
    n_img = len(te)
    sig = list(sigma) if hasattr(sigma, "__len__") else [float(sigma)] * n_img
    return {
        "n_echoes": [int(e) for e in echoes],
        "tr": [float(tr)] * len(echoes) if not hasattr(tr, "__len__") else [float(t) for t in tr],
        "flip": [math.radians(f) for f in flips_deg],
        "mt": [int(m) for m in mt],
        "te": te,
        "sigma": sig,
    }


def encode(pd, r1, r2, mt):
    """Physical parameters -> (log A, log R1, log R2*, logit MTsat) maps [4][N]."""
    pd, r1, r2, mt = (np.asarray(v, dtype=np.float64).reshape(-1) for v in (pd, r1, r2, mt))
    return np.stack([np.log(pd), np.log(r1), np.log(r2), np.log(mt) - np.log1p(-mt)])


def maps_iid(shape, rng):
    """Independent uniform draws per voxel (PD, R1, R2*, MTsat), cfg-1 ranges."""
    n = int(np.prod(shape))
    pd = rng.uniform(*PD_RANGE, size=n)
    r1 = rng.uniform(*R1_RANGE, size=n)
    r2 = rng.uniform(*R2_RANGE, size=n)
    mt = rng.uniform(*MT_RANGE, size=n)
    return encode(pd, r1, r2, mt)


def _smooth(field, sigma):
    """Gaussian filter (truncated at 3 sigma, reflected borders): the 1-D
    filter along each axis in turn, as scipy's gaussian_filter applies it, with
    the lines of each pass split over threads (the same values)."""
    from concurrent.futures import ThreadPoolExecutor

    from scipy.ndimage import gaussian_filter1d
    out = np.asarray(field, dtype=np.float64).copy()
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as pool:
        for axis in range(out.ndim):
            other = 0 if axis != 0 else 1  # split along an axis that is not filtered
            bounds = np.linspace(0, out.shape[other], workers + 1).astype(int)

            def run(k, axis=axis, other=other, bounds=bounds):
                sl = [slice(None)] * out.ndim
                sl[other] = slice(bounds[k], bounds[k + 1])
                sl = tuple(sl)
                out[sl] = gaussian_filter1d(out[sl], sigma, axis=axis, truncate=3.0, mode="reflect")
            list(pool.map(run, range(workers)))
    return out


def maps_tissue(shape, rng, n_classes=3, class_sigma=6.0, texture=0.05, texture_sigma=1.5):
    """Piecewise-smooth maps: argmax of smoothed noise fields picks one of
    ``n_classes`` tissues whose means are drawn from the cfg-1 ranges; each map
    is then multiplied by (1 + texture * t) with t unit-variance smoothed noise
    and clipped to its range.  ``shape`` is (nz, ny, nx)."""
    fields = np.stack([_smooth(rng.standard_normal(shape), class_sigma) for _ in range(n_classes)])
    label = np.argmax(fields, axis=0)
    out = []
    for lo, hi in (PD_RANGE, R1_RANGE, R2_RANGE, MT_RANGE):
        means = rng.uniform(lo, hi, size=n_classes)
        t = _smooth(rng.standard_normal(shape), texture_sigma)
        t /= max(float(t.std()), 1e-12)
        m = means[label] * (1.0 + texture * t)
        out.append(np.clip(m, lo, hi).reshape(-1))
    return encode(*out)


def b1_field(shape, rng, lo=0.8, hi=1.2, sigma=20.0):
    """Smooth transmit-efficiency field: Gaussian-filtered white noise mapped
    affinely so that its minimum is ``lo`` and its maximum ``hi``."""
    f = _smooth(rng.standard_normal(shape), sigma)
    fmin, fmax = float(f.min()), float(f.max())
    f = lo + (hi - lo) * (f - fmin) / max(fmax - fmin, 1e-30)
    return f.reshape(-1).astype(np.float64)


def noise(n_images, n, rng):
    """Unit Gaussian noise [I][N] in float32 (scaled by sigma_i by the caller)."""
    return rng.standard_normal((n_images, n), dtype=np.float32)


def rigid_space(recon_dims, acq_dims, rng, rot_deg=2.0, shift=1.5):
    """An acquisition space moved by a seeded rigid motion relative to the
    reconstruction grid (subject motion between contrasts, Sec. 2.4): rotation
    angles uniform in +-rot_deg about each axis, composed about the centre of
    the reconstruction grid, and a translation uniform in +-shift voxels per
    axis.  Returns {"dims": acq_dims, "affine": 3x4 array} mapping acquisition
    voxel indices to reconstruction-grid coordinates."""
    a, b, c = np.deg2rad(rng.uniform(-rot_deg, rot_deg, 3))
    Rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rz = np.array([[np.cos(c), -np.sin(c), 0], [np.sin(c), np.cos(c), 0], [0, 0, 1]])
    R = Rz @ Ry @ Rx
    centre_r = (np.asarray(recon_dims, dtype=np.float64) - 1) / 2
    centre_a = (np.asarray(acq_dims, dtype=np.float64) - 1) / 2
    t = centre_r - R @ centre_a + rng.uniform(-shift, shift, 3)
    return {"dims": tuple(int(v) for v in acq_dims), "affine": np.hstack([R, t[:, None]])}


def e1_problems(n, rng):
    """The paper's convergence experiment (Sec. 3.1; sampling as read from its
    text): per voxel, log-parameters (log A, log R1, log R2*, logit MTsat) and
    the log TR of each of three contrasts uniform in [-5, 5], flip angles
    uniform in [0, pi/4], and the log TE of each of 15 echoes (5 per contrast)
    uniform in [-5, 5].  Returns y [4][n], tr [3][n], flip [3][n], te [15][n];
    draw order y, tr, flip, te.  The last contrast carries the MT pulse and
    sigma = 1 (so x = s + eps with unit Gaussian eps)."""
    y = rng.uniform(-5, 5, (4, n))
    tr = np.exp(rng.uniform(-5, 5, (3, n)))
    flip = rng.uniform(0, math.pi / 4, (3, n))
    te = np.exp(rng.uniform(-5, 5, (15, n)))
    return y, tr, flip, te


def identity_space(dims):
    return {"dims": tuple(int(v) for v in dims), "affine": np.hstack([np.eye(3), np.zeros((3, 1))])}


# --------------------------------------------------------------------------
# Named workloads.  Shapes are (nx, ny, nz); arrays are flat with x fastest.
# --------------------------------------------------------------------------
CASES = {
    # plain ML voxelwise fit, 32^3, 6/6/6 echoes, iid maps, B1 = 1, sigma 1% of mean PD
    "ml32": dict(dims=(32, 32, 32), echoes=(6, 6, 6), maps="iid", b1=None, noise_frac=0.01,
                 seed=101, mode="ml", n_gn=20),
    # plain ML, whole-brain grid, 8/8/6 echoes, tissue maps, B1 in [0.8, 1.2]
    "ml_brain": dict(dims=(192, 240, 256), echoes=(8, 8, 6), maps="tissue", b1=(0.8, 1.2),
                     noise_frac=0.01, seed=102, mode="ml", n_gn=20),
    # JTV-MAP on the same whole-brain volume, 10 x 8 x 32
    "map_brain": dict(dims=(192, 240, 256), echoes=(8, 8, 6), maps="tissue", b1=(0.8, 1.2),
                      noise_frac=0.01, seed=102, mode="map", n_outer=10, n_gn=8, n_cg=32),
    # high-resolution JTV-MAP + uncertainty, B1 in [0.7, 1.3], sigma 2% of mean PD
    "map_hires": dict(dims=(416, 384, 320), echoes=(8, 8, 6), maps="tissue", b1=(0.7, 1.3),
                      noise_frac=0.02, seed=105, mode="map", n_outer=10, n_gn=8, n_cg=32),
}


def make_case(name=None, dims=None, seed=None, **over):
    """Draw one workload.  Returns a dict with keys
    ``dims, proto, truth [4][N], b1 [N] or None, eps [I][N] float32, sigma, lam, opts``.

    ``name`` picks a preset from CASES; ``dims``/``seed``/other keys override it
    (e.g. a 64^3 crop-sized volume drawn with the same recipe)."""
    cfg = dict(CASES[name]) if name else dict(dims=(32, 32, 32), echoes=(6, 6, 6), maps="iid",
                                              b1=None, noise_frac=0.01, seed=0, mode="ml", n_gn=20)
    cfg.update(over)
    if dims is not None:
        cfg["dims"] = tuple(int(v) for v in dims)
    if seed is not None:
        cfg["seed"] = int(seed)
    nx, ny, nz = cfg["dims"]
    shape = (nz, ny, nx)
    n = nx * ny * nz
    rng = np.random.default_rng(cfg["seed"])
    truth = maps_iid(shape, rng) if cfg["maps"] == "iid" else maps_tissue(shape, rng)
    b1 = None
    if cfg["b1"] is not None:
        b1 = b1_field(shape, rng, *cfg["b1"], sigma=cfg.get("b1_sigma", 20.0))
    proto = protocol(echoes=cfg["echoes"])
    n_img = sum(cfg["echoes"])
    eps = noise(n_img, n, rng)
    sigma = cfg["noise_frac"] * float(np.exp(truth[0]).mean())
    proto["sigma"] = [sigma] * n_img
    lam = [1e-3 * float(truth[k].max() - truth[k].min()) for k in range(4)]
    opts = {"mode": cfg["mode"], "n_gn": cfg.get("n_gn", 20), "n_outer": cfg.get("n_outer", 1),
            "n_cg": cfg.get("n_cg", 32), "max_halvings": 4,
            "lam": lam if cfg["mode"] == "map" else [0.0] * 4}
    return {"name": name, "dims": cfg["dims"], "proto": proto, "truth": truth, "b1": b1,
            "eps": eps, "sigma": sigma, "lam": lam, "opts": opts, "seed": cfg["seed"]}


def head_mask(dims, frac=0.8):
    """Ellipsoid occupying `frac` of each axis' extent, centred: True inside
    (the head), False outside (air).  Flat [N], x fastest."""
    nx, ny, nz = (int(v) for v in dims)
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) / n - 0.5 for n in (nz, ny, nx)], indexing="ij")
    r = (x / (0.5 * frac)) ** 2 + (y / (0.5 * frac)) ** 2 + (z / (0.5 * frac)) ** 2
    return (r <= 1.0).reshape(-1)


def head_case(dims, seed, noise_frac=0.02, echoes=(8, 8, 6)):
    """Magnitude echoes of a head in air, as the paper's noise estimation
    (Sec. 2.7) expects them: tissue maps inside an ellipsoid, no signal
    outside; the noise is complex Gaussian of std sigma per channel, so every
    value is |s + sigma (e1 + i e2)| (Rician; Rayleigh in the air).  Returns
    the case dict of make_case plus ``mask`` [N] and ``rice`` = (e1, e2), two
    float32 [I][N] noise arrays; the magnitudes are formed by the caller
    from its own forward model."""
    c = make_case("map_brain", dims=dims, seed=seed, noise_frac=noise_frac, echoes=echoes)
    rng = np.random.default_rng(seed + 7)
    n_img, n = len(c["proto"]["te"]), c["truth"].shape[1]
    c["mask"] = head_mask(dims)
    c["rice"] = (noise(n_img, n, rng), noise(n_img, n, rng))
    # sigma relative to the mean PD inside the head
    c["sigma"] = noise_frac * float(np.exp(c["truth"][0][c["mask"]]).mean())
    c["proto"]["sigma"] = [c["sigma"]] * n_img
    return c


def magnitudes(signal, case):
    """|s + sigma (e1 + i e2)| with the signal zeroed outside the head."""
    s = np.where(case["mask"][None, :], signal, 0.0)
    e1, e2 = case["rice"]
    return np.hypot(s + case["sigma"] * e1, case["sigma"] * e2)
