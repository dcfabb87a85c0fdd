"""Plain FP64 CPU oracle for model-based multi-parameter mapping (arXiv 2102.01604).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import
it; the GPU library never does, and the two share no code.

The arithmetic lives in ``mpm_oracle.c`` (plain C, double precision); this
module only marshals numpy arrays into it.  Protocols are plain dicts::

    {"n_echoes": [8, 8, 6], "tr": [0.025]*3, "flip": [rad, ...], "mt": [0, 0, 1],
     "te": [s, ...] (contrast-major, one per image), "sigma": [...] (one per image)}

Arrays are C-contiguous float64: maps ``[4][N]``, echoes ``[I][N]``, with voxel
index ``n = x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpm_oracle.c")
# MPM_ORACLE_LIB selects another build of the same source (the sanitizer build
# the tests make with build_sanitized)
_LIB_PATH = os.environ.get("MPM_ORACLE_LIB") or os.path.join(_HERE, "libmpm_oracle.so")

MAX_CONTRASTS = 8
MAX_IMAGES = 64
ML, MAP = 0, 1
INIT_DEFAULT, INIT_CONST, INIT_FROM_MAPS = 0, 1, 2
LOAD_PROPOSED, LOAD_GN, LOAD_PLUS = 0, 1, 2
LOADINGS = {"proposed": LOAD_PROPOSED, "gn": LOAD_GN, "plus": LOAD_PLUS}
BASES = {"log": 0, "rate": 1, "time": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) to `path`; load it by setting MPM_ORACLE_LIB in a
    process started with the ASan runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", path, _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    return path


class Protocol(C.Structure):
    _fields_ = [("n_contrasts", C.c_int32), ("n_echoes", C.c_int32 * MAX_CONTRASTS),
                ("tr", C.c_double * MAX_CONTRASTS), ("flip", C.c_double * MAX_CONTRASTS),
                ("mt", C.c_int32 * MAX_CONTRASTS), ("te", C.c_double * MAX_IMAGES),
                ("sigma", C.c_double * MAX_IMAGES)]


class Space(C.Structure):
    _fields_ = [("dims", C.c_int64 * 3), ("affine", C.c_double * 12)]


class Options(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_outer", C.c_int32), ("n_gn", C.c_int32),
                ("n_cg", C.c_int32), ("max_halvings", C.c_int32), ("loading", C.c_int32),
                ("init_kind", C.c_int32), ("basis", C.c_int32), ("lam", C.c_double * 4),
                ("jtv_eps", C.c_double), ("cg_stop", C.c_double),
                ("init_const", C.c_double * 4), ("tol_gn", C.c_double), ("tol_outer", C.c_double),
                ("b1_receive", C.c_void_p), ("start_outer", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("objective", C.c_double), ("nll", C.c_double), ("jtv", C.c_double),
                ("outer_done", C.c_int32), ("gn_done", C.c_int32), ("cg_done", C.c_int32),
                ("rejected", C.c_int32), ("degenerate_voxels", C.c_int64),
                ("nonfinite_voxels", C.c_int64), ("nll_increases", C.c_int64)]


_lib = None
_dp = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = C.CDLL(_LIB_PATH)
        lib.orc_spgr_derivs.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                        _dp, _dp, _dp]
        lib.orc_spgr_hess.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_int, _dp]
        lib.orc_bessel_i01e.argtypes = [C.c_double, _dp, _dp]
        lib.orc_histogram.argtypes = [_dp, C.c_int64, C.c_int, C.POINTER(C.c_int64)]
        lib.orc_histogram.restype = C.c_float
        lib.orc_rice_mixture.argtypes = [C.POINTER(C.c_int64), C.c_int, C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp]
        lib.orc_rice_mixture.restype = C.c_int
        lib.orc_estimate_noise.argtypes = [C.POINTER(Protocol), C.c_int64, _dp, _dp, C.c_int, C.c_int, _dp, _dp, _dp,
                                           _dp]
        lib.orc_estimate_noise.restype = C.c_int
        lib.orc_spgr_basis.argtypes = [_dp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, _dp, _dp, _dp]
        lib.orc_lik_voxel_basis.argtypes = [C.POINTER(Protocol), _dp, C.c_int64, _dp, C.c_int, C.c_int, _dp, _dp,
                                            _dp]
        lib.orc_simulate.argtypes = [C.POINTER(Protocol), C.c_int64, _dp, _dp, _dp]
        lib.orc_lik_voxel.argtypes = [C.POINTER(Protocol), _dp, C.c_int64, _dp, C.c_double,
                                      C.c_int, _dp, _dp, _dp]
        lib.orc_solve4.argtypes = [_dp, _dp, _dp]
        lib.orc_solve4.restype = C.c_int
        lib.orc_jtv_weights.argtypes = [C.POINTER(C.c_int64), _dp, _dp, C.c_double, _dp, _dp]
        lib.orc_jtv_weights.restype = C.c_double
        lib.orc_apply_L.argtypes = [C.POINTER(C.c_int64), _dp, _dp, _dp, _dp]
        lib.orc_pcg.argtypes = [C.POINTER(C.c_int64), _dp, _dp, _dp, _dp, _dp, C.c_int,
                                C.c_double, _dp]
        lib.orc_pcg.restype = C.c_int
        lib.orc_default_init.argtypes = [C.POINTER(Protocol), C.c_int64, _dp, _dp, _dp]
        lib.orc_default_init.restype = C.c_int
        lib.orc_fit.argtypes = [C.POINTER(Protocol), C.POINTER(C.c_int64), _dp, _dp,
                                C.POINTER(Options), _dp, C.POINTER(Report), _dp, C.c_int32]
        lib.orc_fit.restype = C.c_int
        lib.orc_uncertainty.argtypes = [C.POINTER(Protocol), C.POINTER(C.c_int64), _dp, _dp,
                                        C.POINTER(Options), _dp, _dp, _dp]
        lib.orc_uncertainty.restype = C.c_int
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_num_threads.argtypes = [C.c_int]
        lib.orc_set_num_threads.restype = None
        sp = C.POINTER(Space)
        lib.orc_pull.argtypes = [C.POINTER(C.c_int64), sp, _dp, _dp]
        lib.orc_push.argtypes = [C.POINTER(C.c_int64), sp, _dp, _dp]
        lib.orc_proj_lik.argtypes = [C.POINTER(Protocol), C.POINTER(C.c_int64), sp, _dp, _dp, C.c_int, _dp,
                                     _dp, _dp]
        lib.orc_proj_lik.restype = C.c_double
        lib.orc_default_init_projected.argtypes = [C.POINTER(Protocol), C.POINTER(C.c_int64), sp, _dp, _dp, _dp]
        lib.orc_default_init_projected.restype = C.c_int
        lib.orc_fit_projected.argtypes = [C.POINTER(Protocol), C.POINTER(C.c_int64), sp, _dp, _dp,
                                          C.POINTER(Options), _dp, C.POINTER(Report), _dp, C.c_int32]
        lib.orc_fit_projected.restype = C.c_int
        lib.orc_uncertainty_projected.argtypes = [C.POINTER(Protocol), C.POINTER(C.c_int64), sp, _dp, _dp,
                                                  C.POINTER(Options), _dp, _dp, _dp]
        lib.orc_uncertainty_projected.restype = C.c_int
        lib.orc_fit_voxelwise.argtypes = [C.POINTER(Protocol), C.c_int64, _dp, _dp, _dp, _dp, C.POINTER(Options),
                                          C.c_double, _dp, C.POINTER(C.c_int32), _dp, C.POINTER(Report)]
        lib.orc_fit_voxelwise.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def n_images(proto) -> int:
    return int(sum(proto["n_echoes"]))


def make_protocol(proto) -> Protocol:
    p = Protocol()
    C_ = len(proto["n_echoes"])
    p.n_contrasts = C_
    for c in range(C_):
        p.n_echoes[c] = int(proto["n_echoes"][c])
        p.tr[c] = float(proto["tr"][c])
        p.flip[c] = float(proto["flip"][c])
        p.mt[c] = int(proto["mt"][c])
    for i in range(n_images(proto)):
        p.te[i] = float(proto["te"][i])
        p.sigma[i] = float(proto["sigma"][i])
    return p


def make_options(opts: dict) -> Options:
    o = Options()
    o.mode = {"ml": ML, "map": MAP}[opts.get("mode", "ml")]
    o.n_outer = int(opts.get("n_outer", 1))
    o.n_gn = int(opts.get("n_gn", 20))
    o.n_cg = int(opts.get("n_cg", 32))
    o.max_halvings = int(opts.get("max_halvings", 4))
    o.loading = LOADINGS[opts.get("loading", "proposed")]
    kind = opts.get("init", "default")
    o.init_kind = {"default": INIT_DEFAULT, "const": INIT_CONST, "maps": INIT_FROM_MAPS}[kind]
    lam = opts.get("lam", (0.0, 0.0, 0.0, 0.0))
    for k in range(4):
        o.lam[k] = float(lam[k])
    o.jtv_eps = float(opts.get("jtv_eps", 0.0))
    o.cg_stop = float(opts.get("cg_stop", 0.0))
    ic = opts.get("init_const", (0.0, 0.0, 0.0, 0.0))
    for k in range(4):
        o.init_const[k] = float(ic[k])
    o.tol_gn = float(opts.get("tol_gn", 0.0))
    o.tol_outer = float(opts.get("tol_outer", 0.0))
    o.basis = BASES[opts.get("basis", "log")]
    o.start_outer = int(opts.get("start_outer", 0))
    bm = opts.get("b1_receive")
    if bm is not None:  # the caller keeps the array alive (fit and uncertainty hold it)
        o.b1_receive = bm.ctypes.data
    return o


def _dims(dims):
    d = (C.c_int64 * 3)(*[int(v) for v in dims])
    return d


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's voxel-parallel loops from now on."""
    _load().orc_set_num_threads(int(n))


def bessel_i01e(z):
    """(e^-z I0(z), e^-z I1(z)) for z >= 0."""
    a, b = np.zeros(1), np.zeros(1)
    _load().orc_bessel_i01e(float(z), _ptr(a), _ptr(b))
    return float(a[0]), float(b[0])


def histogram(x, nbins):
    """(counts [nbins] int64, FP32 scale) of one magnitude image."""
    xv = _f64(np.asarray(x)).reshape(-1)
    counts = np.zeros(nbins, dtype=np.int64)
    scale = _load().orc_histogram(_ptr(xv), xv.size, int(nbins), counts.ctypes.data_as(C.POINTER(C.c_int64)))
    return counts, float(scale)


def rice_mixture(counts, scale, n_iter):
    """Two-class Rician mixture on a histogram: dict of pi, nu, sigma, mean
    (2 each) and the NLL trace [n_iter + 1]."""
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    out = {k: np.zeros(2) for k in ("pi", "nu", "sigma", "mean")}
    nll = np.zeros(n_iter + 1)
    st = _load().orc_rice_mixture(counts.ctypes.data_as(C.POINTER(C.c_int64)), counts.size, float(scale),
                                  int(n_iter), _ptr(out["pi"]), _ptr(out["nu"]), _ptr(out["sigma"]),
                                  _ptr(out["mean"]), _ptr(nll))
    if st:
        raise ValueError("the histogram does not split in two classes")
    out["nll"] = nll
    return out


def estimate_noise(proto, x, b1=None, nbins=1024, n_iter=200):
    """Per-image sigma, per-contrast sigma (geometric mean of the variances),
    per-image foreground mean and the initial maps y0 (Sec. 2.7)."""
    I = n_images(proto)
    x = _f64(x).reshape(I, -1)
    N = x.shape[1]
    b1 = None if b1 is None else _f64(b1).reshape(N)
    si, sc, fg, y0 = np.zeros(I), np.zeros(len(proto["n_echoes"])), np.zeros(I), np.zeros(4)
    p = make_protocol(dict(proto, sigma=[1.0] * I))
    st = _load().orc_estimate_noise(C.byref(p), N, _ptr(x), _ptr(b1), int(nbins), int(n_iter), _ptr(si), _ptr(sc),
                                    _ptr(fg), _ptr(y0))
    if st:
        raise ValueError("an image does not split in two classes")
    return {"sigma_image": si, "sigma_contrast": sc, "fg_mean": fg, "y0": y0}


def spgr_basis(th, basis, alpha, tr, te, mt):
    """Signal, gradient and full second-derivative matrix [4][4] with respect
    to the parameters of basis "rate" (A, R1, R2*, MTsat) or "time"
    (A, T1, T2*, MTsat), for one image."""
    lib = _load()
    tv = _f64(np.asarray(th))
    s = np.zeros(1)
    ds = np.zeros(4)
    H = np.zeros(16)
    lib.orc_spgr_basis(_ptr(tv), BASES[basis], alpha, tr, te, int(mt), _ptr(s), _ptr(ds), _ptr(H))
    return float(s[0]), ds, H.reshape(4, 4)


def lik_voxel_basis(proto, x, th, basis, loading="proposed"):
    """NLL, gradient and loaded Hessian [4][4] of one voxel (x: [I]) with
    respect to the parameters th of basis "log", "rate" or "time"."""
    lib = _load()
    p = make_protocol(proto)
    xv = _f64(np.asarray(x))
    tv = _f64(np.asarray(th))
    nll = np.zeros(1)
    g = np.zeros(4)
    P = np.zeros(16)
    lib.orc_lik_voxel_basis(C.byref(p), _ptr(xv), 1, _ptr(tv), BASES[basis], LOADINGS[loading], _ptr(nll), _ptr(g),
                            _ptr(P))
    return float(nll[0]), g, P.reshape(4, 4)


def spgr_derivs(y, alpha, tr, te, mt):
    """Signal, gradient and diagonal second derivatives for one image."""
    lib = _load()
    yv = _f64(np.asarray(y))
    s = np.zeros(1)
    ds = np.zeros(4)
    d2s = np.zeros(4)
    lib.orc_spgr_derivs(_ptr(yv), alpha, tr, te, int(mt), _ptr(s), _ptr(ds), _ptr(d2s))
    return float(s[0]), ds, d2s


def spgr_hess(y, alpha, tr, te, mt):
    """Full 4x4 matrix of second derivatives of the signal of one image."""
    lib = _load()
    yv = _f64(np.asarray(y))
    H = np.zeros(16)
    lib.orc_spgr_hess(_ptr(yv), alpha, tr, te, int(mt), _ptr(H))
    return H.reshape(4, 4)


def simulate(proto, maps, b1=None):
    """Noise-free echoes [I][N] from maps [4][N]."""
    lib = _load()
    maps = _f64(maps).reshape(4, -1)
    n = maps.shape[1]
    b1 = None if b1 is None else _f64(b1).reshape(-1)
    out = np.empty((n_images(proto), n))
    p = make_protocol(proto)
    lib.orc_simulate(C.byref(p), n, _ptr(maps), _ptr(b1), _ptr(out))
    return out


def lik_voxel(proto, x, y, b1=1.0, loading="proposed"):
    """(nll, g[4], P[4,4]) of one voxel; x holds its I observations."""
    lib = _load()
    xv = _f64(np.asarray(x).reshape(-1))
    yv = _f64(np.asarray(y).reshape(-1))
    nll = np.zeros(1)
    g = np.zeros(4)
    P = np.zeros(16)
    p = make_protocol(proto)
    lib.orc_lik_voxel(C.byref(p), _ptr(xv), 1, _ptr(yv), float(b1),
                      LOADINGS[loading],
                      _ptr(nll), _ptr(g), _ptr(P))
    return float(nll[0]), g, P.reshape(4, 4)


def solve4(P, g):
    """(P^{-1} g with the degenerate rule, status) for one symmetric 4x4 P."""
    lib = _load()
    Pv = _f64(np.asarray(P).reshape(16))
    gv = _f64(np.asarray(g).reshape(4))
    out = np.zeros(4)
    st = lib.orc_solve4(_ptr(Pv), _ptr(gv), _ptr(out))
    return out, int(st)


def jtv_weights(dims, maps, lam, eps):
    """(w[N], d[N], sum sqrt(q+eps^2)) of maps [4][N] on a grid (nx, ny, nz)."""
    lib = _load()
    maps = _f64(maps).reshape(4, -1)
    n = maps.shape[1]
    w = np.empty(n)
    d = np.empty(n)
    lv = _f64(np.asarray(lam, dtype=np.float64))
    jt = lib.orc_jtv_weights(_dims(dims), _ptr(maps), _ptr(lv), float(eps), _ptr(w), _ptr(d))
    return w, d, float(jt)


def apply_L(dims, w, lam, v):
    """(L v) for v [4][N] with L = G^T W G (x) diag(lambda)."""
    lib = _load()
    v = _f64(v).reshape(4, -1)
    w = _f64(w).reshape(-1)
    lv = _f64(np.asarray(lam, dtype=np.float64))
    out = np.empty_like(v)
    lib.orc_apply_L(_dims(dims), _ptr(w), _ptr(lv), _ptr(v), _ptr(out))
    return out


def pcg(dims, P, w, d, lam, b, n_cg, cg_stop=1e-10):
    """PCG solve of (P + L) delta = b; P is [N][4][4].  Returns (delta, iterations)."""
    lib = _load()
    P = _f64(P).reshape(-1, 16)
    b = _f64(b).reshape(4, -1)
    w = _f64(w).reshape(-1)
    d = _f64(d).reshape(-1)
    lv = _f64(np.asarray(lam, dtype=np.float64))
    delta = np.empty_like(b)
    it = lib.orc_pcg(_dims(dims), _ptr(P), _ptr(w), _ptr(d), _ptr(lv), _ptr(b), int(n_cg),
                     float(cg_stop), _ptr(delta))
    return delta, int(it)


def default_init(proto, x, b1=None):
    """Constant initial log-parameters (4,) from per-image volume means."""
    lib = _load()
    x = _f64(x).reshape(n_images(proto), -1)
    b1 = None if b1 is None else _f64(b1).reshape(-1)
    y0 = np.zeros(4)
    p = make_protocol(proto)
    st = lib.orc_default_init(C.byref(p), x.shape[1], _ptr(x), _ptr(b1), _ptr(y0))
    if st:
        raise ValueError("protocol has no usable PDw/T1w/MTw contrasts for the default init")
    return y0


def trace_len(opts: dict) -> int:
    if opts.get("mode", "ml") == "ml":
        return int(opts.get("n_gn", 20)) + 1
    return int(opts.get("n_outer", 1)) * (int(opts.get("n_gn", 20)) + 2)


def _with_receive(opts, N):
    """opts with "b1_receive" (receive field [N]) as a contiguous float64 array."""
    if opts.get("b1_receive") is None:
        return opts
    return dict(opts, b1_receive=np.ascontiguousarray(opts["b1_receive"], dtype=np.float64).reshape(N))


def fit(proto, dims, x, b1, opts: dict, maps0=None):
    """Run the fit.  Returns (maps [4][N], report dict, trace array)."""
    lib = _load()
    N = int(np.prod(dims))
    x = _f64(x).reshape(n_images(proto), N)
    b1 = None if b1 is None else _f64(b1).reshape(N)
    opts = _with_receive(opts, N)
    o = make_options(opts)
    if maps0 is not None:
        maps = _f64(maps0).reshape(4, N).copy()
        o.init_kind = INIT_FROM_MAPS
    else:
        maps = np.zeros((4, N))
        if o.init_kind == INIT_FROM_MAPS:
            raise ValueError("init='maps' needs maps0")
    tl = trace_len(opts)
    trace = np.empty(tl)
    rep = Report()
    p = make_protocol(proto)
    st = lib.orc_fit(C.byref(p), _dims(dims), _ptr(x), _ptr(b1), C.byref(o), _ptr(maps),
                     C.byref(rep), _ptr(trace), tl)
    if st:
        raise ValueError("default initialisation failed")
    report = {f[0]: getattr(rep, f[0]) for f in Report._fields_}
    return maps, report, trace


def fit_voxelwise(shape, tr, flip, te, x, opts: dict, maps0=None, rise_rel=1e-12):
    """ML fit with a protocol per voxel (Sec. 3.1): shape gives n_echoes, mt and
    sigma; tr, flip [C][N] and te [I][N] per voxel.  Starts from
    opts["init_const"] or maps0.  Returns (maps [4][N], increases [N], final
    NLL [N], report dict)."""
    lib = _load()
    tr = _f64(tr)
    N = tr.shape[-1]
    C_, I = len(shape["n_echoes"]), n_images(shape)
    tr, flip, te = tr.reshape(C_, N), _f64(flip).reshape(C_, N), _f64(te).reshape(I, N)
    x = _f64(x).reshape(I, N)
    o = make_options(dict(opts, mode="ml"))
    if maps0 is not None:
        maps = _f64(maps0).reshape(4, N).copy()
        o.init_kind = INIT_FROM_MAPS
    else:
        maps = np.zeros((4, N))
    inc = np.zeros(N, dtype=np.int32)
    nll = np.zeros(N)
    rep = Report()
    p = make_protocol(dict(shape, tr=[1.0] * C_, flip=[0.1] * C_, te=[0.0] * I))
    st = lib.orc_fit_voxelwise(C.byref(p), N, _ptr(tr), _ptr(flip), _ptr(te), _ptr(x), C.byref(o), float(rise_rel),
                               _ptr(maps), inc.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(nll), C.byref(rep))
    if st:
        raise ValueError("fit_voxelwise needs init='const' or maps0")
    return maps, inc, nll, {f[0]: getattr(rep, f[0]) for f in Report._fields_}


def uncertainty(proto, dims, x, b1, opts: dict, maps, moments=False):
    """Laplace posterior variance [4][N] (and optional moments [4][N])."""
    lib = _load()
    N = int(np.prod(dims))
    x = _f64(x).reshape(n_images(proto), N)
    b1 = None if b1 is None else _f64(b1).reshape(N)
    maps = _f64(maps).reshape(4, N)
    opts = _with_receive(opts, N)
    o = make_options(opts)
    var = np.empty((4, N))
    mom = np.empty((4, N)) if moments else None
    p = make_protocol(proto)
    lib.orc_uncertainty(C.byref(p), _dims(dims), _ptr(x), _ptr(b1), C.byref(o), _ptr(maps),
                        _ptr(var), _ptr(mom))
    return (var, mom) if moments else var


def default_eps(lam) -> float:
    return 1e-3 * math.sqrt(float(sum(lam)))


# ---------------------------------------------------------------------------
# spatial projection (Sec. 2.4): each contrast has its own acquisition space,
# {"dims": (mx, my, mz), "affine": 3x4 map from its voxel indices to
# reconstruction-grid coordinates}; echoes are one flat array with the images
# back to back (image i holds the voxels of its contrast's space), or a list
# of per-contrast arrays [E_c][M_c].
# ---------------------------------------------------------------------------
def make_spaces(spaces):
    arr = (Space * len(spaces))()
    for c, sp in enumerate(spaces):
        for d in range(3):
            arr[c].dims[d] = int(sp["dims"][d])
        a = np.asarray(sp["affine"], dtype=np.float64).reshape(3, 4)
        for k in range(12):
            arr[c].affine[k] = float(a.reshape(-1)[k])
    return arr


def space_voxels(sp) -> int:
    return int(np.prod(sp["dims"]))


def flat_echoes(proto, spaces, x):
    if isinstance(x, (list, tuple)):
        x = np.concatenate([np.asarray(v, dtype=np.float64).reshape(-1) for v in x])
    x = _f64(x).reshape(-1)
    need = sum(int(proto["n_echoes"][c]) * space_voxels(sp) for c, sp in enumerate(spaces))
    if x.size != need:
        raise ValueError(f"projected echoes hold {x.size} values, the spaces need {need}")
    return x


def pull(dims, space, vol):
    """Psi vol: recon [N] -> acquisition [M] (0 outside the field of view)."""
    lib = _load()
    vol = _f64(vol).reshape(-1)
    out = np.empty(space_voxels(space))
    lib.orc_pull(_dims(dims), make_spaces([space]), _ptr(vol), _ptr(out))
    return out


def push(dims, space, acq):
    """Psi^T acq: acquisition [M] -> recon [N]."""
    lib = _load()
    acq = _f64(acq).reshape(-1)
    out = np.empty(int(np.prod(dims)))
    lib.orc_push(_dims(dims), make_spaces([space]), _ptr(acq), _ptr(out))
    return out


def proj_lik(proto, dims, spaces, x, b1, maps, loading="proposed"):
    """(total NLL, pushed g [4][N], pushed blocks P [N][4][4]) with projection."""
    lib = _load()
    N = int(np.prod(dims))
    x = flat_echoes(proto, spaces, x)
    b1 = None if b1 is None else _f64(b1).reshape(N)
    maps = _f64(maps).reshape(4, N)
    g = np.empty((4, N))
    P = np.empty((N, 16))
    p = make_protocol(proto)
    nll = lib.orc_proj_lik(C.byref(p), _dims(dims), make_spaces(spaces), _ptr(x), _ptr(b1), LOADINGS[loading],
                           _ptr(maps), _ptr(g), _ptr(P))
    return float(nll), g, P.reshape(N, 4, 4)


def default_init_projected(proto, dims, spaces, x, b1=None):
    lib = _load()
    x = flat_echoes(proto, spaces, x)
    b1 = None if b1 is None else _f64(b1).reshape(-1)
    y0 = np.zeros(4)
    p = make_protocol(proto)
    if lib.orc_default_init_projected(C.byref(p), _dims(dims), make_spaces(spaces), _ptr(x), _ptr(b1), _ptr(y0)):
        raise ValueError("protocol has no usable PDw/T1w/MTw contrasts for the default init")
    return y0


def fit_projected(proto, dims, spaces, x, b1, opts: dict, maps0=None):
    """The fit with spatial projection.  Returns (maps [4][N], report, trace)."""
    lib = _load()
    N = int(np.prod(dims))
    x = flat_echoes(proto, spaces, x)
    b1 = None if b1 is None else _f64(b1).reshape(N)
    o = make_options(opts)
    if maps0 is not None:
        maps = _f64(maps0).reshape(4, N).copy()
        o.init_kind = INIT_FROM_MAPS
    else:
        maps = np.zeros((4, N))
        if o.init_kind == INIT_FROM_MAPS:
            raise ValueError("init='maps' needs maps0")
    tl = trace_len(opts)
    trace = np.empty(tl)
    rep = Report()
    p = make_protocol(proto)
    st = lib.orc_fit_projected(C.byref(p), _dims(dims), make_spaces(spaces), _ptr(x), _ptr(b1), C.byref(o),
                               _ptr(maps), C.byref(rep), _ptr(trace), tl)
    if st:
        raise ValueError("default initialisation failed")
    return maps, {f[0]: getattr(rep, f[0]) for f in Report._fields_}, trace


def uncertainty_projected(proto, dims, spaces, x, b1, opts: dict, maps):
    lib = _load()
    N = int(np.prod(dims))
    x = flat_echoes(proto, spaces, x)
    b1 = None if b1 is None else _f64(b1).reshape(N)
    maps = _f64(maps).reshape(4, N)
    var = np.empty((4, N))
    p = make_protocol(proto)
    lib.orc_uncertainty_projected(C.byref(p), _dims(dims), make_spaces(spaces), _ptr(x), _ptr(b1),
                                  C.byref(make_options(opts)), _ptr(maps), _ptr(var), None)
    return var

