"""ctypes binding of libmpm (include/mpm.h): argument marshalling only.

Every step of the fit runs in the HIP library; torch is used for device memory
and streams.  Importing this module does not load the library; the first call
does, and raises if ``libmpm.so`` has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

MPM_MAX_CONTRASTS = 8
MPM_MAX_IMAGES = 64
MPM_F32, MPM_F16, MPM_BF16 = 0, 1, 2
MPM_ML, MPM_MAP_JTV = 0, 1
MPM_INIT_DEFAULT, MPM_INIT_CONST, MPM_INIT_FROM_MAPS = 0, 1, 2
MPM_LOAD_PROPOSED, MPM_LOAD_GN, MPM_LOAD_PROPOSED_PLUS = 0, 1, 2
MPM_BASES = {"log": 0, "rate": 1, "time": 2}
STATUS = {0: "MPM_OK", 1: "MPM_ERR_INVALID_ARG", 2: "MPM_ERR_UNSUPPORTED", 3: "MPM_ERR_OUT_OF_MEMORY",
          4: "MPM_ERR_DEVICE", 5: "MPM_ERR_BUSY", 6: "MPM_ERR_NOT_FOUND", 7: "MPM_ERR_CANCELLED"}


class mpm_protocol(C.Structure):
    _fields_ = [("n_contrasts", C.c_int32), ("n_echoes", C.c_int32 * MPM_MAX_CONTRASTS),
                ("tr_s", C.c_double * MPM_MAX_CONTRASTS), ("flip_rad", C.c_double * MPM_MAX_CONTRASTS),
                ("mt", C.c_int32 * MPM_MAX_CONTRASTS), ("te_s", C.c_double * MPM_MAX_IMAGES),
                ("sigma", C.c_double * MPM_MAX_IMAGES)]


class mpm_grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64)]


class mpm_options(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_outer", C.c_int32), ("n_gn", C.c_int32), ("n_cg", C.c_int32),
                ("max_halvings", C.c_int32), ("loading", C.c_int32), ("init_kind", C.c_int32),
                ("flags", C.c_int32), ("lam", C.c_double * 4), ("jtv_eps", C.c_double),
                ("cg_stop", C.c_double), ("init_const", C.c_double * 4), ("tol_gn", C.c_double),
                ("tol_outer", C.c_double), ("b1_receive", C.c_void_p), ("basis", C.c_int32),
                ("start_outer", C.c_int32), ("echo_offset", C.POINTER(C.c_float))]


class mpm_report(C.Structure):
    _fields_ = [("objective", C.c_double), ("nll", C.c_double), ("jtv", C.c_double),
                ("outer_done", C.c_int32), ("gn_done", C.c_int32), ("cg_done", C.c_int32),
                ("rejected", C.c_int32), ("degenerate_voxels", C.c_int64),
                ("nonfinite_voxels", C.c_int64), ("nll_increases", C.c_int64)]


class mpm_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("timed", C.c_int64),
                ("timed_ms", C.c_double), ("bytes", C.c_double)]


class mpm_request(C.Structure):
    _fields_ = [("protocol", mpm_protocol), ("grid", mpm_grid), ("dtype", C.c_int32), ("reserved", C.c_int32),
                ("echoes", C.c_void_p), ("b1", C.c_void_p), ("options", mpm_options), ("maps", C.c_void_p)]


MPM_SERVER_THREAD = 1
MPM_SERVER_NO_GROUPS = 2


class mpm_space(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64), ("affine", C.c_double * 12)]


class mpm_voxel_protocols(C.Structure):
    _fields_ = [("n_contrasts", C.c_int32), ("n_echoes", C.c_int32 * MPM_MAX_CONTRASTS),
                ("mt", C.c_int32 * MPM_MAX_CONTRASTS), ("sigma", C.c_double * MPM_MAX_IMAGES),
                ("tr_s", C.c_void_p), ("flip_rad", C.c_void_p), ("te_s", C.c_void_p)]


class mpm_rice_fit(C.Structure):
    _fields_ = [("pi", C.c_double * 2), ("nu", C.c_double * 2), ("sigma", C.c_double * 2), ("mean", C.c_double * 2),
                ("nll", C.c_double)]


class mpm_tune_result(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("chosen", C.c_int32), ("target", C.c_int32 * 8),
                ("workgroups", C.c_int32 * 8), ("planes_per_run", C.c_int32 * 8), ("ms", C.c_double * 8)]


class MpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

# every function declared in include/mpm.h, with its ctypes signature
_P, _G, _O, _R = C.POINTER(mpm_protocol), C.POINTER(mpm_grid), C.POINTER(mpm_options), C.POINTER(mpm_report)
SIGNATURES = {
    "mpm_fit": (C.c_int, [_P, _G, C.c_int, C.c_void_p, C.c_void_p, _O, C.c_void_p, _R,
                          C.POINTER(C.c_double), C.c_int32, C.c_void_p]),
    "mpm_fit_batch": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                C.c_void_p]),
    "mpm_pack_echoes": (C.c_int, [C.c_int32, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_float),
                                  C.c_void_p]),
    "mpm_fit_noalloc": (C.c_int, [_P, _G, C.c_int, C.c_void_p, C.c_void_p, _O, C.c_void_p, _R,
                                  C.POINTER(C.c_double), C.c_int32, C.c_void_p]),
    "mpm_uncertainty": (C.c_int, [_P, _G, C.c_int, C.c_void_p, C.c_void_p, _O, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]),
    "mpm_simulate": (C.c_int, [_P, _G, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "mpm_footprint_bytes": (C.c_size_t, [_P, _G, C.c_int, C.c_int32]),
    "mpm_fit_projected": (C.c_int, [_P, _G, C.POINTER(mpm_space), C.c_int, C.c_void_p, C.c_void_p, _O, C.c_void_p,
                                    _R, C.POINTER(C.c_double), C.c_int32, C.c_void_p]),
    "mpm_uncertainty_projected": (C.c_int, [_P, _G, C.POINTER(mpm_space), C.c_int, C.c_void_p, C.c_void_p, _O,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpm_simulate_projected": (C.c_int, [_P, _G, C.POINTER(mpm_space), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                         C.c_void_p, C.c_void_p]),
    "mpm_fit_voxelwise": (C.c_int, [C.POINTER(mpm_voxel_protocols), C.c_int64, C.c_int, C.c_void_p, _O, C.c_void_p,
                                    C.c_void_p, C.c_void_p, _R, C.c_void_p]),
    "mpm_simulate_voxelwise": (C.c_int, [C.POINTER(mpm_voxel_protocols), C.c_int64, C.c_void_p, C.c_void_p, C.c_int,
                                         C.c_void_p, C.c_void_p]),
    "mpm_estimate_noise": (C.c_int, [_P, _G, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(mpm_rice_fit), C.POINTER(C.c_uint32),
                                     C.c_void_p]),
    "mpm_autotune": (C.c_int, [_G, C.c_int32, C.POINTER(mpm_tune_result), C.c_void_p]),
    "mpm_autotune_set": (C.c_int, [_G, C.c_int32, C.c_int32]),
    "mpm_autotune_clear": (None, []),
    "mpm_last_error": (C.c_char_p, []),
    "mpm_version": (C.c_char_p, []),
    "mpm_profile_enable": (None, [C.c_int32]),
    "mpm_profile_reset": (None, []),
    "mpm_profile_read": (C.c_int32, [C.POINTER(mpm_kernel_stat), C.c_int32]),
    "mpm_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    "mpm_server_submit": (C.c_int, [C.c_void_p, C.POINTER(mpm_request), C.POINTER(C.c_uint64)]),
    "mpm_server_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mpm_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), _R]),
    "mpm_server_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "mpm_server_destroy": (C.c_int, [C.c_void_p]),
}


def load():
    """Load libmpm.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "python paper_2102_01604_amd/build.py")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(st):
    if st != 0:
        raise MpmError(st, load().mpm_last_error().decode())


def make_protocol(proto: dict) -> mpm_protocol:
    p = mpm_protocol()
    nc = len(proto["n_echoes"])
    p.n_contrasts = nc
    for c in range(min(nc, MPM_MAX_CONTRASTS)):
        p.n_echoes[c] = int(proto["n_echoes"][c])
        p.tr_s[c] = float(proto["tr"][c])
        p.flip_rad[c] = float(proto["flip"][c])
        p.mt[c] = int(proto["mt"][c])
    for i in range(min(len(proto["te"]), MPM_MAX_IMAGES)):
        p.te_s[i] = float(proto["te"][i])
        p.sigma[i] = float(proto["sigma"][i])
    return p


def make_grid(dims) -> mpm_grid:
    g = mpm_grid()
    g.nx, g.ny, g.nz = (int(v) for v in dims)
    return g


def make_options(opts: dict) -> mpm_options:
    o = mpm_options()
    o.mode = {"ml": MPM_ML, "map": MPM_MAP_JTV}[opts.get("mode", "ml")]
    o.n_outer = int(opts.get("n_outer", 1))
    o.n_gn = int(opts.get("n_gn", 20))
    o.n_cg = int(opts.get("n_cg", 32))
    o.max_halvings = int(opts.get("max_halvings", 4))
    o.loading = {"proposed": MPM_LOAD_PROPOSED, "gn": MPM_LOAD_GN,
                 "plus": MPM_LOAD_PROPOSED_PLUS}[opts.get("loading", "proposed")]
    o.init_kind = {"default": MPM_INIT_DEFAULT, "const": MPM_INIT_CONST,
                   "maps": MPM_INIT_FROM_MAPS}[opts.get("init", "default")]
    o.flags = int(opts.get("flags", 0))
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
    bm = opts.get("b1_receive")
    o.b1_receive = None if bm is None else _f32(bm, "b1_receive").value
    o.basis = MPM_BASES[opts.get("basis", "log")]
    o.start_outer = int(opts.get("start_outer", 0))
    off = opts.get("echo_offset")
    if off is not None:
        arr = (C.c_float * len(off))(*[float(v) for v in off])
        o._echo_offset_keep = arr  # the struct holds a raw pointer into it
        o.echo_offset = C.cast(arr, C.POINTER(C.c_float))
    return o


def trace_len(opts: dict) -> int:
    if opts.get("mode", "ml") == "ml":
        return int(opts.get("n_gn", 20)) + 1
    return int(opts.get("n_outer", 1)) * (int(opts.get("n_gn", 20)) + 2)


def _dtype_code(t):
    import torch
    return {torch.float32: MPM_F32, torch.float16: MPM_F16, torch.bfloat16: MPM_BF16}[t.dtype]


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f32(t, name):
    """Device pointer of a float32 tensor argument (maps, b1, var, moments,
    noise): the library reads these as FP32, so any other dtype is an error."""
    if t is None:
        return None
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor (got {t.dtype})")
    return C.c_void_p(t.data_ptr())


def mpm_fit(protocol: dict, dims, echoes, b1, options: dict, maps, stream=None):
    """Run mpm_fit on device tensors.  ``maps`` (float32 [4][N]) is updated in
    place.  Returns (report dict, trace numpy array)."""
    lib = load()
    tl = trace_len(options)
    trace = (C.c_double * tl)()
    rep = mpm_report()
    _check(lib.mpm_fit(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)), _dtype_code(echoes),
                       _ptr(echoes), _f32(b1, "b1"), C.byref(make_options(options)), _f32(maps, "maps"), C.byref(rep),
                       trace, tl, _stream(stream)))
    report = {f[0]: getattr(rep, f[0]) for f in mpm_report._fields_}
    return report, np.array(trace[:], dtype=np.float64)


def make_request(protocol: dict, dims, echoes, b1, options: dict, maps):
    """An mpm_request for device tensors (the struct keeps raw pointers: keep
    the tensors and the returned object alive while it is in use)."""
    r = mpm_request()
    r.protocol = make_protocol(protocol)
    r.grid = make_grid(dims)
    r.dtype = _dtype_code(echoes)
    r.echoes = echoes.data_ptr()
    r.b1 = None if b1 is None else _f32(b1, "b1").value
    o = make_options(options)
    r.options = o
    r._options_keep = o
    r.maps = _f32(maps, "maps").value
    return r


def mpm_fit_batch(fits, stream=None):
    """Fit several JTV-MAP volumes together (batched launches).  fits: list of
    (protocol, dims, echoes, b1, options, maps) with device tensors; maps are
    updated in place.  Returns a list of (report dict, trace array)."""
    lib = load()
    n = len(fits)
    reqs = (mpm_request * n)()
    keep = []
    for i, (protocol, dims, echoes, b1, options, maps) in enumerate(fits):
        r = make_request(protocol, dims, echoes, b1, options, maps)
        keep.append(r)
        reqs[i] = r
    tl = max(trace_len(f[4]) for f in fits)
    traces = (C.c_double * (n * tl))()
    reps = (mpm_report * n)()
    _check(lib.mpm_fit_batch(n, reqs, reps, traces, tl, _stream(stream)))
    out = []
    for i in range(n):
        rep = {f[0]: getattr(reps[i], f[0]) for f in mpm_report._fields_}
        out.append((rep, np.array(traces[i * tl:(i + 1) * tl], dtype=np.float64)[:trace_len(fits[i][4])]))
    return out


def mpm_pack_echoes(src, dst, stream=None):
    """Pack float32 echoes src [I][N] into dst (float16 / bfloat16 [I][N]) with
    per-image offsets; returns the offsets (list of I floats) for the options'
    "echo_offset"."""
    lib = load()
    I, N = int(src.shape[0]), int(src.shape[1])
    off = (C.c_float * I)()
    _check(lib.mpm_pack_echoes(I, N, _f32(src, "src"), _dtype_code(dst), _ptr(dst), off, _stream(stream)))
    return [float(v) for v in off]


def mpm_fit_noalloc(protocol: dict, dims, echoes, b1, options: dict, maps, stream=None):
    """mpm_fit with the library's fixed scratch as workspace (no allocation);
    same arguments and results as mpm_fit."""
    lib = load()
    tl = trace_len(options)
    trace = (C.c_double * tl)()
    rep = mpm_report()
    _check(lib.mpm_fit_noalloc(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)), _dtype_code(echoes),
                               _ptr(echoes), _f32(b1, "b1"), C.byref(make_options(options)), _f32(maps, "maps"),
                               C.byref(rep), trace, tl, _stream(stream)))
    report = {f[0]: getattr(rep, f[0]) for f in mpm_report._fields_}
    return report, np.array(trace[:], dtype=np.float64)


def mpm_uncertainty(protocol: dict, dims, echoes, b1, options: dict, maps, var, moments=None, stream=None):
    lib = load()
    _check(lib.mpm_uncertainty(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)), _dtype_code(echoes),
                               _ptr(echoes), _f32(b1, "b1"), C.byref(make_options(options)), _f32(maps, "maps"),
                               _f32(var, "var"), _f32(moments, "moments"), _stream(stream)))


def mpm_simulate(protocol: dict, dims, maps, b1, noise, out, stream=None):
    lib = load()
    _check(lib.mpm_simulate(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)), _f32(maps, "maps"),
                            _f32(b1, "b1"), _f32(noise, "noise"), _dtype_code(out), _ptr(out), _stream(stream)))


def make_spaces(spaces):
    """Acquisition spaces: a list (one per contrast) of {"dims": (nx, ny, nz),
    "affine": 3x4 map from the space's voxel indices to reconstruction-grid
    coordinates}."""
    arr = (mpm_space * len(spaces))()
    for c, sp in enumerate(spaces):
        arr[c].nx, arr[c].ny, arr[c].nz = (int(v) for v in sp["dims"])
        a = np.asarray(sp["affine"], dtype=np.float64).reshape(-1)
        for k in range(12):
            arr[c].affine[k] = float(a[k])
    return arr


def mpm_fit_projected(protocol: dict, dims, spaces, echoes, b1, options: dict, maps, stream=None):
    """mpm_fit_projected on device tensors; echoes: the images back to back,
    each on its contrast's space.  Returns (report dict, trace)."""
    lib = load()
    tl = trace_len(options)
    trace = (C.c_double * tl)()
    rep = mpm_report()
    _check(lib.mpm_fit_projected(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)), make_spaces(spaces),
                                 _dtype_code(echoes), _ptr(echoes), _f32(b1, "b1"), C.byref(make_options(options)),
                                 _f32(maps, "maps"), C.byref(rep), trace, tl, _stream(stream)))
    report = {f[0]: getattr(rep, f[0]) for f in mpm_report._fields_}
    return report, np.array(trace[:], dtype=np.float64)


def mpm_uncertainty_projected(protocol: dict, dims, spaces, echoes, b1, options: dict, maps, var, moments=None,
                              stream=None):
    lib = load()
    _check(lib.mpm_uncertainty_projected(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)),
                                         make_spaces(spaces), _dtype_code(echoes), _ptr(echoes), _f32(b1, "b1"),
                                         C.byref(make_options(options)), _f32(maps, "maps"), _f32(var, "var"),
                                         _f32(moments, "moments"), _stream(stream)))


def mpm_simulate_projected(protocol: dict, dims, spaces, maps, b1, noise, out, stream=None):
    lib = load()
    _check(lib.mpm_simulate_projected(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)),
                                      make_spaces(spaces), _f32(maps, "maps"), _f32(b1, "b1"), _f32(noise, "noise"),
                                      _dtype_code(out), _ptr(out), _stream(stream)))


def make_voxel_protocols(shape: dict, tr=None, flip=None, te=None) -> mpm_voxel_protocols:
    """shape: {"n_echoes", "mt", "sigma"} shared by every voxel; tr, flip
    [C][N] and te [I][N]: float32 device tensors (or None)."""
    p = mpm_voxel_protocols()
    nc = len(shape["n_echoes"])
    p.n_contrasts = nc
    for c in range(min(nc, MPM_MAX_CONTRASTS)):
        p.n_echoes[c] = int(shape["n_echoes"][c])
        p.mt[c] = int(shape["mt"][c])
    for i in range(min(len(shape["sigma"]), MPM_MAX_IMAGES)):
        p.sigma[i] = float(shape["sigma"][i])
    p.tr_s = None if tr is None else _f32(tr, "tr").value
    p.flip_rad = None if flip is None else _f32(flip, "flip").value
    p.te_s = None if te is None else _f32(te, "te").value
    return p


def mpm_fit_voxelwise(shape: dict, tr, flip, te, echoes, options: dict, maps, nll_increases=None, nll=None,
                      stream=None):
    """mpm_fit_voxelwise on device tensors (a protocol per voxel): tr, flip
    [C][N], te [I][N] float32; echoes [I][N]; maps [4][N] float32;
    nll_increases [N] int32 and nll [N] float32 optional.  Returns the report
    dict."""
    import torch
    lib = load()
    if nll_increases is not None and (nll_increases.dtype != torch.int32 or not nll_increases.is_contiguous()):
        raise TypeError("nll_increases must be a contiguous int32 tensor")
    rep = mpm_report()
    N = int(maps.shape[-1])
    _check(lib.mpm_fit_voxelwise(C.byref(make_voxel_protocols(shape, tr, flip, te)), N, _dtype_code(echoes),
                                 _ptr(echoes), C.byref(make_options(options)), _f32(maps, "maps"), _ptr(nll_increases),
                                 _f32(nll, "nll"), C.byref(rep), _stream(stream)))
    return {f[0]: getattr(rep, f[0]) for f in mpm_report._fields_}


def mpm_simulate_voxelwise(shape: dict, tr, flip, te, maps, noise, out, stream=None):
    """Echoes out [I][N] for per-voxel protocols (tr, flip [C][N], te [I][N])."""
    lib = load()
    N = int(maps.shape[-1])
    _check(lib.mpm_simulate_voxelwise(C.byref(make_voxel_protocols(shape, tr, flip, te)), N, _f32(maps, "maps"),
                                      _f32(noise, "noise"), _dtype_code(out), _ptr(out), _stream(stream)))


def mpm_estimate_noise(protocol: dict, dims, echoes, b1=None, nbins: int = 1024, n_iter: int = 200,
                       want_hist: bool = False, stream=None) -> dict:
    """Noise level and initial maps from magnitude echoes with a background
    (Sec. 2.7).  Returns sigma_image [I], sigma_contrast [C], fg_mean [I],
    init_const [4], the per-image mixtures and (want_hist) the histograms."""
    lib = load()
    proto = dict(protocol)
    I = sum(proto["n_echoes"])
    proto.setdefault("sigma", [1.0] * I)
    n_c = len(proto["n_echoes"])
    si, sc, fg, y0 = (C.c_double * I)(), (C.c_double * n_c)(), (C.c_double * I)(), (C.c_double * 4)()
    fits = (mpm_rice_fit * I)()
    hist = (C.c_uint32 * (I * nbins))() if want_hist else None
    _check(lib.mpm_estimate_noise(C.byref(make_protocol(proto)), C.byref(make_grid(dims)), _dtype_code(echoes),
                                  _ptr(echoes), _f32(b1, "b1"), int(nbins), int(n_iter), si, sc, fg, y0, fits, hist,
                                  _stream(stream)))
    out = {"sigma_image": list(si), "sigma_contrast": list(sc), "fg_mean": list(fg), "init_const": list(y0),
           "fits": [{k: (list(getattr(f, k)) if k != "nll" else f.nll) for k, _ in mpm_rice_fit._fields_}
                    for f in fits]}
    if want_hist:
        out["hist"] = list(hist)
    return out


def mpm_autotune(dims, reps: int = 5, stream=None) -> dict:
    """Time the MAP fit's CG sweep A for each workgroup-count candidate on a
    grid of `dims` and keep the fastest for that size (this process)."""
    lib = load()
    r = mpm_tune_result()
    _check(lib.mpm_autotune(C.byref(make_grid(dims)), int(reps), C.byref(r), _stream(stream)))
    n = r.n_candidates
    return {"chosen": r.chosen, "target": list(r.target[:n]), "workgroups": list(r.workgroups[:n]),
            "planes_per_run": list(r.planes_per_run[:n]), "ms": list(r.ms[:n])}


def mpm_autotune_set(dims, cg_workgroups: int, column_workgroups: int = 0):
    """Fix the CG sweep A and column-walk workgroup targets of MAP fits on a
    grid of `dims` (this process); 0 keeps the built-in choice."""
    _check(load().mpm_autotune_set(C.byref(make_grid(dims)), int(cg_workgroups), int(column_workgroups)))


def mpm_autotune_clear():
    load().mpm_autotune_clear()


def mpm_footprint_bytes(protocol: dict, dims, dtype: int, mode: int) -> int:
    return int(load().mpm_footprint_bytes(C.byref(make_protocol(protocol)), C.byref(make_grid(dims)), dtype, mode))


def mpm_version() -> str:
    return load().mpm_version().decode()


def mpm_profile_enable(every: int):
    load().mpm_profile_enable(int(every))


def mpm_profile_reset():
    load().mpm_profile_reset()


def mpm_profile_read():
    lib = load()
    arr = (mpm_kernel_stat * 64)()
    n = lib.mpm_profile_read(arr, 64)
    return {arr[i].name.decode(): {"launches": arr[i].launches, "timed": arr[i].timed,
                                   "timed_ms": arr[i].timed_ms, "bytes": arr[i].bytes}
            for i in range(min(n, 64))}


class MpmServer:
    """Thin wrapper of the mpm_server_* calls (continuous batching of fits)."""

    def __init__(self, hbm_budget: int, max_active: int = 4, thread: bool = False, groups: bool = True):
        lib = load()
        h = C.c_void_p()
        flags = (MPM_SERVER_THREAD if thread else 0) | (0 if groups else MPM_SERVER_NO_GROUPS)
        _check(lib.mpm_server_create(int(hbm_budget), int(max_active), flags, C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, protocol: dict, dims, echoes, b1, options: dict, maps) -> int:
        """Queue a fit; device buffers must already hold their inputs and stay
        alive until poll() reports it done."""
        r = mpm_request()
        r.protocol = make_protocol(protocol)
        r.grid = make_grid(dims)
        r.dtype = _dtype_code(echoes)
        r.echoes = echoes.data_ptr()
        r.b1 = None if b1 is None else b1.data_ptr()
        o = make_options(options)
        r.options = o
        r.maps = maps.data_ptr()
        t = C.c_uint64()
        _check(load().mpm_server_submit(self._h, C.byref(r), C.byref(t)))
        self._keep[t.value] = (echoes, b1, maps, options.get("b1_receive"), o)
        return t.value

    def step(self) -> int:
        p = C.c_int32()
        _check(load().mpm_server_step(self._h, C.byref(p)))
        return p.value

    def poll(self, ticket: int):
        """None while the fit is queued or running, else its report (raises on a failed fit)."""
        d = C.c_int32()
        rep = mpm_report()
        st = load().mpm_server_poll(self._h, C.c_uint64(ticket), C.byref(d), C.byref(rep))
        if st != 0:
            if d.value:
                self._keep.pop(ticket, None)
            _check(st)
        if not d.value:
            return None
        self._keep.pop(ticket, None)
        return {f[0]: getattr(rep, f[0]) for f in mpm_report._fields_}

    def cancel(self, ticket: int):
        """Cancel a queued or running request; poll then raises MPM_ERR_CANCELLED
        (the buffers stay borrowed until it does)."""
        _check(load().mpm_server_cancel(self._h, C.c_uint64(ticket)))

    def close(self):
        if self._h:
            _check(load().mpm_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def nan_trace_ok(trace) -> bool:
    return all(math.isnan(v) or math.isfinite(v) for v in trace)
