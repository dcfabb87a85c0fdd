"""GPU parity of the JTV-MAP fit (SPGR+JTV) and of the Laplace uncertainty
against the FP64 oracle, through the C ABI."""
import json
import os

import numpy as np
import pytest

from conftest import cuda, f32, map_errors, observations, well_posed
from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
# Laplace variance and moments, relative per voxel (FP32 assembly of the
# 4 x 4 block and its inverse; measured at a few 1e-6)
VAR_TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _inputs(orc, name, dims, seed=None, **over):
    c = synth.make_case(name, dims=dims, seed=seed, **over)
    if c["b1"] is not None:
        c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    return c, x


def _gpu(torch, c, x, opts, dtype=None, maps0=None):
    X = cuda(x.astype(np.float32))
    if dtype is not None:
        X = X.to(dtype)
    b1 = None if c["b1"] is None else cuda(c["b1"].astype(np.float32))
    maps = cuda(np.zeros((4, x.shape[1]), np.float32) if maps0 is None else maps0.astype(np.float32))
    rep, trace = _lib.mpm_fit(c["proto"], c["dims"], X, b1, opts, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy().astype(np.float64), rep, trace


def _const_opts(orc, c, x, **kw):
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    o = dict(c["opts"], init="const", init_const=[float(v) for v in y0])
    o.update(kw)
    return o


def _compare(orc, torch, c, x, opts, tol=TOL, trace_rtol=1e-5):
    y_gpu, rep, tr = _gpu(torch, c, x, opts)
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    good = well_posed(y_orc, c["truth"])
    rel, ab, rms = map_errors(y_gpu, y_orc, good)
    rel_all, ab_all, _ = map_errors(y_gpu, y_orc)
    print(c["dims"], "well-posed", good.mean(), "rel", rel, "abs", ab, "rms", rms, "| all voxels rel", rel_all)
    print("gpu report", rep)
    print("orc report", rep_o)
    assert (rel <= tol).all() and (rel_all <= tol).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(tr), fin)
    assert np.allclose(tr[fin], tr_o[fin], rtol=trace_rtol)
    assert rep["gn_done"] == rep_o["gn_done"] and rep["rejected"] == rep_o["rejected"]
    assert rep["nonfinite_voxels"] == 0
    assert rep["objective"] == pytest.approx(rep_o["objective"], rel=trace_rtol)
    return y_gpu, y_orc, rep, rep_o


@pytest.mark.parametrize("dims,sched", [((24, 20, 12), (4, 4, 16)), ((70, 9, 5), (3, 3, 8)),
                                        ((2, 1, 1), (2, 2, 4)), ((1, 1, 5), (2, 3, 4))])
def test_map_parity_small(torch_cuda, orc, dims, sched):
    c, x = _inputs(orc, "map_brain", dims, seed=31)
    T, J, K = sched
    opts = _const_opts(orc, c, x, n_outer=T, n_gn=J, n_cg=K)
    _compare(orc, torch_cuda, c, x, opts)


def test_map_parity_crop_full_schedule(torch_cuda, orc):
    """A 64^3 volume drawn with the high-resolution recipe (B1 in [0.7, 1.3],
    sigma 2% of mean PD) fitted with the full 10 x 8 x 32 schedule on both
    sides."""
    c, x = _inputs(orc, "map_hires", (64, 64, 64))
    opts = _const_opts(orc, c, x)
    _compare(orc, torch_cuda, c, x, opts)


# Launch shapes whose workgroups walk z-runs of several planes on a ragged
# 70 x 37 x 41 grid (nz not a multiple of the run length): CG sweep A tiles
# are 64 x 16 (2 x 3 = 6 per plane), column-walk tiles 64 x 4 (2 x 10 = 20).
# (sweep A target, column target) -> planes per run: (123, 410) -> 2 / 2,
# (50, 164) -> 5 / 5, (1, 1) -> 32 / 32 (the longest run the sweeps take).
SHAPE_DIMS = (70, 37, 41)


def _runs(tiles, nz, target):
    zc = min(32, nz, max(1, -(-tiles * nz // target)))
    return zc, -(-nz // zc)


@pytest.fixture(scope="module")
def shape_case(orc):
    c, x = _inputs(orc, "map_brain", SHAPE_DIMS, seed=37)
    opts = _const_opts(orc, c, x)  # the full 10 x 8 x 32 schedule
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    return c, x, opts, y_orc, rep_o, tr_o


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cg_wg,col_wg", [(123, 410), (50, 164), (1, 1)])
def test_map_parity_multi_plane_runs(torch_cuda, shape_case, cg_wg, col_wg):
    """CG sweep A's cross-plane register rotation and double-buffered LDS
    planes, and the column walks of the JTV weights and of the halved-step
    acceptance, compared with the oracle voxel by voxel over the full
    schedule."""
    c, x, opts, y_orc, rep_o, tr_o = shape_case
    nx, ny, nz = SHAPE_DIMS
    za = _runs(2 * 3, nz, cg_wg)
    zw = _runs(2 * 10, nz, col_wg)
    assert za[0] >= 2 and zw[0] >= 2 and nz % za[0] and nz % zw[0]
    _lib.mpm_autotune_set(SHAPE_DIMS, cg_wg, col_wg)
    try:
        y_gpu, rep, tr = _gpu(torch_cuda, c, x, opts)
    finally:
        _lib.mpm_autotune_clear()
    good = well_posed(y_orc, c["truth"])
    rel, ab, rms = map_errors(y_gpu, y_orc, good)
    rel_all, _, _ = map_errors(y_gpu, y_orc)
    print("sweep A runs", za, "column runs", zw, "well-posed", good.mean(), "rel", rel, "all", rel_all)
    print("gpu report", rep, "| oracle report", rep_o)
    assert (rel <= TOL).all() and (rel_all <= TOL).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(tr), fin)
    assert np.allclose(tr[fin], tr_o[fin], rtol=1e-6)
    # (CG counts differ in the first outer loop, where one iteration solves each
    # system and the FP64 residual vanishes while the FP32 one does not)
    assert rep["gn_done"] == rep_o["gn_done"] and rep["rejected"] == rep_o["rejected"]
    assert rep["objective"] == pytest.approx(rep_o["objective"], rel=1e-6)


def test_map_without_prior_equals_ml_on_gpu(torch_cuda, orc):
    c, x = _inputs(orc, "map_brain", (40, 24, 8), seed=32)
    ml = _const_opts(orc, c, x, mode="ml", n_gn=9)
    mp = _const_opts(orc, c, x, mode="map", n_outer=3, n_gn=3, n_cg=6, lam=[0, 0, 0, 0])
    y_ml, _, _ = _gpu(torch_cuda, c, x, ml)
    y_mp, rep, _ = _gpu(torch_cuda, c, x, mp)
    good = well_posed(y_ml, c["truth"])
    rel, _, _ = map_errors(y_mp, y_ml, good)
    print("MAP(lambda=0) vs ML", rel)
    assert (rel <= TOL).all()


def test_map_objective_monotone_on_gpu(torch_cuda, orc):
    c, x = _inputs(orc, "map_brain", (48, 40, 24), seed=33)
    opts = _const_opts(orc, c, x, n_outer=5, n_gn=4, n_cg=16)
    _, rep, tr = _gpu(torch_cuda, c, x, opts)
    t = tr.reshape(5, 6)
    for row in t:
        fw = row[:5][np.isfinite(row[:5])]
        assert np.all(np.diff(fw) <= 1e-9 * np.abs(fw[:-1]))  # the acceptance test's slack
    assert np.all(np.diff(t[:, -1]) <= 1e-9 * np.abs(t[:-1, -1]))


def _pack(torch, x, dtype, offsets):
    """(device echoes in dtype, offsets or None, dequantised values): FP16 /
    BF16 of x - per-image offsets (mpm_pack_echoes) or of x itself."""
    dt = {"f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    X = cuda(x.astype(np.float32))
    if offsets:
        Q = torch.empty(X.shape, dtype=dt, device="cuda")
        off = _lib.mpm_pack_echoes(X, Q)
        o = np.asarray(off, np.float64)[:, None]
    else:
        Q, off, o = X.to(dt), None, 0.0
    torch.cuda.synchronize()
    return Q, off, Q.float().cpu().numpy().astype(np.float64) + o


def _fit_packed(torch, c, Q, opts, off):
    maps = torch.zeros((4, Q.shape[1]), dtype=torch.float32, device="cuda")
    b1 = None if c["b1"] is None else cuda(c["b1"].astype(np.float32))
    rep, tr = _lib.mpm_fit(c["proto"], c["dims"], Q, b1, dict(opts, echo_offset=off), maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy().astype(np.float64), rep, tr


@pytest.mark.parametrize("offsets", [True, False], ids=["offsets", "plain"])
@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_map_reduced_precision_storage(torch_cuda, orc, dtype, offsets):
    """As the ML test: arithmetic parity with the oracle on the dequantised
    values (1e-4, all voxels); against the unquantised data FP16 with
    per-image offsets meets 1e-3, the other forms stay within the oracle's own
    storage floor plus the FP32 bound."""
    torch = torch_cuda
    c, x = _inputs(orc, "map_brain", (32, 24, 16), seed=34)
    opts = _const_opts(orc, c, x, n_outer=4, n_gn=4, n_cg=16)
    Q, off, xq = _pack(torch, x, dtype, offsets)
    y_gpu, rep, tr = _fit_packed(torch, c, Q, opts, off)
    y_orc_q, rep_q, tr_q = orc.fit(c["proto"], c["dims"], xq, c["b1"], opts)
    rel, ab, rms = map_errors(y_gpu, y_orc_q)
    print(dtype, offsets, "vs dequantised oracle (all voxels)", rel, ab, rms)
    assert (rel <= TOL).all()
    fin = np.isfinite(tr_q)
    assert np.allclose(tr[fin], tr_q[fin], rtol=1e-6)
    y_orc, _, _ = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    rel_u, _, _ = map_errors(y_gpu, y_orc)
    good = well_posed(y_orc, c["truth"])
    floor = map_errors(y_orc_q, y_orc)[0]
    print(dtype, offsets, "vs unquantised oracle (all voxels)", rel_u, "well-posed",
          map_errors(y_gpu, y_orc, good)[0], "| oracle's own storage floor", floor)
    if dtype == "f16" and offsets:
        assert (rel_u <= 1e-3).all()
    else:
        assert (rel_u <= floor + TOL).all()


@pytest.mark.timeout(600)
def test_map_high_resolution_crop_fp16(torch_cuda, orc):
    """The high-resolution recipe's parity case: a 64^3 volume drawn with it
    (B1 0.7-1.3, sigma 2% of mean PD), FP16 echo storage with per-image
    offsets, the full 10 x 8 x 32 schedule, then the Laplace variance, against
    the oracle on the unquantised data: maps within 1e-3 (all voxels), the
    objective trace within 1e-5, the variance at the oracle's maps within
    1e-3."""
    torch = torch_cuda
    c, x = _inputs(orc, "map_hires", (64, 64, 64))
    opts = _const_opts(orc, c, x)
    Q, off, xq = _pack(torch, x, "f16", True)
    y_gpu, rep, tr = _fit_packed(torch, c, Q, opts, off)
    print("hires crop: fitting the oracle", flush=True)
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    rel, ab, rms = map_errors(y_gpu, y_orc)
    good = well_posed(y_orc, c["truth"])
    print("hires crop FP16: rel (all voxels)", rel, "well-posed", map_errors(y_gpu, y_orc, good)[0], "rms", rms)
    print("gpu report", rep, "| oracle", rep_o)
    assert (rel <= 1e-3).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(tr), fin) and np.allclose(tr[fin], tr_o[fin], rtol=1e-5)
    assert rep["gn_done"] == rep_o["gn_done"] and rep["rejected"] == rep_o["rejected"]
    maps = f32(y_orc)
    var_o = orc.uncertainty(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts, maps)
    N = x.shape[1]
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], Q, cuda(c["b1"].astype(np.float32)), dict(opts, echo_offset=off),
                         cuda(maps.astype(np.float32)), var)
    v = var.cpu().numpy().astype(np.float64)
    ok = np.all(np.isfinite(var_o), axis=0)
    assert np.array_equal(np.isfinite(v), np.isfinite(var_o))
    rv = np.abs(v[:, ok] - var_o[:, ok]) / var_o[:, ok]
    print("hires crop FP16: variance rel err max", rv.max(axis=1))
    assert rv.max() <= 1e-3


@pytest.mark.parametrize("mode", ["ml", "map"])
def test_uncertainty_parity(torch_cuda, orc, mode):
    torch = torch_cuda
    c, x = _inputs(orc, "map_brain", (30, 20, 10), seed=35)
    opts = _const_opts(orc, c, x, n_outer=3, n_gn=4, n_cg=8, mode=mode)
    if mode == "ml":
        opts["n_gn"] = 12
    y_orc, _, _ = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    maps = f32(y_orc)
    var_o, mom_o = orc.uncertainty(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts, maps, moments=True)
    N = x.shape[1]
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    mom = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], cuda(x.astype(np.float32)), cuda(c["b1"].astype(np.float32)),
                         opts, cuda(maps.astype(np.float32)), var, mom)
    v = var.cpu().numpy().astype(np.float64)
    m = mom.cpu().numpy().astype(np.float64)
    good = well_posed(y_orc, c["truth"]) & np.all(np.isfinite(var_o), axis=0)
    assert np.array_equal(np.isfinite(v), np.isfinite(var_o))
    rv = np.abs(v[:, good] - var_o[:, good]) / var_o[:, good]
    rm = np.abs(m[:, good] - mom_o[:, good]) / np.abs(mom_o[:, good])
    print(mode, "variance rel err max", rv.max(axis=1), "moments", rm.max(axis=1))
    assert rv.max() <= VAR_TOL and rm.max() <= VAR_TOL


@pytest.mark.timeout(900)
def test_map_whole_brain_launch_configuration(torch_cuda, orc):
    """The whole-brain workload (192 x 240 x 256, 22 echoes, B1 0.8-1.2) in the
    launch configuration the benchmark times (CG sweep A walks 2-plane z-runs,
    the column walks 6-plane runs), against the oracle run on the same volume:
    a 2 x 3 x 16 MAP fit equals the oracle's at every voxel, with the same
    objective trace, no rejected step and a strictly decreasing objective
    within each outer loop; the first objective value equals the oracle's NLL
    at the constant start; the Laplace variance at the true maps equals the
    oracle's at every voxel; the benchmark's ML leg (its default
    initialisation from the whole volume) starts from the oracle's initial
    maps and equals the oracle on 2048 sampled voxels."""
    torch = torch_cuda
    c, x = _inputs(orc, "map_brain", (192, 240, 256))
    del c["eps"]
    N = x.shape[1]
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    opts = dict(c["opts"], n_outer=2, n_gn=3, n_cg=16, init="const", init_const=[float(v) for v in y0])
    X = cuda(x)
    B1 = cuda(c["b1"].astype(np.float32))
    maps = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    rep, tr = _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, maps)
    torch.cuda.synchronize()
    y_gpu = maps.cpu().numpy().astype(np.float64)
    del maps
    _, rep0, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], {"mode": "ml", "n_gn": 0, "init": "const",
                                                              "init_const": y0})
    print("whole brain: first objective gpu", tr[0], "oracle NLL", rep0["nll"], "| report", rep)
    assert tr[0] == pytest.approx(rep0["nll"], rel=1e-6)
    S = opts["n_gn"] + 2
    for t in range(opts["n_outer"]):
        f = tr[t * S:t * S + opts["n_gn"] + 1]
        assert np.isfinite(f).all() and np.all(np.diff(f) < 0.0), (t, f)
    assert rep["nonfinite_voxels"] == 0 and rep["rejected"] == 0
    print("whole brain: oracle MAP fit of the whole volume", flush=True)
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    good = well_posed(y_orc, c["truth"])
    rel, ab, rms = map_errors(y_gpu, y_orc, good)
    rel_all, ab_all, _ = map_errors(y_gpu, y_orc)
    print("whole brain MAP 2x3x16 vs oracle: well-posed", good.mean(), "rel", rel, "all voxels rel", rel_all,
          "abs", ab_all)
    del y_gpu, y_orc
    assert (rel <= TOL).all() and (rel_all <= TOL).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(tr), fin) and np.allclose(tr[fin], tr_o[fin], rtol=1e-6)
    # (CG iteration counts may differ: in the first outer loop, without JTV
    # weights, one iteration solves each system and the FP64 residual then
    # vanishes, the FP32 one does not)
    assert rep["gn_done"] == rep_o["gn_done"] and rep_o["rejected"] == 0
    # Laplace variance at the true maps (JTV weights from them)
    truth = f32(c["truth"])
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], X, B1, opts, cuda(truth.astype(np.float32)), var)
    v = var.cpu().numpy().astype(np.float64)
    var_o = orc.uncertainty(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts, truth)
    ok = np.all(np.isfinite(var_o), axis=0)
    assert ok.mean() > 0.99 and np.array_equal(np.isfinite(v), np.isfinite(var_o))
    rv = np.abs(v[:, ok] - var_o[:, ok]) / var_o[:, ok]
    print("whole brain: variance at the truth, rel err max", rv.max(axis=1))
    assert rv.max() <= VAR_TOL
    del var
    # the benchmark's ML leg with its own options (default initialisation from
    # the whole volume): the initial maps equal the oracle's, and the fit
    # equals the oracle's on 2048 sampled voxels fitted one by one from them
    ml = {"mode": "ml", "n_gn": 20, "init": "default"}
    mm = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_fit(c["proto"], c["dims"], X, B1, dict(ml, n_gn=0), mm)
    torch.cuda.synchronize()
    init = mm[:, 0].cpu().numpy().astype(np.float64)
    print("whole brain: default init gpu", init, "oracle", y0)
    assert np.allclose(init, y0, rtol=1e-5, atol=1e-6)
    _lib.mpm_fit(c["proto"], c["dims"], X, B1, ml, mm)
    idx = np.sort(np.random.default_rng(106).choice(N, 2048, replace=False))
    ym = mm[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    del mm
    yo, _, _ = orc.fit(c["proto"], (len(idx), 1, 1), x[:, idx].astype(np.float64), c["b1"][idx],
                       {"mode": "ml", "n_gn": 20, "init": "const", "init_const": [float(v) for v in init]})
    good = well_posed(yo, c["truth"][:, idx])
    rel, _, _ = map_errors(ym, yo, good)
    print("whole brain ML on sampled voxels: well-posed", good.mean(), "rel", rel)
    assert good.mean() > 0.8 and (rel <= TOL).all()


GOLDEN_WHOLE_BRAIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "whole_brain_map_10x8x32.json")


def test_map_whole_brain_full_schedule_against_stored_oracle(torch_cuda, orc):
    """The benchmarked MAP fit itself: the whole-brain workload with the full
    10 x 8 x 32 schedule, in the benchmark's launch configuration, against the
    oracle's fit of the same volume (an hour of FP64 CPU time, stored by
    tests/golden/make_whole_brain_map.py): the objective trace, the report,
    the maps at 1024 seeded voxels and the per-map means over the whole volume
    (and, for the same fit of FP16 echoes stored with per-image offsets, the
    maps and means within the 1e-3 of reduced-precision storage);
    the Laplace variance at the GPU's maps at those voxels equals the oracle's
    computed at the same maps on the 5 x 5 x 5 crop around each voxel (clipped
    at the volume's faces; the JTV weights of a voxel and its neighbours depend
    on nothing farther), and the stored variance at the oracle's maps."""
    torch = torch_cuda
    g = json.load(open(GOLDEN_WHOLE_BRAIN))
    c, x = _inputs(orc, g["case"], tuple(g["dims"]))
    assert c["seed"] == g["seed"]
    del c["eps"]
    opts = g["options"]
    assert opts["lam"] == [float(v) for v in c["lam"]]
    N = x.shape[1]
    X = cuda(x)
    B1 = cuda(c["b1"].astype(np.float32))
    maps = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    rep, tr = _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, maps)
    torch.cuda.synchronize()
    tr_o = np.array([np.nan if v is None else v for v in g["trace"]])
    fin = np.isfinite(tr_o)
    print("whole brain 10x8x32: gpu objective", rep["objective"], "oracle", g["report"]["objective"], flush=True)
    assert np.array_equal(np.isfinite(tr), fin) and np.allclose(tr[fin], tr_o[fin], rtol=1e-6)
    assert rep["objective"] == pytest.approx(g["report"]["objective"], rel=1e-6)
    assert rep["gn_done"] == g["report"]["gn_done"] == 80
    assert rep["rejected"] == g["report"]["rejected"] == 0 and rep["nonfinite_voxels"] == 0
    idx = torch.tensor(g["sample_index"], dtype=torch.int64, device="cuda")
    ys = maps[:, idx].cpu().numpy().astype(np.float64)
    scale = np.array(g["map_max_abs"])
    rel = np.abs(ys - np.array(g["sample_maps"])).max(axis=1) / scale
    mean = maps.double().mean(dim=1).cpu().numpy()
    rel_mean = np.abs(mean - np.array(g["map_mean"])) / scale
    print("whole brain 10x8x32: sampled maps rel", rel, "means rel", rel_mean, flush=True)
    assert (rel <= TOL).all() and (rel_mean <= TOL).all()
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], X, B1, opts, maps, var)
    vg = var[:, idx].cpu().numpy().astype(np.float64)
    del var
    y = maps.cpu().numpy().astype(np.float64)
    # the benchmark's FP16 leg: echoes stored as FP16 of each image minus its
    # mean (mpm_pack_echoes); against the oracle's fit of the unquantised data,
    # within the 1e-3 of reduced-precision storage
    Q = torch.empty(X.shape, dtype=torch.float16, device="cuda")
    off = _lib.mpm_pack_echoes(X, Q)
    del X
    maps.zero_()
    rep16, _ = _lib.mpm_fit(c["proto"], c["dims"], Q, B1, dict(opts, echo_offset=off), maps)
    torch.cuda.synchronize()
    del Q, B1
    rel16 = np.abs(maps[:, idx].cpu().numpy().astype(np.float64) - np.array(g["sample_maps"])).max(axis=1) / scale
    mean16 = np.abs(maps.double().mean(dim=1).cpu().numpy() - np.array(g["map_mean"])) / scale
    del maps
    print("whole brain 10x8x32, FP16 echoes with offsets: sampled maps rel", rel16, "means rel", mean16, rep16,
          flush=True)
    assert (rel16 <= 1e-3).all() and (mean16 <= 1e-3).all()
    assert rep16["gn_done"] == 80 and rep16["nonfinite_voxels"] == 0
    nx, ny, nz = c["dims"]
    worst = 0.0
    for k, n in enumerate(g["sample_index"]):
        p = (n % nx, (n // nx) % ny, n // (nx * ny))
        rx, ry, rz = (range(max(0, q - 2), min(m, q + 3)) for q, m in zip(p, (nx, ny, nz)))
        cr = np.array([i + nx * (j + ny * l) for l in rz for j in ry for i in rx])
        cen = (p[0] - rx.start) + len(rx) * ((p[1] - ry.start) + len(ry) * (p[2] - rz.start))
        vo = orc.uncertainty(c["proto"], (len(rx), len(ry), len(rz)), x[:, cr].astype(np.float64), c["b1"][cr],
                             opts, y[:, cr])[:, cen]
        worst = max(worst, float(np.max(np.abs(vg[:, k] - vo) / vo)))
    # and against the oracle's at its own maps (those differ from the GPU's by
    # the map errors above)
    v_o = np.array(g["sample_var"])
    rv = (np.abs(vg - v_o) / v_o).max(axis=1)
    print("whole brain 10x8x32: sampled variance rel err max", worst, "| against the oracle's at its own maps", rv)
    assert worst <= VAR_TOL and (rv <= VAR_TOL).all()


GOLDEN_HIRES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hires_map_10x8x32.json")


def _fp16_echoes(orc, c, b1, planes=16):
    """s(truth) + sigma * eps in FP64, rounded to FP32 and then to FP16, a few
    z-planes at a time (as the stored oracle fit's generator builds them)."""
    nx, ny, nz = c["dims"]
    x16 = np.empty((c["eps"].shape[0], nx * ny * nz), np.float16)
    for z0 in range(0, nz, planes):
        sl = slice(z0 * nx * ny, min(nz, z0 + planes) * nx * ny)
        s = orc.simulate(c["proto"], c["truth"][:, sl], b1[sl])
        x16[:, sl] = (s + c["sigma"] * c["eps"][:, sl].astype(np.float64)).astype(np.float32).astype(np.float16)
    return x16


def test_map_high_resolution_full_schedule_against_stored_oracle(torch_cuda, orc):
    """The high-resolution workload (416 x 384 x 320 = 51 M voxels, FP16
    echoes, B1 0.7-1.3, noise 2% of the mean PD) with the full 10 x 8 x 32
    schedule, in the benchmark's launch configuration, against the oracle's
    fit of the same FP16 echoes (about three hours of FP64 CPU time, stored by
    tests/golden/make_hires_map.py): the objective trace, the report, the maps
    at 1024 seeded voxels and the per-map means over the whole volume; the
    Laplace variance at the GPU's maps at those voxels against the oracle's at
    the same maps on the 5 x 5 x 5 crop around each voxel (clipped at the
    volume's faces), and against the stored variance at the oracle's maps."""
    torch = torch_cuda
    g = json.load(open(GOLDEN_HIRES))
    c = synth.make_case(g["case"])
    assert c["seed"] == g["seed"] and list(c["dims"]) == g["dims"]
    opts = g["options"]
    assert opts["lam"] == [float(v) for v in c["lam"]]
    b1 = f32(c["b1"])
    x16 = _fp16_echoes(orc, c, b1)
    del c["eps"]
    N = x16.shape[1]
    X = torch.from_numpy(x16).cuda()
    B1 = cuda(b1.astype(np.float32))
    maps = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    print("high resolution 10x8x32: GPU fit", flush=True)
    rep, tr = _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, maps)
    torch.cuda.synchronize()
    tr_o = np.array([np.nan if v is None else v for v in g["trace"]])
    fin = np.isfinite(tr_o)
    print("high resolution 10x8x32: gpu objective", rep["objective"], "oracle", g["report"]["objective"], flush=True)
    assert np.array_equal(np.isfinite(tr), fin) and np.allclose(tr[fin], tr_o[fin], rtol=1e-6)
    assert rep["objective"] == pytest.approx(g["report"]["objective"], rel=1e-6)
    assert rep["gn_done"] == g["report"]["gn_done"] == 80
    assert rep["rejected"] == g["report"]["rejected"] == 0 and rep["nonfinite_voxels"] == 0
    idx = torch.tensor(g["sample_index"], dtype=torch.int64, device="cuda")
    scale = np.array(g["map_max_abs"])
    rel = np.abs(maps[:, idx].cpu().numpy().astype(np.float64) - np.array(g["sample_maps"])).max(axis=1) / scale
    rel_mean = np.abs(maps.double().mean(dim=1).cpu().numpy() - np.array(g["map_mean"])) / scale
    print("high resolution 10x8x32: sampled maps rel", rel, "means rel", rel_mean, flush=True)
    assert (rel <= TOL).all() and (rel_mean <= TOL).all()
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], X, B1, opts, maps, var)
    vg = var[:, idx].cpu().numpy().astype(np.float64)
    del var, X, B1
    y = maps.cpu().numpy().astype(np.float64)
    del maps
    nx, ny, nz = c["dims"]
    worst = 0.0
    for k, n in enumerate(g["sample_index"]):
        p = (n % nx, (n // nx) % ny, n // (nx * ny))
        rx, ry, rz = (range(max(0, q - 2), min(m, q + 3)) for q, m in zip(p, (nx, ny, nz)))
        cr = np.array([i + nx * (j + ny * l) for l in rz for j in ry for i in rx])
        cen = (p[0] - rx.start) + len(rx) * ((p[1] - ry.start) + len(ry) * (p[2] - rz.start))
        vo = orc.uncertainty(c["proto"], (len(rx), len(ry), len(rz)), x16[:, cr].astype(np.float64), b1[cr],
                             opts, y[:, cr])[:, cen]
        worst = max(worst, float(np.max(np.abs(vg[:, k] - vo) / vo)))
    v_o = np.array(g["sample_var"])
    rv = (np.abs(vg - v_o) / v_o).max(axis=1)
    print("high resolution 10x8x32: sampled variance rel err max", worst, "| against the oracle's at its own maps", rv)
    assert worst <= VAR_TOL and (rv <= VAR_TOL).all()


@pytest.mark.parametrize("which,seed,sched", [("tol_gn", 81, (3, 8, 16)), ("tol_outer", 82, (8, 2, 12))])
def test_map_early_stopping_parity(torch_cuda, orc, which, seed, sched):
    """Gain-based early stopping (Sec. 2.7): the same steps and loops are cut
    as by the oracle (the trace's NaN pattern), and the maps agree."""
    c, x = _inputs(orc, "map_brain", (24, 20, 12), seed=seed)
    opts = _const_opts(orc, c, x, n_outer=sched[0], n_gn=sched[1], n_cg=sched[2])
    opts[which] = 0.05
    y_gpu, y_orc, rep, rep_o = _compare(orc, torch_cuda, c, x, opts)
    print(which, "gpu", rep, "orc", rep_o)
    assert rep["outer_done"] == rep_o["outer_done"]
    full = sched[0] * sched[1]
    assert rep["gn_done"] < full  # something was cut


def test_map_high_resolution_launch_configuration(torch_cuda, orc):
    """The high-resolution workload at full size (416 x 384 x 320 = 51 M voxels,
    22 FP16 echoes, B1 0.7-1.3, sigma 2% of mean PD) in the launch
    configuration the benchmark times, checked where the oracle follows with
    inputs of its own (the dequantised FP16 echoes): the first objective value
    equals the oracle's NLL at the same constant maps (summed over z-slabs: the
    NLL is a sum over voxels); the objective does not rise within an outer
    loop; an ML fit equals the oracle's on 2048 sampled voxels fitted one by
    one; the Laplace variance at the true maps equals the oracle's at 1024
    sampled voxels, each computed on the 5 x 5 x 5 crop around it (the JTV
    weights of a voxel and of its neighbours depend on nothing farther)."""
    torch = torch_cuda
    c = synth.make_case("map_hires")
    nx, ny, nz = c["dims"]
    N, I = nx * ny * nz, 22
    truth = cuda(c["truth"].astype(np.float32))
    b1 = f32(c["b1"])
    B1 = cuda(b1.astype(np.float32))
    X = torch.empty((I, N), dtype=torch.float16, device="cuda")
    _lib.mpm_simulate(c["proto"], c["dims"], truth, B1, cuda(c["eps"]), X)
    del c["eps"]
    torch.cuda.synchronize()
    xh = X.cpu()  # the FP16 values the library reads
    y0 = [6.5, 0.0, 3.2, -4.2]
    opts = dict(c["opts"], n_outer=2, n_gn=3, n_cg=16, init="const", init_const=y0)
    maps = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    rep, tr = _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, maps)
    torch.cuda.synchronize()
    del maps
    nll, slab = 0.0, 20
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        xs = xh[:, z0 * nx * ny:z1 * nx * ny].float().numpy().astype(np.float64)
        _, r, _ = orc.fit(c["proto"], (nx, ny, z1 - z0), xs, b1[z0 * nx * ny:z1 * nx * ny],
                          {"mode": "ml", "n_gn": 0, "init": "const", "init_const": y0})
        nll += r["nll"]
    print("high resolution: first objective gpu", tr[0], "oracle NLL", nll, "| report", rep)
    assert tr[0] == pytest.approx(nll, rel=1e-6)
    S = opts["n_gn"] + 2
    for t in range(opts["n_outer"]):
        f = tr[t * S:t * S + opts["n_gn"] + 1]
        f = f[np.isfinite(f)]
        assert np.all(np.diff(f) <= 1e-9 * np.abs(f[:-1])), (t, f)
    assert rep["nonfinite_voxels"] == 0
    rng = np.random.default_rng(105)
    # ML on sampled voxels
    ml = {"mode": "ml", "n_gn": 20, "init": "const", "init_const": y0}
    mm = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_fit(c["proto"], c["dims"], X, B1, ml, mm)
    idx = np.sort(rng.choice(N, 2048, replace=False))
    ym = mm[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    del mm
    xs = xh[:, torch.from_numpy(idx)].float().numpy().astype(np.float64)
    yo, _, _ = orc.fit(c["proto"], (len(idx), 1, 1), xs, b1[idx], ml)
    good = well_posed(yo, c["truth"][:, idx])
    rel, ab, _ = map_errors(ym, yo, good)
    print("high resolution ML on sampled voxels: well-posed", good.mean(), "rel", rel)
    assert good.mean() > 0.6 and (rel <= TOL).all()  # sigma 2%: more ML optima leave the truth
    # Laplace variance at the true maps, on sampled interior voxels
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], X, B1, opts, truth, var)
    tz, ty, tx = (rng.integers(2, n - 2, 1024) for n in (nz, ny, nx))
    cen = tx + nx * (ty + ny * tz)
    vg = var[:, torch.from_numpy(cen).cuda()].cpu().numpy().astype(np.float64)
    del var
    tt = f32(c["truth"])
    off = np.array([(dx + nx * (dy + ny * dz)) for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)])
    worst = 0.0
    for k, n in enumerate(cen):
        cr = n + off  # crop voxels, x fastest
        vo = orc.uncertainty(c["proto"], (5, 5, 5), xh[:, torch.from_numpy(cr)].float().numpy().astype(np.float64),
                             b1[cr], opts, tt[:, cr])
        v = vo[:, 62]  # the centre of the crop
        worst = max(worst, float(np.max(np.abs(vg[:, k] - v) / v)))
    print("high resolution: variance at the truth on sampled voxels, rel err max", worst)
    assert worst <= VAR_TOL
