"""GPU parity on the less common paths: missing (non-finite) echoes, other
protocol shapes, the Proposed+ and Gauss-Newton loadings, acceptance off,
early CG stop, the default initialisation in the MAP fit, reduced-precision
uncertainty."""
import numpy as np
import pytest

from conftest import cuda, f32, map_errors, observations, well_posed
from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _gpu(torch, c, x, opts, dtype=None):
    X = cuda(x.astype(np.float32))
    if dtype is not None:
        X = X.to(dtype)
    b1 = None if c["b1"] is None else cuda(c["b1"].astype(np.float32))
    maps = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
    rep, trace = _lib.mpm_fit(c["proto"], c["dims"], X, b1, opts, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy().astype(np.float64), rep, trace


def _compare(orc, torch, c, x, opts, tol=TOL, mask=None):
    y_gpu, rep, tr = _gpu(torch, c, x, opts)
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    good = well_posed(y_orc, c["truth"]) if mask is None else mask
    rel, ab, rms = map_errors(y_gpu, y_orc, good)
    print(c["dims"], opts.get("mode"), "rel", rel, "abs", ab, "| gpu", rep, "| orc", rep_o)
    assert (rel <= tol).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(tr), fin)
    assert np.allclose(tr[fin], tr_o[fin], rtol=1e-5)
    return y_gpu, y_orc, rep, rep_o


@pytest.mark.parametrize("mode", ["ml", "map"])
def test_missing_echoes(torch_cuda, orc, mode):
    c = synth.make_case("map_brain", dims=(36, 20, 10), seed=41)
    c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    rng = np.random.default_rng(1)
    x[rng.random(x.shape) < 0.02] = np.nan
    x[:, 77] = np.inf  # a voxel with no observation at all
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    opts = (dict(c["opts"], n_outer=3, n_gn=3, n_cg=10) if mode == "map" else {"mode": "ml", "n_gn": 12})
    opts.update(init="const", init_const=[float(v) for v in y0])
    y_gpu, y_orc, rep, rep_o = _compare(orc, torch_cuda, c, x, opts)
    if mode == "ml":
        assert rep["degenerate_voxels"] == rep_o["degenerate_voxels"] >= 1
        assert np.allclose(y_gpu[:, 77], y0)


# Echo counts per contrast covering every register shape of the kernels
# (4 x 8, 4 x 16, 8 x 8) and protocols beyond them, whose echoes are read from
# memory at every use.
SHAPES = [(2, 2, 2, 2, 2), (12, 12, 10), (1, 1, 1), (8, 8, 6, 8, 8, 6), (16, 16, 17), (9, 9, 9, 9, 9)]


def _shape_case(orc, echoes, dims):
    n = len(echoes)
    flips = [6.0, 21.0, 6.0, 10.0, 15.0, 8.0][:n]
    mt = [0, 0, 1, 0, 0, 1][:n]
    c = synth.make_case("map_brain", dims=dims, seed=43, echoes=echoes)
    c["proto"] = synth.protocol(echoes=echoes, flips_deg=flips, mt=mt, sigma=c["sigma"])
    c["b1"] = f32(c["b1"])
    return c, observations(orc, c)


@pytest.mark.parametrize("echoes", SHAPES[1:2] + SHAPES[3:])
def test_map_protocol_shapes(torch_cuda, orc, echoes):
    c, x = _shape_case(orc, echoes, (26, 20, 9))
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    opts = dict(c["opts"], n_outer=2, n_gn=3, n_cg=10, init="const", init_const=[float(v) for v in y0])
    _compare(orc, torch_cuda, c, x, opts)


@pytest.mark.parametrize("echoes", SHAPES)
def test_ml_protocol_shapes(torch_cuda, orc, echoes):
    n = len(echoes)
    flips = [6.0, 21.0, 6.0, 10.0, 15.0, 8.0][:n]
    mt = [0, 0, 1, 0, 0, 1][:n]
    c = synth.make_case("ml32", dims=(40, 12, 5), seed=42, echoes=echoes)
    c["proto"] = synth.protocol(echoes=echoes, flips_deg=flips, mt=mt, sigma=c["sigma"])
    x = observations(orc, c)
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64)))
    opts = {"mode": "ml", "n_gn": 15, "init": "const", "init_const": y0}
    y_orc = orc.fit(c["proto"], c["dims"], x.astype(np.float64), None, opts)[0]
    good = well_posed(y_orc, c["truth"])
    if not good.any():  # under-determined protocol (3 observations, 4 unknowns): every voxel degenerate
        good = np.ones_like(good)
    _compare(orc, torch_cuda, c, x, opts, mask=good)


def test_ml_proposed_plus_loading(torch_cuda, orc):
    """The Proposed+ loading (absolute row sums of the signal's second
    derivatives, Sec. 2.3) through the ML kernel, bench-like protocol and B1."""
    c = synth.make_case("map_brain", dims=(40, 30, 8), seed=46)
    c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    _compare(orc, torch_cuda, c, x, {"mode": "ml", "n_gn": 15, "init": "const", "init_const": [float(v) for v in y0],
                                      "loading": "plus"})


def test_ml_gauss_newton_loading(torch_cuda, orc):
    c = synth.make_case("ml32", dims=(30, 20, 4), seed=43)
    x = observations(orc, c)
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64)))
    opts = {"mode": "ml", "n_gn": 10, "init": "const", "init_const": y0, "loading": "gn"}
    y_gpu, rep, tr = _gpu(torch_cuda, c, x, opts)
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), None, opts)
    # plain Gauss-Newton is not monotone: compare where the oracle stayed near the truth
    good = well_posed(y_orc, c["truth"], tol=0.5) & np.all(np.isfinite(y_orc), axis=0)
    rel, _, _ = map_errors(y_gpu, y_orc, good)
    print("gn loading rel", rel, good.mean())
    assert (rel <= 1e-3).all()


@pytest.mark.parametrize("variant", ["accept_off", "cg_stop", "default_init", "halvings_0", "loading_plus"])
def test_map_variants(torch_cuda, orc, variant):
    c = synth.make_case("map_brain", dims=(30, 26, 14), seed=44)
    c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    opts = dict(c["opts"], n_outer=3, n_gn=4, n_cg=12, init="const", init_const=[float(v) for v in y0])
    if variant == "accept_off":
        opts["max_halvings"] = -1
    elif variant == "cg_stop":
        opts["cg_stop"] = 1e-6
    elif variant == "default_init":
        opts["init"] = "default"
    elif variant == "loading_plus":
        opts["loading"] = "plus"
    else:
        opts["max_halvings"] = 0
    _compare(orc, torch_cuda, c, x, opts)


def test_uncertainty_reduced_precision(torch_cuda, orc):
    torch = torch_cuda
    c = synth.make_case("map_brain", dims=(20, 18, 8), seed=45)
    c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    xq = torch.from_numpy(x).half().float().numpy().astype(np.float64)
    maps = f32(orc.fit(c["proto"], c["dims"], xq, c["b1"], dict(c["opts"], n_outer=2, n_gn=3, n_cg=8))[0])
    var_o = orc.uncertainty(c["proto"], c["dims"], xq, c["b1"], c["opts"], maps)
    N = x.shape[1]
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], cuda(x).half(), cuda(c["b1"].astype(np.float32)), c["opts"],
                         cuda(maps.astype(np.float32)), var, None)
    v = var.cpu().numpy().astype(np.float64)
    ok = np.isfinite(var_o)
    assert np.array_equal(np.isfinite(v), ok)
    assert (np.abs(v[ok] - var_o[ok]) / var_o[ok]).max() <= 1e-4
