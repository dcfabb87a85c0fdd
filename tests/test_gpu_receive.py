"""GPU parity of the fits and of the Laplace uncertainty with a net receive
field (Sec. 2.4 footnote: the signal of voxel n is multiplied by b-_n), option
b1_receive, against the FP64 oracle given the same FP32 field.  Same bars as
without it: 1e-4 on log maps over well-posed voxels, 1e-4 on variances."""
import numpy as np
import pytest

from conftest import cuda, f32, map_errors, well_posed
from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _inputs(orc, dims, seed):
    """map_brain recipe; echoes = s(truth) * b- + sigma * eps (FP32), b- a
    smooth field in [0.7, 1.3] like the transmit field."""
    c = synth.make_case("map_brain", dims=dims, seed=seed)
    c["b1"] = f32(c["b1"])
    bm = f32(synth.b1_field((dims[2], dims[1], dims[0]), np.random.default_rng(seed + 1000), 0.7, 1.3, sigma=4.0))
    s = orc.simulate(c["proto"], c["truth"], c["b1"]) * bm[None, :]
    x = (s + c["sigma"] * c["eps"].astype(np.float64)).astype(np.float32)
    return c, x, bm


def _opts(orc, c, x, bm, **kw):
    """Options with the constant start the oracle's default initialisation
    gives (the receive field left out of it on both sides)."""
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    o = dict(c["opts"], init="const", init_const=[float(v) for v in y0])
    o.update(kw)
    return dict(o, b1_receive=bm), dict(o, b1_receive=cuda(bm.astype(np.float32)))


def _gpu_fit(torch, c, x, opts):
    maps = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
    rep, trace = _lib.mpm_fit(c["proto"], c["dims"], cuda(x), cuda(c["b1"].astype(np.float32)), opts, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy().astype(np.float64), rep, trace


@pytest.mark.parametrize("mode,dims,sched", [("ml", (24, 20, 12), (1, 20, 0)), ("ml", (17, 13, 11), (1, 12, 0)),
                                             ("map", (24, 20, 12), (4, 4, 16)), ("map", (70, 9, 5), (3, 3, 8))])
def test_fit_parity_with_receive_field(torch_cuda, orc, mode, dims, sched):
    c, x, bm = _inputs(orc, dims, seed=101 + dims[0])
    T, J, K = sched
    o_orc, o_gpu = _opts(orc, c, x, bm, mode=mode, n_outer=T, n_gn=J, n_cg=max(K, 1))
    y_gpu, rep, tr = _gpu_fit(torch_cuda, c, x, o_gpu)
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], o_orc)
    good = well_posed(y_orc, c["truth"])
    rel, ab, rms = map_errors(y_gpu, y_orc, good)
    print(mode, dims, "well-posed", good.mean(), "rel", rel, "abs", ab, "rms", rms)
    assert good.mean() > 0.8
    assert (rel <= TOL).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(tr), fin)
    assert np.allclose(tr[fin], tr_o[fin], rtol=2e-5)
    assert rep["nonfinite_voxels"] == 0
    assert rep["objective"] == pytest.approx(rep_o["objective"], rel=2e-5)
    # leaving the field out changes the fit: it moves into log A instead
    o_off = {k: v for k, v in o_gpu.items() if k != "b1_receive"}
    y_off, _, _ = _gpu_fit(torch_cuda, c, x, o_off)
    shift = np.abs(y_off[0, good] - y_gpu[0, good] - np.log(bm[good]))
    print("log A shift vs log b-: median", np.median(shift))
    if mode == "ml":
        assert np.median(shift) <= 1e-3


def test_uncertainty_parity_with_receive_field(torch_cuda, orc):
    torch = torch_cuda
    c, x, bm = _inputs(orc, (30, 20, 10), seed=135)
    o_orc, o_gpu = _opts(orc, c, x, bm, mode="map", n_outer=3, n_gn=4, n_cg=8)
    y_orc, _, _ = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], o_orc)
    maps = f32(y_orc)
    var_o, mom_o = orc.uncertainty(c["proto"], c["dims"], x.astype(np.float64), c["b1"], o_orc, maps, moments=True)
    N = x.shape[1]
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    mom = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty(c["proto"], c["dims"], cuda(x), cuda(c["b1"].astype(np.float32)), o_gpu,
                         cuda(maps.astype(np.float32)), var, mom)
    v = var.cpu().numpy().astype(np.float64)
    m = mom.cpu().numpy().astype(np.float64)
    good = well_posed(y_orc, c["truth"]) & np.all(np.isfinite(var_o), axis=0)
    assert np.array_equal(np.isfinite(v), np.isfinite(var_o))
    rv = np.abs(v[:, good] - var_o[:, good]) / var_o[:, good]
    rm = np.abs(m[:, good] - mom_o[:, good]) / np.abs(mom_o[:, good])
    print("variance rel err max", rv.max(axis=1), "moments", rm.max(axis=1))
    assert rv.max() <= 1e-4 and rm.max() <= 1e-4


def test_server_fit_with_receive_field_equals_alone(torch_cuda, orc):
    """The serving loop passes the field through: the same result, bit for
    bit, as mpm_fit."""
    torch = torch_cuda
    c, x, bm = _inputs(orc, (32, 24, 10), seed=140)
    _, o_gpu = _opts(orc, c, x, bm, mode="map", n_outer=2, n_gn=3, n_cg=8)
    y_alone, rep_alone, _ = _gpu_fit(torch, c, x, o_gpu)
    X, b1 = cuda(x), cuda(c["b1"].astype(np.float32))
    maps = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
    with _lib.MpmServer(hbm_budget=8 << 30, max_active=2) as srv:
        t = srv.submit(c["proto"], c["dims"], X, b1, o_gpu, maps)
        rep = None
        for _ in range(10000):
            srv.step()
            rep = srv.poll(t)
            if rep is not None:
                break
        assert rep is not None
    torch.cuda.synchronize()
    assert np.array_equal(maps.cpu().numpy().astype(np.float64), y_alone)
    assert rep["objective"] == rep_alone["objective"]
