"""Resuming a MAP fit on the GPU (option start_outer): a fit stopped after t
outer loops and resumed from its maps at loop t equals the uninterrupted fit
bit for bit (maps, the trace from loop t on, the report), plain, projected
and through the serving queue; and it equals the oracle's resumed fit."""
import numpy as np
import pytest

from conftest import cuda, map_errors, well_posed
from paper_2102_01604_amd import _lib
from test_gpu_map import _const_opts, _inputs
from test_gpu_proj import _problem

pytestmark = pytest.mark.gpu
T, T0 = 5, 2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _run(torch, fit, opts, maps0):
    maps = cuda(maps0.astype(np.float32))
    rep, tr = fit(opts, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy().astype(np.float64), rep, np.asarray(tr)


def _check(full, part, res, S):
    (yf, rf, tf), (_, rp, _), (yr, rr, tr) = full, part, res
    assert np.array_equal(yr, yf)
    assert np.all(np.isnan(tr[:T0 * S]))
    assert np.array_equal(tr[T0 * S:], tf[T0 * S:], equal_nan=True)
    assert rr["outer_done"] == T - T0
    assert rr["gn_done"] == rf["gn_done"] - rp["gn_done"]
    assert rr["cg_done"] == rf["cg_done"] - rp["cg_done"]
    assert rr["objective"] == rf["objective"]


def _resume(torch, fit, opts, y0):
    full = _run(torch, fit, dict(opts, n_outer=T), y0)
    part = _run(torch, fit, dict(opts, n_outer=T0), y0)
    res = _run(torch, fit, dict(opts, n_outer=T, start_outer=T0, init="maps"), part[0])
    _check(full, part, res, opts["n_gn"] + 2)
    return part, res


def test_resumed_fit_equals_uninterrupted_and_oracle(torch_cuda, orc):
    torch = torch_cuda
    c, x = _inputs(orc, "map_brain", (40, 36, 20), seed=111)
    opts = _const_opts(orc, c, x, n_gn=3, n_cg=12)
    opts["lam"] = list(np.array(c["lam"]) * 20)
    y0 = np.repeat(np.asarray(opts["init_const"], dtype=np.float64)[:, None], x.shape[1], 1)
    X, B1 = cuda(x), cuda(c["b1"].astype(np.float32))
    fit = lambda o, m: _lib.mpm_fit(c["proto"], c["dims"], X, B1, dict(o, init="maps"), m)
    part, res = _resume(torch, fit, opts, y0)
    # the oracle resumed from the same (FP32) maps
    ro = dict(opts, n_outer=T, start_outer=T0, init="maps")
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], ro, maps0=part[0])
    good = well_posed(y_orc, c["truth"])
    rel, _, _ = map_errors(res[0], y_orc, good)
    print("resumed fit vs oracle: rel", rel, "well-posed", good.mean())
    assert good.mean() > 0.8 and (rel <= 1e-4).all()
    fin = np.isfinite(tr_o)
    assert np.array_equal(np.isfinite(res[2]), fin)
    assert np.allclose(res[2][fin], tr_o[fin], rtol=1e-5)
    # the serving queue runs the resumed request to the same maps
    out = cuda(part[0].astype(np.float32))
    with _lib.MpmServer(hbm_budget=4 << 30, max_active=2) as srv:
        t = srv.submit(c["proto"], c["dims"], X, B1, ro, out)
        got = None
        for _ in range(100000):
            srv.step()
            got = srv.poll(t)
            if got is not None:
                break
        assert got is not None
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.float64), res[0])
    assert got["objective"] == res[1]["objective"]


def test_resumed_projected_fit(torch_cuda, orc):
    torch = torch_cuda
    c, spaces, x = _problem(orc, dims=(20, 18, 10), seed=112)
    y0c = orc.default_init_projected(c["proto"], c["dims"], spaces, x.astype(np.float64), c["b1"])
    y0 = np.repeat(np.asarray(y0c, dtype=np.float32).astype(np.float64)[:, None], int(np.prod(c["dims"])), 1)
    opts = {"mode": "map", "n_gn": 3, "n_cg": 10, "lam": list(np.array(c["lam"]) * 20), "max_halvings": 4}
    X, B1 = cuda(x.astype(np.float32)), cuda(c["b1"].astype(np.float32))
    fit = lambda o, m: _lib.mpm_fit_projected(c["proto"], c["dims"], spaces, X, B1, dict(o, init="maps"), m)
    _resume(torch, fit, opts, y0)
