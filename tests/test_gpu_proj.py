"""GPU parity of the spatial projection (Sec. 2.4, "Spatial projection"):
mpm_simulate_projected, mpm_fit_projected (ML, MAP, Proposed+ loading, FP32
and FP16 echo storage) and mpm_uncertainty_projected against the oracle, on
three contrasts of which two are acquired on moved and resized grids; and the
projected path with identity spaces against the plain GPU fit."""
import json
import os
import sys

import numpy as np
import pytest

from conftest import cuda, f32, map_errors, well_posed
from paper_2102_01604_amd import _lib, synth
from test_oracle_proj import _affine, _identity, _space

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _problem(orc, dims=(20, 18, 10), seed=61, fine=False):
    """Three contrasts: the reconstruction grid itself, and two grids moved by a
    rigid motion (one with an extra row and a slice less); echoes simulated by
    the oracle on the pulled maps and b1, rounded to FP32.  fine: the third
    grid has 0.55x the voxel size (and is rotated by up to 20 degrees), so the
    push gathers more acquisition voxels per workgroup tile than its LDS
    buffer holds and reads them from global memory."""
    rng = np.random.default_rng(seed)
    c = synth.make_case("map_brain", dims=dims, seed=seed)
    c["b1"] = f32(c["b1"])
    centre = (np.asarray(dims) - 1) / 2
    if fine:
        md = tuple(int(d / 0.55) + 6 for d in dims)
        A = _affine(rng, 20.0, 0.7, scale=(0.55, 0.55, 0.55))
        A[:, 3] = centre - A[:, :3] @ ((np.asarray(md) - 1) / 2) + rng.uniform(-0.7, 0.7, 3)  # centred, covers the FOV
        third = _space(md, A)
    else:
        third = _space((dims[0] + 1, dims[1], dims[2] - 1), _affine(rng, 3.0, 0.7, centre=centre))
    spaces = [_identity(dims),
              _space((dims[0], dims[1] + 1, dims[2]), _affine(rng, 3.0, 0.7, centre=centre)), third]
    xs = []
    for ci, sp in enumerate(spaces):
        yp = np.stack([orc.pull(dims, sp, c["truth"][k]) for k in range(4)])
        bp = orc.pull(dims, sp, c["b1"])
        first = sum(c["proto"]["n_echoes"][:ci])
        ne = c["proto"]["n_echoes"][ci]
        pc = dict(c["proto"], n_echoes=[ne], tr=[c["proto"]["tr"][ci]], flip=[c["proto"]["flip"][ci]],
                  mt=[c["proto"]["mt"][ci]], te=c["proto"]["te"][first:first + ne],
                  sigma=c["proto"]["sigma"][first:first + ne])
        s = orc.simulate(pc, yp, np.where(bp > 0, bp, 1.0)) + c["sigma"] * rng.normal(size=(ne, yp.shape[1]))
        xs.append(f32(s))
    return c, spaces, np.concatenate([v.reshape(-1) for v in xs])


def _gpu_fit(torch, c, spaces, x, opts, dtype=None):
    X = cuda(x.astype(np.float32))
    if dtype is not None:
        X = X.to(dtype)
    maps = torch.zeros((4, int(np.prod(c["dims"]))), dtype=torch.float32, device="cuda")
    rep, tr = _lib.mpm_fit_projected(c["proto"], c["dims"], spaces, X, cuda(c["b1"].astype(np.float32)), opts, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy().astype(np.float64), rep, tr


def _compare(orc, torch, c, spaces, x, opts, tol=TOL, dtype=None, x_orc=None):
    y_gpu, rep, tr = _gpu_fit(torch, c, spaces, x, opts, dtype)
    xo = x if x_orc is None else x_orc
    y_orc, rep_o, tr_o = orc.fit_projected(c["proto"], c["dims"], spaces, xo.astype(np.float64), c["b1"], opts)
    good = well_posed(y_orc, c["truth"])
    rel, ab, rms = map_errors(y_gpu, y_orc, good)
    print(c["dims"], opts.get("mode"), opts.get("loading", "proposed"), "rel", rel, "well-posed", good.mean(),
          "| gpu", rep, "| orc", rep_o)
    assert good.mean() > 0.8
    assert (rel <= tol).all()
    n = min(len(tr), len(tr_o))
    fin = np.isfinite(tr_o[:n])
    assert np.array_equal(np.isfinite(tr[:n]), fin)
    assert np.allclose(tr[:n][fin], tr_o[:n][fin], rtol=1e-5)
    return y_gpu, y_orc


def test_simulate_projected_parity(torch_cuda, orc):
    torch = torch_cuda
    c, spaces, _ = _problem(orc)
    sizes = [int(np.prod(sp["dims"])) * ne for sp, ne in zip(spaces, c["proto"]["n_echoes"])]
    out = torch.empty(sum(sizes), dtype=torch.float32, device="cuda")
    _lib.mpm_simulate_projected(c["proto"], c["dims"], spaces, cuda(c["truth"].astype(np.float32)),
                                cuda(c["b1"].astype(np.float32)), None, out)
    got = out.cpu().numpy().astype(np.float64)
    off = 0
    for ci, sp in enumerate(spaces):
        M = int(np.prod(sp["dims"]))
        ne = c["proto"]["n_echoes"][ci]
        yp = np.stack([orc.pull(c["dims"], sp, f32(c["truth"][k]).astype(np.float64)) for k in range(4)])
        bp = orc.pull(c["dims"], sp, c["b1"].astype(np.float64))
        inside = orc.pull(c["dims"], sp, np.ones(int(np.prod(c["dims"])))) > 0.5
        first = sum(c["proto"]["n_echoes"][:ci])
        pc = dict(c["proto"], n_echoes=[ne], tr=[c["proto"]["tr"][ci]], flip=[c["proto"]["flip"][ci]],
                  mt=[c["proto"]["mt"][ci]], te=c["proto"]["te"][first:first + ne],
                  sigma=c["proto"]["sigma"][first:first + ne])
        ref = orc.simulate(pc, yp, np.where(inside, bp, 1.0))
        g = got[off:off + ne * M].reshape(ne, M)
        assert np.all(np.isnan(g[:, ~inside])) and np.all(np.isfinite(g[:, inside]))
        assert np.abs(g[:, inside] - ref[:, inside]).max() <= 2e-5 * np.abs(ref).max()
        off += ne * M


@pytest.mark.parametrize("mode,loading", [("ml", "proposed"), ("ml", "plus"), ("map", "proposed")])
def test_projected_fit_parity(torch_cuda, orc, mode, loading):
    c, spaces, x = _problem(orc)
    y0 = f32(orc.default_init_projected(c["proto"], c["dims"], spaces, x.astype(np.float64), c["b1"]))
    opts = (dict(c["opts"], n_outer=3, n_gn=3, n_cg=10) if mode == "map" else {"mode": "ml", "n_gn": 12})
    opts.update(init="const", init_const=[float(v) for v in y0], loading=loading)
    _compare(orc, torch_cuda, c, spaces, x, opts)


def test_projected_fit_parity_fine_space(torch_cuda, orc):
    """A finer, strongly rotated acquisition grid: the push takes its global-memory path."""
    c, spaces, x = _problem(orc, dims=(16, 16, 10), seed=65, fine=True)
    y0 = f32(orc.default_init_projected(c["proto"], c["dims"], spaces, x.astype(np.float64), c["b1"]))
    for opts in ({"mode": "ml", "n_gn": 10}, dict(c["opts"], n_outer=2, n_gn=3, n_cg=10)):
        _compare(orc, torch_cuda, c, spaces, x, dict(opts, init="const", init_const=[float(v) for v in y0]))


def test_projected_default_init_matches_oracle(torch_cuda, orc):
    c, spaces, x = _problem(orc)
    opts = {"mode": "ml", "n_gn": 0, "init": "default"}
    y_gpu, _, _ = _gpu_fit(torch_cuda, c, spaces, x, opts)
    y0 = orc.default_init_projected(c["proto"], c["dims"], spaces, x.astype(np.float64), c["b1"])
    assert np.allclose(y_gpu[:, 0], y0, rtol=1e-5, atol=1e-6)


def test_projected_fp16_storage(torch_cuda, orc):
    torch = torch_cuda
    c, spaces, x = _problem(orc, seed=62)
    xq = torch.from_numpy(x).half().float().numpy().astype(np.float64)
    y0 = f32(orc.default_init_projected(c["proto"], c["dims"], spaces, xq, c["b1"]))
    opts = dict(c["opts"], n_outer=2, n_gn=3, n_cg=10, init="const", init_const=[float(v) for v in y0])
    # same arithmetic on the dequantised values: FP32 level
    _compare(orc, torch, c, spaces, x, opts, dtype=torch.float16, x_orc=xq)


def test_identity_projection_equals_plain_gpu_fit(torch_cuda, orc):
    torch = torch_cuda
    c = synth.make_case("map_brain", dims=(24, 20, 12), seed=63)
    c["b1"] = f32(c["b1"])
    x = f32(orc.simulate(c["proto"], c["truth"], c["b1"]) + c["sigma"] * c["eps"].astype(np.float64))
    y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
    spaces = [_identity(c["dims"])] * 3
    for opts in ({"mode": "ml", "n_gn": 10}, dict(c["opts"], n_outer=2, n_gn=3, n_cg=10)):
        opts = dict(opts, init="const", init_const=[float(v) for v in y0])
        X = cuda(x.astype(np.float32))
        m0 = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
        m1 = torch.zeros_like(m0)
        B1 = cuda(c["b1"].astype(np.float32))
        _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, m0)
        _lib.mpm_fit_projected(c["proto"], c["dims"], spaces, X.reshape(-1), B1, opts, m1)
        torch.cuda.synchronize()
        a, b = m0.cpu().numpy(), m1.cpu().numpy()
        good = well_posed(a.astype(np.float64), c["truth"])
        rel = np.abs(a - b)[:, good].max(axis=1) / np.abs(a).max(axis=1)
        print(opts["mode"], "plain vs identity-projected", rel)
        assert (rel <= 1e-5).all()


def test_projected_uncertainty_parity(torch_cuda, orc):
    torch = torch_cuda
    c, spaces, x = _problem(orc, seed=64)
    opts = dict(c["opts"], n_outer=2, n_gn=2, n_cg=8)
    maps = f32(orc.fit_projected(c["proto"], c["dims"], spaces, x.astype(np.float64), c["b1"], opts)[0])
    var_o = orc.uncertainty_projected(c["proto"], c["dims"], spaces, x.astype(np.float64), c["b1"], opts, maps)
    N = int(np.prod(c["dims"]))
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty_projected(c["proto"], c["dims"], spaces, cuda(x.astype(np.float32)),
                                   cuda(c["b1"].astype(np.float32)), opts, cuda(maps.astype(np.float32)), var)
    v = var.cpu().numpy().astype(np.float64)
    ok = np.isfinite(var_o)
    assert np.array_equal(np.isfinite(v), ok)
    rel = np.abs(v[ok] - var_o[ok]) / var_o[ok]
    print("projected variance rel max", rel.max())
    assert rel.max() <= 1e-4


def test_space_outside_the_field_of_view(torch_cuda, orc):
    """A contrast acquired entirely outside the reconstruction field of view
    carries no observation (all its echoes are missing): the fit equals the
    oracle's, every map stays finite, and the MT map keeps its start (only the
    MT contrast informs it)."""
    torch = torch_cuda
    c, spaces, x = _problem(orc, seed=66)
    far = dict(spaces[2])
    A = np.array(far["affine"], dtype=np.float64).reshape(3, 4).copy()
    A[:, 3] += np.array([1000.0, 0.0, 0.0])
    far["affine"] = A
    spaces = [spaces[0], spaces[1], far]
    sizes = [int(np.prod(sp["dims"])) * ne for sp, ne in zip(spaces, c["proto"]["n_echoes"])]
    X = torch.empty(sum(sizes), dtype=torch.float32, device="cuda")
    _lib.mpm_simulate_projected(c["proto"], c["dims"], spaces, cuda(c["truth"].astype(np.float32)),
                                cuda(c["b1"].astype(np.float32)), None, X)
    xs = X.cpu().numpy().astype(np.float64)
    assert np.all(np.isnan(xs[sizes[0] + sizes[1]:]))
    y0 = [6.6, 0.0, 3.2, -4.2]
    opts = dict(c["opts"], n_outer=2, n_gn=2, n_cg=8, init="const", init_const=y0)
    y_gpu, rep, _ = _gpu_fit(torch, c, spaces, xs, opts)
    y_orc, rep_o, _ = orc.fit_projected(c["proto"], c["dims"], spaces, xs, c["b1"], dict(opts, init_const=f32(y0)))
    assert np.all(np.isfinite(y_gpu)) and rep["nonfinite_voxels"] == 0
    rel, _, _ = map_errors(y_gpu, y_orc)
    print("outside-FOV contrast: rel", rel)
    assert (rel <= TOL).all()
    assert np.abs(y_gpu[3] - np.float32(y0[3])).max() <= 1e-6


GOLDEN_PROJECTED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "projected_map_10x8x32.json")


def test_projected_whole_brain_full_schedule_against_stored_oracle(torch_cuda, orc):
    """The benchmark's projected workload (maps on the 192 x 240 x 256 grid,
    T1w and MTw acquired on grids moved by its seeded rigid motions, MTw with 8
    slices fewer) with the full 10 x 8 x 32 schedule, against the oracle's fit
    of the same echoes (stored by tests/golden/make_projected_map.py, which
    builds them as this test does): the objective trace, the report, the maps
    at 1024 seeded voxels (those whose oracle maps lie within 1 of the truth)
    and at all 1024, the per-map means, and the Laplace variance at the GPU's
    maps against the stored variance at the oracle's maps (well-posed voxels)."""
    torch = torch_cuda
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from make_projected_map import projected_echoes, spaces_of
    g = json.load(open(GOLDEN_PROJECTED))
    c = synth.make_case(g["case"])
    del c["eps"]
    assert c["seed"] == g["seed"] and list(c["dims"]) == g["dims"]
    opts = g["options"]
    assert opts["lam"] == [float(v) for v in c["lam"]]
    b1 = f32(c["b1"])
    spaces = spaces_of(c["dims"])
    x = projected_echoes(orc, c, spaces, b1)
    N = int(np.prod(c["dims"]))
    X = cuda(x)
    del x
    B1 = cuda(b1.astype(np.float32))
    maps = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    print("projected whole brain 10x8x32: GPU fit", flush=True)
    rep, tr = _lib.mpm_fit_projected(c["proto"], c["dims"], spaces, X, B1, opts, maps)
    torch.cuda.synchronize()
    tr_o = np.array([np.nan if v is None else v for v in g["trace"]])
    fin = np.isfinite(tr_o)
    print("projected whole brain 10x8x32: gpu objective", rep["objective"], "oracle", g["report"]["objective"],
          "| gpu", rep, flush=True)
    assert np.array_equal(np.isfinite(tr), fin) and np.allclose(tr[fin], tr_o[fin], rtol=1e-6)
    assert rep["objective"] == pytest.approx(g["report"]["objective"], rel=1e-6)
    assert rep["gn_done"] == g["report"]["gn_done"] == 80 and rep["nonfinite_voxels"] == 0
    idx = np.array(g["sample_index"])
    ys = maps[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    yo = np.array(g["sample_maps"])
    good = well_posed(yo, c["truth"][:, idx])
    scale = np.array(g["map_max_abs"])
    rel = np.abs(ys - yo)[:, good].max(axis=1) / scale
    rel_all = np.abs(ys - yo).max(axis=1) / scale
    rel_mean = np.abs(maps.double().mean(dim=1).cpu().numpy() - np.array(g["map_mean"])) / scale
    print("projected whole brain 10x8x32: well-posed", good.mean(), "sampled maps rel", rel, "all sampled",
          rel_all, "means rel", rel_mean, flush=True)
    assert good.mean() > 0.8 and (rel <= TOL).all() and (rel_all <= TOL).all() and (rel_mean <= TOL).all()
    var = torch.empty((4, N), dtype=torch.float32, device="cuda")
    _lib.mpm_uncertainty_projected(c["proto"], c["dims"], spaces, X, B1, opts, maps, var)
    vg = var[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    v_o = np.array(g["sample_var"])
    ok = np.isfinite(v_o).all(axis=0) & good
    rv = (np.abs(vg - v_o)[:, ok] / v_o[:, ok]).max(axis=1)
    print("projected whole brain 10x8x32: sampled variance rel (well-posed voxels)", rv)
    assert (rv <= 1e-4).all()
