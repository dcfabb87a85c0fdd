"""GPU parity of mpm_fit_voxelwise, the ML fit with a protocol per voxel
(the convergence experiment of Sec. 3.1), against the oracle's
orc_fit_voxelwise; and its agreement with mpm_fit when every voxel has the
same protocol."""
import math

import numpy as np
import pytest

from conftest import cuda, f32, map_errors, well_posed
from paper_2102_01604_amd import _lib, synth
from test_oracle_voxelwise import _e1_problems, _random_protocols, _shape, _simulate_voxelwise

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _gpu(torch, shape, tr, flip, te, x, opts, maps0=None, dtype=None):
    N = tr.shape[1]
    X = cuda(x.astype(np.float32))
    if dtype is not None:
        X = X.to(dtype)
    maps = cuda(maps0.astype(np.float32)) if maps0 is not None else torch.zeros((4, N), dtype=torch.float32,
                                                                               device="cuda")
    inc = torch.zeros(N, dtype=torch.int32, device="cuda")
    nll = torch.zeros(N, dtype=torch.float32, device="cuda")
    o = dict(opts, mode="ml")
    if maps0 is not None:
        o["init"] = "maps"
    rep = _lib.mpm_fit_voxelwise(shape, cuda(tr.astype(np.float32)), cuda(flip.astype(np.float32)),
                                 cuda(te.astype(np.float32)), X, o, maps, inc, nll)
    torch.cuda.synchronize()
    return (maps.cpu().numpy().astype(np.float64), inc.cpu().numpy(), nll.cpu().numpy().astype(np.float64), rep)


def _jittered_problem(orc, N, seed, n_echoes=(6, 6, 6), mt=(0, 0, 1), frac=0.01):
    rng = np.random.default_rng(seed)
    tr, flip, te = _random_protocols(rng, N, n_echoes)
    truth = synth.maps_iid((1, 1, N), rng)
    sigma = frac * float(np.exp(truth[0]).mean())
    x = _simulate_voxelwise(orc, n_echoes, mt, tr, flip, te, truth) + sigma * rng.normal(size=(sum(n_echoes), N))
    # the arrays the device reads, as the oracle sees them
    return _shape(n_echoes, mt, sigma), f32(tr), f32(flip), f32(te), f32(x), truth


def test_simulate_voxelwise_matches_oracle(torch_cuda, orc):
    torch = torch_cuda
    rng = np.random.default_rng(70)
    N = 2048
    tr, flip, te = (f32(a) for a in _random_protocols(rng, N, (8, 8, 6)))
    truth = f32(synth.maps_iid((1, 1, N), rng))
    shape = _shape((8, 8, 6), (0, 0, 1), 2.0)
    noise = f32(rng.normal(size=(22, N)))
    out = torch.empty((22, N), dtype=torch.float32, device="cuda")
    _lib.mpm_simulate_voxelwise(shape, cuda(tr.astype(np.float32)), cuda(flip.astype(np.float32)),
                                cuda(te.astype(np.float32)), cuda(truth.astype(np.float32)),
                                cuda(noise.astype(np.float32)), out)
    ref = _simulate_voxelwise(orc, (8, 8, 6), (0, 0, 1), tr, flip, te, truth) + 2.0 * noise
    got = out.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()
    tr[0, 5] = -1.0
    _lib.mpm_simulate_voxelwise(shape, cuda(tr.astype(np.float32)), cuda(flip.astype(np.float32)),
                                cuda(te.astype(np.float32)), cuda(truth.astype(np.float32)), None, out)
    got = out.cpu().numpy()
    assert np.all(np.isnan(got[:, 5])) and np.all(np.isfinite(np.delete(got, 5, axis=1)))


@pytest.mark.parametrize("loading", ["proposed", "plus", "gn"])
def test_random_protocols_parity(torch_cuda, orc, loading):
    shape, tr, flip, te, x, truth = _jittered_problem(orc, 3000, 71)
    y0 = [6.5, 0.0, 3.2, -4.2]
    opts = {"n_gn": 20, "init": "const", "init_const": y0, "loading": loading}
    yg, ig, ng, rg = _gpu(torch_cuda, shape, tr, flip, te, x, opts)
    yo, io, no, ro = orc.fit_voxelwise(shape, tr, flip, te, x, dict(opts, init_const=f32(y0)), rise_rel=1e-5)
    good = well_posed(yo, truth)
    rel, ab, rms = map_errors(yg, yo, good)
    print(loading, "rel", rel, "well-posed", good.mean(), "| gpu", rg, "| orc", ro)
    assert good.mean() > 0.8
    assert (rel <= TOL).all()
    assert np.allclose(ng[good], no[good], rtol=1e-4, atol=1e-4)
    assert rg["nonfinite_voxels"] == ro["nonfinite_voxels"]


def test_shared_protocol_matches_mpm_fit(torch_cuda, orc):
    """All voxels on one protocol: the same Newton steps as the ML kernel of mpm_fit."""
    torch = torch_cuda
    rng = np.random.default_rng(72)
    N = 4096
    proto = synth.protocol()
    truth = synth.maps_iid((1, 1, N), rng)
    sigma = 0.01 * float(np.exp(truth[0]).mean())
    proto["sigma"] = [sigma] * 22
    x = f32(orc.simulate(proto, truth) + sigma * rng.normal(size=(22, N)))
    opts = {"mode": "ml", "n_gn": 20, "init": "const", "init_const": [6.5, 0.0, 3.2, -4.2]}
    m0 = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    rep0 = _lib.mpm_fit(proto, (N, 1, 1), cuda(x.astype(np.float32)), None, opts, m0)[0]
    tr = np.repeat(f32(proto["tr"])[:, None], N, axis=1)
    flip = np.repeat(f32(proto["flip"])[:, None], N, axis=1)
    te = np.repeat(f32(proto["te"])[:, None], N, axis=1)
    y1, inc, nll, rep1 = _gpu(torch, _shape((8, 8, 6), (0, 0, 1), sigma), tr, flip, te, x, opts)
    y0 = m0.cpu().numpy().astype(np.float64)
    d = np.abs(y1 - y0).max(axis=1) / np.abs(y0).max(axis=1)
    print("voxelwise vs mpm_fit rel", d, "nll", rep1["nll"], rep0["nll"])
    # the same per-echo arithmetic on the same values: bit for bit
    assert np.array_equal(y1, y0)
    assert rep1["nll"] == rep0["nll"]


def test_convergence_experiment_statistics(torch_cuda, orc):
    """Sec. 3.1 on the GPU: the proposed loadings keep the NLL from rising in
    far more voxels than Gauss-Newton; the per-voxel rise flags agree with the
    oracle's (same 1e-5 threshold) up to a few voxels near the threshold."""
    rng = np.random.default_rng(2104)
    N, n_it = 2000, 300
    y, tr, flip, te = _e1_problems(rng, N)
    with np.errstate(all="ignore"):
        x = _simulate_voxelwise(orc, (5, 5, 5), (0, 0, 1), tr, flip, te, y) + rng.normal(size=(15, N))
    shape = _shape((5, 5, 5), (0, 0, 1), 1.0)
    tr, flip, te, x = f32(tr), f32(flip), f32(te), f32(x)
    frac = {}
    for load in ("proposed", "plus", "gn"):
        opts = {"n_gn": n_it, "init": "const", "init_const": [0.0] * 4, "loading": load}
        _, ig, _, rg = _gpu(torch_cuda, shape, tr, flip, te, x, opts)
        with np.errstate(all="ignore"):
            _, io, _, ro = orc.fit_voxelwise(shape, tr, flip, te, x, opts, rise_rel=1e-5)
        fg, fo = float((ig > 0).mean()), float((io > 0).mean())
        agree = float(((ig > 0) == (io > 0)).mean())
        print(f"{load}: voxels whose NLL rose gpu {fg:.4f} oracle {fo:.4f}, flags agree {agree:.4f}")
        frac[load] = fg
        assert abs(fg - fo) <= 0.03 and agree >= 0.95
    assert frac["gn"] > 0.3
    assert frac["proposed"] < 0.25 * frac["gn"]


def test_invalid_voxel_protocols_are_isolated(torch_cuda, orc):
    shape, tr, flip, te, x, truth = _jittered_problem(orc, 512, 73)
    opts = {"n_gn": 10, "init": "const", "init_const": [6.5, 0.0, 3.2, -4.2]}
    y_ok, _, _, _ = _gpu(torch_cuda, shape, tr, flip, te, x, opts)
    tr2, flip2, te2 = tr.copy(), flip.copy(), te.copy()
    tr2[1, 10] = 0.0
    flip2[0, 20] = math.pi
    te2[3, 30] = float("nan")
    te2[7, 40] = -1e-3
    y, inc, nll, rep = _gpu(torch_cuda, shape, tr2, flip2, te2, x, opts)
    bad = [10, 20, 30, 40]
    assert np.all(np.isnan(y[:, bad])) and np.all(np.isnan(nll[bad]))
    keep = np.setdiff1d(np.arange(512), bad)
    assert np.array_equal(y[:, keep], y_ok[:, keep])
    assert rep["nonfinite_voxels"] >= 4


def test_generic_shape_and_fp16_and_start_maps(torch_cuda, orc):
    """5 contrasts with up to 9 echoes (echoes read from memory at every
    step), FP16 echo storage, start from given maps."""
    torch = torch_cuda
    ne, mt = (9, 4, 4, 4, 4), (0, 0, 1, 0, 1)
    rng = np.random.default_rng(74)
    N = 1024
    C = len(ne)
    tr = rng.uniform(0.015, 0.040, (C, N))
    lo, hi = np.array([4.0, 18.0, 4.0, 10.0, 8.0])[:, None], np.array([8.0, 30.0, 8.0, 14.0, 12.0])[:, None]
    flip = np.deg2rad(lo + (hi - lo) * rng.uniform(size=(C, N)))
    te = np.concatenate([np.sort(rng.uniform(0.002, 0.020, (e, N)), axis=0) for e in ne])
    truth = synth.maps_iid((1, 1, N), rng)
    sigma = 0.01 * float(np.exp(truth[0]).mean())
    x = _simulate_voxelwise(orc, ne, mt, tr, flip, te, truth) + sigma * rng.normal(size=(sum(ne), N))
    shape = _shape(ne, mt, sigma)
    tr, flip, te = f32(tr), f32(flip), f32(te)
    xq = torch.from_numpy(x.astype(np.float32)).half().float().numpy().astype(np.float64)
    y0 = f32(truth + rng.uniform(-0.2, 0.2, truth.shape))
    opts = {"n_gn": 15}
    yg, _, _, _ = _gpu(torch, shape, tr, flip, te, x, opts, maps0=y0, dtype=torch.float16)
    yo, _, _, _ = orc.fit_voxelwise(shape, tr, flip, te, xq, {"n_gn": 15}, maps0=y0)
    good = well_posed(yo, truth)
    rel, _, _ = map_errors(yg, yo, good)
    print("generic shape, FP16 storage: rel", rel, "well-posed", good.mean())
    assert good.mean() > 0.9 and (rel <= TOL).all()


def test_single_voxel_and_zero_steps(torch_cuda, orc):
    shape, tr, flip, te, x, truth = _jittered_problem(orc, 1, 75)
    y0 = [6.5, 0.0, 3.2, -4.2]
    for steps in (0, 12):
        opts = {"n_gn": steps, "init": "const", "init_const": y0}
        yg, ig, ng, rg = _gpu(torch_cuda, shape, tr, flip, te, x, opts)
        yo, io, no, ro = orc.fit_voxelwise(shape, tr, flip, te, x, dict(opts, init_const=f32(y0)), rise_rel=1e-5)
        assert np.allclose(yg, yo, rtol=1e-5, atol=1e-5)
        assert ng[0] == pytest.approx(no[0], rel=1e-4)
        if steps == 0:
            assert np.array_equal(yg[:, 0], f32(y0)) and ig[0] == 0 and rg["degenerate_voxels"] == 0

