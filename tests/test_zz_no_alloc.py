"""mpm_fit_noalloc (its workspace in the library's fixed device scratch: no
allocation) against mpm_fit, through the C ABI: the same maps, report and
objective trace bit for bit (the same kernels in the same launch shapes), on
two calls in a row whose second is smaller, so the second runs on the first
call's leftover scratch contents; ML and JTV-MAP, with the default
initialisation (its partial sums also live in the scratch).  A fit larger
than the scratch is rejected before any device work."""
import numpy as np
import pytest

from conftest import cuda, f32, observations
from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _run(fn, torch, c, X, B1, opts):
    maps = torch.zeros((4, X.shape[1]), dtype=torch.float32, device="cuda")
    rep, tr = fn(c["proto"], c["dims"], X, B1, opts, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy(), rep, tr


@pytest.mark.parametrize("mode", ["map", "ml"])
def test_noalloc_equals_mpm_fit(torch_cuda, orc, mode):
    torch = torch_cuda
    for dims, seed in (((64, 60, 48), 61), ((40, 27, 19), 62)):  # the second call is smaller
        c = synth.make_case("map_brain", dims=dims, seed=seed)
        c["b1"] = f32(c["b1"])
        x = observations(orc, c)
        if mode == "map":
            opts = dict(c["opts"], n_outer=3, n_gn=3, n_cg=12)
        else:
            opts = {"mode": "ml", "n_gn": 20}
        X = cuda(x.astype(np.float32))
        B1 = cuda(c["b1"].astype(np.float32))
        print(mode, dims, "noalloc", flush=True)
        y_na, rep_na, tr_na = _run(_lib.mpm_fit_noalloc, torch, c, X, B1, opts)
        print(mode, dims, "mpm_fit", flush=True)
        y_ref, rep_ref, tr_ref = _run(_lib.mpm_fit, torch, c, X, B1, opts)
        print(mode, dims, rep_na, flush=True)
        assert np.array_equal(y_na, y_ref)
        assert rep_na == rep_ref
        assert np.array_equal(tr_na, tr_ref, equal_nan=True)
        assert np.isfinite(y_na).all() and rep_na["nonfinite_voxels"] == 0


def test_noalloc_rejects_fit_beyond_scratch(torch_cuda, orc):
    """A MAP fit of 100 x 100 x 60 voxels needs about 74 MB of workspace, more
    than the 64 MiB scratch: MPM_ERR_OUT_OF_MEMORY, maps untouched; the next
    call that fits still equals mpm_fit."""
    torch = torch_cuda
    c = synth.make_case("map_brain", dims=(100, 100, 60), seed=63)
    I, N = c["eps"].shape
    X = torch.ones((I, N), dtype=torch.float32, device="cuda")
    maps = torch.full((4, N), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.MpmError) as err:
        _lib.mpm_fit_noalloc(c["proto"], c["dims"], X, None, dict(c["opts"], n_outer=1, n_gn=1, n_cg=1), maps)
    print(err.value)
    assert err.value.status == 3 and "scratch" in str(err.value)
    torch.cuda.synchronize()
    assert bool((maps == 7.0).all())
    c = synth.make_case("map_brain", dims=(24, 20, 12), seed=64)
    c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    X = cuda(x.astype(np.float32))
    B1 = cuda(c["b1"].astype(np.float32))
    opts = dict(c["opts"], n_outer=2, n_gn=2, n_cg=8)
    y_na, rep_na, _ = _run(_lib.mpm_fit_noalloc, torch, c, X, B1, opts)
    y_ref, rep_ref, _ = _run(_lib.mpm_fit, torch, c, X, B1, opts)
    assert np.array_equal(y_na, y_ref) and rep_na == rep_ref
