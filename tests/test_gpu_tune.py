"""mpm_autotune: the workgroup count of the MAP fit's CG sweep A picked per
grid size by timing.  A tuned size keeps oracle parity, its fits are
repeatable bit for bit, and the serving queue uses the same choice as
mpm_fit (each request's result equals its solo fit)."""
import numpy as np
import pytest

from conftest import cuda, f32
from paper_2102_01604_amd import _lib
from test_gpu_map import _compare, _const_opts, _inputs

pytestmark = pytest.mark.gpu
# a size no other test fits, large enough (4 tiles x 256 planes) that the
# candidates give different z-run lengths
DIMS = (64, 64, 256)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    yield torch
    _lib.mpm_autotune_clear()


def test_autotune_picks_a_candidate_and_keeps_parity(torch_cuda, orc):
    torch = torch_cuda
    r = _lib.mpm_autotune(DIMS, reps=3)
    print("autotune", r)
    n = len(r["target"])
    assert n >= 2 and 0 <= r["chosen"] < n
    assert all(t > 0 for t in r["ms"])
    assert r["ms"][r["chosen"]] == min(r["ms"])
    assert len(set(zip(r["workgroups"], r["planes_per_run"]))) == n  # distinct launches only
    c, x = _inputs(orc, "map_brain", DIMS, seed=91)
    opts = _const_opts(orc, c, x, n_outer=2, n_gn=2, n_cg=8)
    y1, _, rep, _ = _compare(orc, torch, c, x, opts)
    # repeatable: a second fit with the tuned shape is identical
    maps = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
    b1 = cuda(c["b1"].astype(np.float32))
    X = cuda(x.astype(np.float32))
    rep2, _ = _lib.mpm_fit(c["proto"], c["dims"], X, b1, opts, maps)
    torch.cuda.synchronize()
    assert np.array_equal(maps.cpu().numpy().astype(np.float64), y1)
    assert rep2["objective"] == rep["objective"]
    # the serving queue fits this size with the same shape
    out = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
    with _lib.MpmServer(hbm_budget=8 << 30, max_active=2) as srv:
        t = srv.submit(c["proto"], c["dims"], X, b1, opts, out)
        got = None
        for _ in range(100000):
            srv.step()
            got = srv.poll(t)
            if got is not None:
                break
        assert got is not None
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.float64), y1)
    assert got["objective"] == rep["objective"]
