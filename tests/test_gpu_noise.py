"""GPU parity of mpm_estimate_noise (the noise estimation of Sec. 2.7)
against the oracle: histograms bit for bit (the bin of a value is decided in
FP32 on both sides), the EM mixtures, sigma per image and per contrast, the
foreground means and the initial maps (both sides in FP64; 1e-9)."""
import numpy as np
import pytest

from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu
NB, IT = 1024, 200


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _head(orc, dims, seed, noise_frac=0.02):
    c = synth.head_case(dims, seed=seed, noise_frac=noise_frac)
    s = orc.simulate(c["proto"], c["truth"], c["b1"])
    x = synth.magnitudes(s, c).astype(np.float32)
    return c, x


def _check(orc, torch, c, x, dtype=None, nbins=NB, n_iter=IT):
    X = torch.from_numpy(x).cuda()
    if dtype is not None:
        X = X.to(dtype)
    xs = X.float().cpu().numpy().astype(np.float64)  # the values the GPU reads
    b1 = None if c["b1"] is None else torch.from_numpy(c["b1"].astype(np.float32)).cuda()
    b1s = None if c["b1"] is None else c["b1"].astype(np.float32).astype(np.float64)
    g = _lib.mpm_estimate_noise(c["proto"], c["dims"], X, b1, nbins=nbins, n_iter=n_iter, want_hist=True)
    torch.cuda.synchronize()
    I = xs.shape[0]
    hist = np.asarray(g["hist"], dtype=np.int64).reshape(I, nbins)
    worst = 0.0
    for i in range(I):
        counts, scale = orc.histogram(xs[i], nbins)
        assert np.array_equal(hist[i], counts), i
        r = orc.rice_mixture(counts, scale, n_iter)
        f = g["fits"][i]
        for k in ("pi", "nu", "sigma", "mean"):
            d = np.abs(np.asarray(f[k]) - r[k]) / np.maximum(np.abs(r[k]), 1e-300)
            worst = max(worst, float(np.where(r[k] == 0, np.abs(f[k]), d).max()))
        assert f["nll"] == pytest.approx(r["nll"][-1], rel=1e-9)
    o = orc.estimate_noise(c["proto"], xs, b1s, nbins=nbins, n_iter=n_iter)
    print("worst mixture parameter rel diff", worst, "sigma per contrast", g["sigma_contrast"], o["sigma_contrast"])
    assert worst <= 1e-9
    assert np.allclose(g["sigma_image"], o["sigma_image"], rtol=1e-9)
    assert np.allclose(g["sigma_contrast"], o["sigma_contrast"], rtol=1e-9)
    assert np.allclose(g["fg_mean"], o["fg_mean"], rtol=1e-9)
    assert np.allclose(g["init_const"], o["y0"], atol=2e-6)  # the library returns FP32 initial maps
    return g, o


def test_noise_parity_head(torch_cuda, orc):
    c, x = _head(orc, (48, 44, 40), 61)
    g, _ = _check(orc, torch_cuda, c, x)
    assert np.allclose(g["sigma_contrast"], c["sigma"], rtol=0.02)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_noise_parity_reduced_precision(torch_cuda, orc, dtype):
    torch = torch_cuda
    c, x = _head(orc, (40, 36, 30), 62)
    _check(orc, torch, c, x, dtype={"f16": torch.float16, "bf16": torch.bfloat16}[dtype])


def test_noise_parity_large_ragged_with_missing_values(torch_cuda, orc):
    """1.4 M voxels (many workgroups per image, a ragged last one), some NaN
    and negative values (not observations), 4096 bins, 20 iterations."""
    c, x = _head(orc, (131, 117, 93), 63)
    rng = np.random.default_rng(64)
    idx = rng.integers(0, x.size, 5000)
    x.reshape(-1)[idx[:2500]] = np.nan
    x.reshape(-1)[idx[2500:]] = -3.0
    _check(orc, torch_cuda, c, x, nbins=4096, n_iter=20)


def test_noise_edge_cases(torch_cuda, orc):
    torch = torch_cuda
    c, x = _head(orc, (9, 7, 5), 65)
    _check(orc, torch, c, x, nbins=16, n_iter=0)  # smallest histogram, the start alone
    # an image with a single value cannot be split: an error, nothing written
    x2 = x.copy()
    x2[3] = 7.0
    with pytest.raises(_lib.MpmError, match="split"):
        _lib.mpm_estimate_noise(c["proto"], c["dims"], torch.from_numpy(x2).cuda())
    # no value > 0 in an image: also an error
    x2[3] = 0.0
    with pytest.raises(_lib.MpmError, match="split"):
        _lib.mpm_estimate_noise(c["proto"], c["dims"], torch.from_numpy(x2).cuda())
