"""Pins for the noise estimation of Sec. 2.7 (a two-class Rician mixture per
acquired volume; lower-mean class = background; geometric mean of the
variances over echoes; initial maps from the other class's means).

* the scaled Bessel functions match scipy's i0e / i1e;
* the histogram equals numpy's over the same range (no value near an edge);
* on samples drawn from a known Rayleigh + Rice mixture the EM recovers the
  weights, the noise sigma and the tissue nu within their sampling error;
* EM never increases the histogram's negative log-likelihood;
* the classes' weighted means add up to the histogram's mean;
* on a synthetic head in air the per-contrast sigma is the true one within
  2% (each image's within 6%), the per-contrast value is the geometric mean
  of its echoes' values, and the foreground means and initial maps
  approximate the head's own mean signal and its default initialisation.
"""
import numpy as np
import pytest
from scipy import special

from paper_2102_01604_amd import synth


def test_bessel_matches_scipy(orc):
    for z in np.concatenate([[0.0, 1e-300, 1e-8], np.logspace(-6, 3, 400), [24.999, 25.0, 25.001, 5e3, 1e6]]):
        i0e, i1e = orc.bessel_i01e(z)
        assert abs(i0e - special.i0e(z)) <= 1e-14 * special.i0e(z), z
        assert abs(i1e - special.i1e(z)) <= 1e-14 * special.i1e(z) + 1e-300, z


def test_histogram_matches_numpy(orc):
    rng = np.random.default_rng(5)
    nb = 512
    x = rng.gamma(2.0, 30.0, 200000).astype(np.float32).astype(np.float64)
    width = float(x.max()) / nb
    frac = (x / width) % 1.0
    x = x[(np.minimum(frac, 1.0 - frac) > 1e-3) | (x == x.max())]  # no value at an inner edge
    x[::1000] = np.nan  # not observations
    x[1::1000] = -1.0
    counts, scale = orc.histogram(x, nb)
    ok = np.isfinite(x) & (x >= 0)
    mx = float(np.float32(x[ok].max()))
    assert scale == pytest.approx(nb / mx, rel=1e-7)
    ref, _ = np.histogram(x[ok], bins=nb, range=(0.0, nb / np.float64(scale)))
    ref[-1] += int((x[ok] >= nb / np.float64(scale)).sum())
    assert np.array_equal(counts, ref)
    assert counts.sum() == ok.sum()


def _mixture_sample(rng, n, w_bg, sigma, nu):
    nb = int(round(w_bg * n))
    bg = np.hypot(sigma * rng.standard_normal(nb), sigma * rng.standard_normal(nb))
    fg = np.hypot(nu + sigma * rng.standard_normal(n - nb), sigma * rng.standard_normal(n - nb))
    return np.concatenate([bg, fg])


@pytest.mark.parametrize("snr,w_bg", [(20.0, 0.4), (8.0, 0.6), (40.0, 0.25)])
def test_em_recovers_a_known_mixture(orc, snr, w_bg):
    rng = np.random.default_rng(int(snr))
    sigma, n = 10.0, 400000
    x = _mixture_sample(rng, n, w_bg, sigma, snr * sigma)
    counts, scale = orc.histogram(x, 2048)
    r = orc.rice_mixture(counts, scale, 300)
    bg = int(np.argmin(r["mean"]))
    print(snr, w_bg, r)
    assert r["pi"][bg] == pytest.approx(w_bg, abs=0.01)
    assert r["sigma"][bg] == pytest.approx(sigma, rel=0.01)
    assert r["nu"][bg] == 0.0  # the background class carries no signal (R-rice)
    assert r["nu"][1 - bg] == pytest.approx(snr * sigma, rel=0.01)
    assert r["sigma"][1 - bg] == pytest.approx(sigma, rel=0.03)
    # the classes' weighted means add up to the histogram's mean (responsibilities sum to 1)
    c = (np.arange(counts.size) + 0.5) / scale
    assert r["pi"] @ r["mean"] == pytest.approx((counts * c).sum() / counts.sum(), rel=1e-9)
    # EM: the negative log-likelihood never increases
    d = np.diff(r["nll"])
    assert np.all(d <= 1e-10 * np.abs(r["nll"][:-1]))
    assert r["nll"][-1] < r["nll"][0]


def test_noise_estimate_on_a_head_in_air(orc):
    c = synth.head_case((48, 44, 40), seed=61, noise_frac=0.02)
    s = orc.simulate(c["proto"], c["truth"], c["b1"])
    x = synth.magnitudes(s, c).astype(np.float32).astype(np.float64)
    est = orc.estimate_noise(c["proto"], x, c["b1"], nbins=1024, n_iter=200)
    print("sigma true", c["sigma"], "per contrast", est["sigma_contrast"], "per image", est["sigma_image"])
    assert np.allclose(est["sigma_contrast"], c["sigma"], rtol=0.02)
    assert np.allclose(est["sigma_image"], c["sigma"], rtol=0.06)
    first = np.cumsum([0] + c["proto"]["n_echoes"])
    for k in range(3):
        si = est["sigma_image"][first[k]:first[k + 1]]
        assert est["sigma_contrast"][k] == pytest.approx(np.exp(np.log(si).mean()), rel=1e-13)
    # one Rician class stands in for the whole head (three tissues and smooth
    # variation): its mean approximates the head's mean magnitude, and the
    # initial maps approximate the default initialisation applied to the head
    head = x[:, c["mask"]].mean(axis=1)
    print("foreground / head mean", est["fg_mean"] / head)
    assert np.allclose(est["fg_mean"], head, rtol=0.1)
    y_head = orc.default_init(c["proto"], x[:, c["mask"]], None if c["b1"] is None else c["b1"][c["mask"]])
    print("y0", est["y0"], "from the head alone", y_head)
    assert np.allclose(est["y0"], y_head, atol=0.1)
