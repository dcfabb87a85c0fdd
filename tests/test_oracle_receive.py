"""Pins for the receive field (Sec. 2.4 footnote: the whole signal of voxel n
is multiplied by the net receive field b-_n), option b1_receive.

* noise-free echoes made by multiplying the simulated signal by b- are fitted
  exactly (ML) when b- is given, and not when it is left out;
* an ML fit with b- equals the fit without it started from log A + log b-,
  with log b- taken off again (A enters the signal only as that product);
* MAP without a prior (lambda = 0) with b- equals ML with b-.
"""
import numpy as np

from paper_2102_01604_amd import synth


def _case(seed=91, dims=(16, 12, 8)):
    c = synth.make_case("map_brain", dims=dims, seed=seed)
    rng = np.random.default_rng(seed + 1)
    N = int(np.prod(dims))
    bm = synth.b1_field((dims[2], dims[1], dims[0]), rng, 0.7, 1.3, sigma=4.0)
    return c, bm, N


def test_noise_free_recovery_with_receive_field(orc):
    c, bm, N = _case()
    x = orc.simulate(c["proto"], c["truth"], c["b1"]) * bm[None, :]  # the footnote's definition
    rng = np.random.default_rng(3)
    y0 = c["truth"] + rng.uniform(-0.2, 0.2, c["truth"].shape)
    opts = {"mode": "ml", "n_gn": 40}
    m, rep, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], dict(opts, b1_receive=bm), maps0=y0)
    assert np.abs(m - c["truth"]).max() <= 1e-9 and rep["nll"] <= 1e-15 * (x ** 2).sum()
    m_off, _, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], opts, maps0=y0)
    assert np.abs(m_off[0] - c["truth"][0] - np.log(bm)).max() <= 1e-8  # absorbed into log A instead


def test_ml_with_receive_field_is_a_shift_of_log_a(orc):
    c, bm, N = _case(seed=93)
    x = orc.simulate(c["proto"], c["truth"], c["b1"]) * bm[None, :] + c["sigma"] * c["eps"].astype(np.float64)
    y0 = orc.default_init(c["proto"], x, c["b1"])
    start = np.repeat(np.asarray(y0)[:, None], N, axis=1)
    opts = {"mode": "ml", "n_gn": 15}
    m1, r1, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], dict(opts, b1_receive=bm), maps0=start)
    shifted = start.copy()
    shifted[0] += np.log(bm)
    m2, r2, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], opts, maps0=shifted)
    m2[0] -= np.log(bm)
    assert np.abs(m1 - m2).max() <= 1e-10
    assert r1["nll"] == np.float64(r2["nll"]) or abs(r1["nll"] - r2["nll"]) <= 1e-12 * r2["nll"]


def test_map_without_prior_equals_ml_with_receive_field(orc):
    c, bm, N = _case(seed=95)
    x = orc.simulate(c["proto"], c["truth"], c["b1"]) * bm[None, :] + c["sigma"] * c["eps"].astype(np.float64)
    y0 = [float(v) for v in orc.default_init(c["proto"], x, c["b1"])]
    ml, _, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], {"mode": "ml", "n_gn": 6, "init": "const",
                                                            "init_const": y0, "b1_receive": bm})
    mp, _, _ = orc.fit(c["proto"], c["dims"], x, c["b1"], {"mode": "map", "n_outer": 1, "n_gn": 6, "n_cg": 4,
                                                            "max_halvings": -1, "lam": [0.0] * 4, "init": "const",
                                                            "init_const": y0, "b1_receive": bm})
    assert np.abs(ml - mp).max() <= 1e-10 * np.abs(ml).max()
