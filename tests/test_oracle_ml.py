"""Pins for the oracle's ML fit (SPGR-ML, Sec. 2.3-2.4, Sec. 3.1, Sec. 4.1).

* exact recovery of the ground truth from noise-free data;
* no per-voxel NLL increase at the synthetic tissue parameter ranges (the paper's
  monotonicity claim, Sec. 4.1) and far fewer non-monotone voxels than plain
  Gauss-Newton on the paper's convergence experiment (Sec. 3.1);
* the ML optimum's mean NLL equals the chi-square expectation (I - K)/2 and
  lies below the NLL of the truth, I/2 (the over-fitting remark of Sec. 4.1);
* the 1-D monotonic-step condition eq. cond_monotonic along each parameter;
* the default initialisation lands near the truth.
"""
import math

import numpy as np
import pytest

from conftest import observations
from paper_2102_01604_amd import synth


def _case(n=2048, seed=1, noise_frac=0.01):
    return synth.make_case(dims=(n, 1, 1), seed=seed, noise_frac=noise_frac)


def test_exact_recovery_noise_free(orc):
    c = _case(2048, seed=11)
    x = orc.simulate(c["proto"], c["truth"])
    maps, rep, trace = orc.fit(c["proto"], c["dims"], x, None, {"mode": "ml", "n_gn": 50})
    assert rep["degenerate_voxels"] == 0 and rep["nonfinite_voxels"] == 0
    assert np.abs(maps - c["truth"]).max() <= 1e-9


def test_no_nll_increase_at_tissue_ranges(orc):
    c = _case(4096, seed=12)
    x = observations(orc, c).astype(np.float64)
    _, rep, trace = orc.fit(c["proto"], c["dims"], x, None, {"mode": "ml", "n_gn": 60})
    assert rep["nll_increases"] == 0
    assert np.all(np.diff(trace) <= 1e-12 * trace[:-1])


def test_chi_square_of_ml_optimum(orc):
    c = _case(8192, seed=13)
    x = observations(orc, c).astype(np.float64)
    I, K = x.shape[0], 4
    maps, rep, _ = orc.fit(c["proto"], c["dims"], x, None, {"mode": "ml", "n_gn": 60})
    mean_nll = rep["nll"] / x.shape[1]
    # E[min NLL] = (I - K)/2 for a well-posed least-squares fit; truth gives I/2
    assert abs(mean_nll - (I - K) / 2) < 0.15
    s_true = orc.simulate(c["proto"], c["truth"])
    nll_true = (((s_true - x) / c["sigma"]) ** 2).sum() / 2 / x.shape[1]
    assert abs(nll_true - I / 2) < 0.15
    assert mean_nll < nll_true


def _e1_voxel(rng):
    """One voxel of the convergence experiment (Sec. 3.1): log-parameters,
    log TR and log TE ~ U[-5, 5], flips ~ U[0, pi/4], three contrasts (one MT)
    with five echoes, sigma^2 = 1, initial maps 0."""
    y = rng.uniform(-5, 5, 4)
    tr = np.exp(rng.uniform(-5, 5, 3))
    flip = rng.uniform(0, math.pi / 4, 3)
    te = np.exp(rng.uniform(-5, 5, 15))
    proto = {"n_echoes": [5, 5, 5], "tr": list(tr), "flip": list(flip), "mt": [0, 0, 1],
             "te": list(te), "sigma": [1.0] * 15}
    return proto, y


def _nonmonotone(trace):
    if not np.all(np.isfinite(trace)):
        return True
    return bool(np.any(np.diff(trace) > 1e-10 * np.abs(trace[:-1]) + 1e-300))


def test_convergence_experiment_proposed_vs_gauss_newton(orc):
    """Sec. 3.1: the proposed loadings (diagonal and Proposed+ row sums) against
    plain Gauss-Newton on random single-voxel problems."""
    rng = np.random.default_rng(2102)
    n_vox, n_it = 300, 400
    bad = {"proposed": 0, "gn": 0, "plus": 0}
    for _ in range(n_vox):
        proto, y = _e1_voxel(rng)
        s = orc.simulate(proto, y.reshape(4, 1))
        x = s + rng.normal(size=s.shape)
        for load in bad:
            with np.errstate(all="ignore"):
                _, _, trace = orc.fit(proto, (1, 1, 1), x, None,
                                      {"mode": "ml", "n_gn": n_it, "init": "const",
                                       "init_const": (0, 0, 0, 0), "loading": load})
            bad[load] += _nonmonotone(trace)
    print(f"non-monotone voxels over {n_vox}: proposed {bad['proposed']}, proposed+ {bad['plus']}, "
          f"Gauss-Newton {bad['gn']}")
    assert bad["gn"] > 0.3 * n_vox
    assert bad["proposed"] < 0.25 * bad["gn"]
    # the majorising row-sum loading is at least as safe as the diagonal one
    assert bad["plus"] <= bad["proposed"]


def test_monotone_step_condition_1d(orc):
    """eq. cond_monotonic: |g_k / P~_kk| <= |y_k - y_k*| along each parameter
    with the others at the optimum (noise-free data, so the optimum is the
    truth)."""
    rng = np.random.default_rng(5)
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    violations = 0
    total = 0
    for _ in range(20):
        ys = synth.encode(rng.uniform(500, 1000, 1), rng.uniform(0.5, 1.5, 1),
                          rng.uniform(10, 40, 1), rng.uniform(0.005, 0.02, 1))[:, 0]
        x = orc.simulate(proto, ys.reshape(4, 1))[:, 0]
        for k in range(4):
            for dv in np.linspace(-3, 3, 25):
                if abs(dv) < 1e-9:
                    continue
                y = ys.copy()
                y[k] += dv
                _, g, P = orc.lik_voxel(proto, x, y)
                total += 1
                if abs(g[k] / P[k, k]) > abs(dv) * (1 + 1e-9):
                    violations += 1
    print(f"1-D step-condition violations: {violations}/{total}")
    assert violations == 0


def test_default_init_near_truth(orc):
    # constant maps at the centre of the synthetic tissue ranges, noise-free
    n = 64
    truth = synth.encode(np.full(n, 750.0), np.full(n, 1.0), np.full(n, 25.0), np.full(n, 0.0125))
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    x = orc.simulate(proto, truth)
    y0 = orc.default_init(proto, x)
    assert math.exp(y0[0]) == pytest.approx(750.0, rel=0.05)
    assert math.exp(y0[1]) == pytest.approx(1.0, rel=0.05)
    assert math.exp(y0[2]) == pytest.approx(25.0, rel=0.05)
    assert 1 / (1 + math.exp(-y0[3])) == pytest.approx(0.0125, rel=0.1)


def test_default_init_scales_flips_by_mean_b1(orc):
    """R-init applies the small-angle forms to the nominal flips times the mean
    transmit field: noise-free data made with a constant field b1 = c gives
    the same initial maps as the same data with every flip multiplied by c and
    no field, and a field with the same mean but spatial variation gives that
    init too; with the field the init lands near the truth, without it the
    flip error biases R1 (the closed forms scale R1 with 1/alpha^2)."""
    n = 64
    truth = synth.encode(np.full(n, 750.0), np.full(n, 1.0), np.full(n, 25.0), np.full(n, 0.0125))
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    cval = 1.15
    b1 = np.full(n, cval)
    x = orc.simulate(proto, truth, b1)
    y_field = orc.default_init(proto, x, b1)
    scaled = dict(proto, flip=[f * cval for f in proto["flip"]])
    y_scaled = orc.default_init(scaled, x)
    assert np.allclose(y_field, y_scaled, rtol=1e-12, atol=1e-12)
    ramp = cval + 0.1 * np.linspace(-1.0, 1.0, n)  # mean cval
    assert np.allclose(orc.default_init(proto, x, ramp), y_field, rtol=1e-12, atol=1e-12)
    assert math.exp(y_field[1]) == pytest.approx(1.0, rel=0.05)
    y_none = orc.default_init(proto, x)
    assert abs(math.exp(y_none[1]) - 1.0) > 0.2


def test_missing_echo_equals_removed_image(orc):
    """A non-finite echo is a missing observation: fitting with image 9 set to
    NaN equals fitting with image 9 removed from the protocol."""
    c = _case(256, seed=14)
    x = observations(orc, c).astype(np.float64)
    xm = x.copy()
    xm[9, :] = np.nan
    proto2 = dict(c["proto"])
    proto2["n_echoes"] = [6, 5, 6]
    proto2["te"] = [t for i, t in enumerate(c["proto"]["te"]) if i != 9]
    proto2["sigma"] = [s for i, s in enumerate(c["proto"]["sigma"]) if i != 9]
    x2 = np.delete(x, 9, axis=0)
    y0 = orc.default_init(c["proto"], x)
    opts = {"mode": "ml", "n_gn": 15, "init": "const", "init_const": y0}
    m1, r1, _ = orc.fit(c["proto"], c["dims"], xm, None, opts)
    m2, r2, _ = orc.fit(proto2, c["dims"], x2, None, opts)
    assert np.abs(m1 - m2).max() <= 1e-12
    assert r1["nll"] == pytest.approx(r2["nll"], rel=1e-13)
    # the default initialisation averages the finite values only
    assert np.allclose(orc.default_init(c["proto"], xm), orc.default_init(proto2, x2), rtol=1e-12)
