"""Pins for the oracle's fit with a protocol per voxel (the convergence
experiment of Sec. 3.1: every voxel has its own TR, flip angles and echo
times).

* with every voxel on the same protocol it is the ML fit of that protocol
  (maps, per-voxel NLL rises, final NLL);
* noise-free echoes simulated voxel by voxel with each voxel's own protocol
  are recovered exactly (a mixed-up per-voxel index would not be);
* on the experiment's random problems the proposed loading rises in far fewer
  voxels than plain Gauss-Newton, and the flags equal those of single-voxel
  fits.
"""
import numpy as np

from paper_2102_01604_amd import synth


def _shape(n_echoes, mt, sigma):
    return {"n_echoes": list(n_echoes), "mt": list(mt), "sigma": [float(sigma)] * int(sum(n_echoes))}


def test_shared_protocol_equals_ml_fit(orc):
    rng = np.random.default_rng(31)
    N = 2000
    proto = synth.protocol()
    proto["sigma"] = [5.0] * 22
    truth = synth.maps_iid((1, 1, N), rng)
    x = orc.simulate(proto, truth) + 5.0 * rng.normal(size=(22, N))
    opts = {"mode": "ml", "n_gn": 15, "init": "const", "init_const": [6.5, 0.0, 3.2, -4.0]}
    m0, rep0, _ = orc.fit(proto, (N, 1, 1), x, None, opts)
    tr = np.repeat(np.asarray(proto["tr"])[:, None], N, axis=1)
    flip = np.repeat(np.asarray(proto["flip"])[:, None], N, axis=1)
    te = np.repeat(np.asarray(proto["te"])[:, None], N, axis=1)
    m1, inc, nll, rep1 = orc.fit_voxelwise(_shape(proto["n_echoes"], proto["mt"], 5.0), tr, flip, te, x, opts)
    assert np.array_equal(m1, m0)
    assert int(inc.sum()) == rep0["nll_increases"] == rep1["nll_increases"]
    assert float(np.cumsum(nll)[-1]) == rep1["nll"] == rep0["nll"]  # serial sums in voxel order


def _random_protocols(rng, N, n_echoes=(6, 6, 6)):
    """Jittered versions of the paper's protocol (PDw, T1w, MTw): TR 15-40 ms,
    flips 4-8 / 18-30 / 4-8 degrees (two well-separated non-MT flips keep A
    and R1 identifiable), sorted TEs in 2-20 ms."""
    C = len(n_echoes)
    tr = rng.uniform(0.015, 0.040, (C, N))
    lo, hi = np.array([4.0, 18.0, 4.0])[:, None], np.array([8.0, 30.0, 8.0])[:, None]
    flip = np.deg2rad(lo + (hi - lo) * rng.uniform(size=(C, N)))
    te = np.concatenate([np.sort(rng.uniform(0.002, 0.020, (e, N)), axis=0) for e in n_echoes])
    return tr, flip, te


def _simulate_voxelwise(orc, n_echoes, mt, tr, flip, te, maps):
    N = maps.shape[1]
    out = np.empty((sum(n_echoes), N))
    for n in range(N):
        p = {"n_echoes": list(n_echoes), "tr": list(tr[:, n]), "flip": list(flip[:, n]), "mt": list(mt),
             "te": list(te[:, n]), "sigma": [1.0] * sum(n_echoes)}
        out[:, n] = orc.simulate(p, maps[:, n:n + 1])[:, 0]
    return out


def test_noise_free_recovery_with_per_voxel_protocols(orc):
    rng = np.random.default_rng(32)
    N = 400
    mt = (0, 0, 1)
    tr, flip, te = _random_protocols(rng, N)
    truth = synth.maps_iid((1, 1, N), rng)
    x = _simulate_voxelwise(orc, (6, 6, 6), mt, tr, flip, te, truth)
    y0 = truth + rng.uniform(-0.3, 0.3, truth.shape)
    maps, inc, nll, rep = orc.fit_voxelwise(_shape((6, 6, 6), mt, 1.0), tr, flip, te, x, {"n_gn": 40}, maps0=y0)
    assert np.abs(maps - truth).max() <= 1e-8
    assert nll.max() <= 1e-12 * (x ** 2).sum(axis=0).max()
    assert rep["nonfinite_voxels"] == 0 and rep["degenerate_voxels"] == 0
    # the same data fitted with the protocols of other voxels does not come back
    perm = np.roll(np.arange(N), 1)
    wrong, _, _, _ = orc.fit_voxelwise(_shape((6, 6, 6), mt, 1.0), tr[:, perm], flip[:, perm], te[:, perm], x,
                                       {"n_gn": 40}, maps0=y0)
    assert np.abs(wrong - truth).max() > 1e-2


def _e1_problems(rng, N):
    """Sec. 3.1: log-parameters, log TR and log TE ~ U[-5, 5], flips ~ U[0, pi/4],
    three contrasts of five echoes (the last with MT), sigma = 1, start 0."""
    return synth.e1_problems(N, rng)


def test_convergence_experiment_through_voxelwise_fit(orc):
    rng = np.random.default_rng(2103)
    N, n_it = 300, 400
    y, tr, flip, te = _e1_problems(rng, N)
    with np.errstate(all="ignore"):
        x = _simulate_voxelwise(orc, (5, 5, 5), (0, 0, 1), tr, flip, te, y) + rng.normal(size=(15, N))
    shape = _shape((5, 5, 5), (0, 0, 1), 1.0)
    rises = {}
    for load in ("proposed", "plus", "gn"):
        opts = {"n_gn": n_it, "init": "const", "init_const": [0.0] * 4, "loading": load}
        with np.errstate(all="ignore"):
            _, inc, _, _ = orc.fit_voxelwise(shape, tr, flip, te, x, opts, rise_rel=1e-10)
        rises[load] = inc > 0
        # the flags of the first voxels equal those of single-voxel fits
        for n in range(20):
            p = {"n_echoes": [5, 5, 5], "tr": list(tr[:, n]), "flip": list(flip[:, n]), "mt": [0, 0, 1],
                 "te": list(te[:, n]), "sigma": [1.0] * 15}
            with np.errstate(all="ignore"):
                _, _, trace = orc.fit(p, (1, 1, 1), x[:, n:n + 1], None, dict(opts, mode="ml"))
            fin = np.isfinite(trace)
            rose = bool(np.any((trace[1:] > trace[:-1] * (1 + 1e-10)) | (fin[:-1] & ~fin[1:])))
            assert rose == bool(rises[load][n]), (load, n)
    counts = {k: int(v.sum()) for k, v in rises.items()}
    print("voxels whose NLL rose:", counts, "of", N)
    assert counts["gn"] > 0.3 * N
    assert counts["proposed"] < 0.25 * counts["gn"]
    assert counts["plus"] <= counts["proposed"]
