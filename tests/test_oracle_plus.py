"""Pins for the "Proposed+" loading of the oracle (Sec. 2.3: load each echo's
term with the absolute row sums of the signal's second-derivative matrix,
diag(|H_s| 1), instead of its absolute diagonal).

* The full second-derivative matrix of the signal (the paper prints only the
  diagonal) equals central differences of the printed gradient, with and
  without an MT pulse, and is symmetric.
* P+ majorises the exact Hessian of the NLL in the Loewner order at random
  points far from the optimum (Sec. 2.3 cites this property for the row-sum
  choice only); the exact Hessian here comes from central differences of the
  oracle's gradient, not from the second derivatives.  The diagonal loading
  does not have this property: it fails at most such points.
* P+ - P differs from the diagonal loading by a non-negative diagonal.
"""
import numpy as np
import pytest

from paper_2102_01604_amd import synth

DEG = np.pi / 180


def _rand_point(rng):
    y = np.array([np.log(rng.uniform(300, 1500)), np.log(rng.uniform(0.2, 3.0)), np.log(rng.uniform(5, 80)),
                  np.log(rng.uniform(0.002, 0.05) / (1 - rng.uniform(0.002, 0.05)))])
    return y, rng.uniform(3, 35) * DEG, rng.uniform(0.01, 0.05), rng.uniform(0.002, 0.03)


@pytest.mark.parametrize("mt", [0, 1])
def test_signal_hessian_matches_fd_of_gradient(orc, mt):
    rng = np.random.default_rng(7 + mt)
    for _ in range(40):
        y, alpha, tr, te = _rand_point(rng)
        H = orc.spgr_hess(y, alpha, tr, te, mt)
        assert np.array_equal(H, H.T)
        fd = np.zeros((4, 4))
        for k in range(4):
            # Richardson-extrapolated central differences of the gradient
            def d(h):
                yp, ym = y.copy(), y.copy()
                yp[k] += h
                ym[k] -= h
                return (orc.spgr_derivs(yp, alpha, tr, te, mt)[1] - orc.spgr_derivs(ym, alpha, tr, te, mt)[1]) / (2 * h)
            fd[:, k] = (4 * d(1e-4) - d(2e-4)) / 3
        scale = np.abs(H).max()
        assert np.abs(H - fd).max() <= 1e-8 * scale
        if not mt:
            assert np.all(H[3, :] == 0) and np.all(H[:, 3] == 0)


def _fd_nll_hessian(orc, proto, x, y):
    H = np.zeros((4, 4))
    for k in range(4):
        def d(h):
            yp, ym = y.copy(), y.copy()
            yp[k] += h
            ym[k] -= h
            return (orc.lik_voxel(proto, x, yp)[1] - orc.lik_voxel(proto, x, ym)[1]) / (2 * h)
        H[:, k] = (4 * d(1e-5) - d(2e-5)) / 3
    return 0.5 * (H + H.T)


def test_plus_loading_majorises_the_nll_hessian(orc):
    rng = np.random.default_rng(11)
    proto = synth.protocol()
    proto["sigma"] = [7.5] * 22
    n, diag_fails = 200, 0
    for _ in range(n):
        ys = synth.encode(rng.uniform(500, 1000, 1), rng.uniform(0.5, 1.5, 1), rng.uniform(10, 40, 1),
                          rng.uniform(0.005, 0.02, 1))[:, 0]
        x = orc.simulate(proto, ys.reshape(4, 1))[:, 0] + rng.normal(0, 7.5, 22)
        y = ys + rng.normal(0, 1.0, 4)  # far from the optimum: large residuals
        Hn = _fd_nll_hessian(orc, proto, x, y)
        Pp = orc.lik_voxel(proto, x, y, loading="plus")[2]
        Pd = orc.lik_voxel(proto, x, y, loading="proposed")[2]
        scale = np.abs(Pp).max()
        assert np.linalg.eigvalsh(Pp - Hn).min() >= -1e-7 * scale
        diag_fails += np.linalg.eigvalsh(Pd - Hn).min() < -1e-7 * scale
        # same Gauss-Newton part, larger non-negative diagonal loading
        D = Pp - Pd
        assert np.allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-9 * scale)
        assert np.all(np.diag(D) >= -1e-12 * scale)
    print(f"diagonal loading fails to majorise at {diag_fails}/{n} points")
    assert diag_fails > n // 2
