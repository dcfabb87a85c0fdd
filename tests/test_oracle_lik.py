"""Pins for the oracle's per-voxel likelihood block and 4x4 solve
(Sec. 2.3 eqs. chainrule / precond, Sec. 2.4).

g is pinned to finite differences of the NLL; the loaded approximate Hessian
is rebuilt from finite-difference derivatives of the signal alone (so a wrong
printed derivative, a dropped |.| or a missing 1/sigma^2 weight shows up); at a
zero-residual point it must equal the true Hessian of the NLL.
"""
import math

import numpy as np
import pytest

from paper_2102_01604_amd import synth


def _proto(sig=3.0):
    p = synth.protocol(echoes=(4, 3, 3))
    # unequal noise levels so that a missing 1/sigma^2 weight is caught
    p["sigma"] = [sig * (1.0 + 0.1 * i) for i in range(10)]
    return p


def _nll(orc, proto, x, y, b1=1.0):
    return orc.lik_voxel(proto, x, y, b1)[0]


def _signals(orc, proto, y, b1=1.0):
    out = []
    k0 = 0
    for c, ne in enumerate(proto["n_echoes"]):
        for e in range(ne):
            out.append(orc.spgr_derivs(np.asarray(y, dtype=np.float64), proto["flip"][c] * b1,
                                       proto["tr"][c], proto["te"][k0 + e], proto["mt"][c])[0])
        k0 += ne
    return np.array(out)


def _point(rng):
    return np.array([rng.uniform(6.2, 6.9), rng.uniform(-0.7, 0.4), rng.uniform(2.3, 3.7), rng.uniform(-5.3, -3.9)])


@pytest.mark.parametrize("seed", range(6))
def test_gradient_matches_fd_of_nll(orc, seed):
    rng = np.random.default_rng(seed)
    proto = _proto()
    y_true, y = _point(rng), _point(rng)
    b1 = rng.uniform(0.8, 1.2)
    x = _signals(orc, proto, y_true, b1) + rng.normal(0, 3.0, 10)
    _, g, _ = orc.lik_voxel(proto, x, y, b1)
    h = 1e-6
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        fd = (_nll(orc, proto, x, y + e, b1) - _nll(orc, proto, x, y - e, b1)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-6 * (abs(g).max() + 1.0))


@pytest.mark.parametrize("seed", range(6))
def test_loaded_hessian_from_fd_signal_derivatives(orc, seed):
    """P~ = sum_i [ds ds^T + |r| diag|d2s|] / sigma^2 with every derivative
    taken by finite differences of the signal (brute force)."""
    rng = np.random.default_rng(10 + seed)
    proto = _proto()
    y_true, y = _point(rng), _point(rng)
    x = _signals(orc, proto, y_true) + rng.normal(0, 3.0, 10)
    _, _, P = orc.lik_voxel(proto, x, y)
    s0 = _signals(orc, proto, y)
    J = np.zeros((10, 4))
    H = np.zeros((10, 4))
    for k in range(4):
        e = np.zeros(4)
        e[k] = 1e-5
        sp, sm = _signals(orc, proto, y + e), _signals(orc, proto, y - e)
        J[:, k] = (sp - sm) / 2e-5
        e[k] = 1e-3
        sp, sm = _signals(orc, proto, y + e), _signals(orc, proto, y - e)
        e[k] = 5e-4
        sp2, sm2 = _signals(orc, proto, y + e), _signals(orc, proto, y - e)
        H[:, k] = (4 * (sp2 - 2 * s0 + sm2) / 2.5e-7 - (sp - 2 * s0 + sm) / 1e-6) / 3
    wgt = 1.0 / np.array(proto["sigma"]) ** 2
    r = s0 - x
    ref = (J * wgt[:, None]).T @ J + np.diag((wgt[:, None] * np.abs(r)[:, None] * np.abs(H)).sum(0))
    assert np.allclose(P, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())
    # the loading term is diagonal and non-negative; P~ is SPD
    _, _, Pgn = orc.lik_voxel(proto, x, y, loading="gn")
    load = P - Pgn
    assert np.allclose(load - np.diag(np.diag(load)), 0.0)
    assert (np.diag(load) >= 0).all()
    assert np.linalg.eigvalsh(P).min() > 0


def test_zero_residual_hessian_is_exact(orc):
    """At x = s(y) every residual vanishes, so P~ is the true NLL Hessian."""
    rng = np.random.default_rng(7)
    proto = _proto()
    y = _point(rng)
    x = _signals(orc, proto, y)
    _, _, P = orc.lik_voxel(proto, x, y)
    h = 1e-4
    Hfd = np.zeros((4, 4))
    for k in range(4):
        for j in range(4):
            ek = np.zeros(4)
            ej = np.zeros(4)
            ek[k] = h
            ej[j] = h
            Hfd[k, j] = (_nll(orc, proto, x, y + ek + ej) - _nll(orc, proto, x, y + ek - ej)
                         - _nll(orc, proto, x, y - ek + ej) + _nll(orc, proto, x, y - ek - ej)) / (4 * h * h)
    assert np.allclose(P, Hfd, rtol=1e-5, atol=1e-5 * np.abs(P).max())


def test_solve4_matches_dense_solve(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        A = rng.normal(size=(4, 4))
        P = A @ A.T + 0.5 * np.eye(4)
        g = rng.normal(size=4)
        out, st = orc.solve4(P, g)
        assert st == 0
        assert np.allclose(out, np.linalg.solve(P, g), rtol=1e-12, atol=1e-12)


def test_solve4_frozen_and_degenerate(orc):
    P = np.diag([4.0, 2.0, 1.0, 1e-40])
    P[0, 3] = P[3, 0] = 1e-21
    g = np.array([4.0, 2.0, 3.0, 5.0])
    out, st = orc.solve4(P, g)
    assert st == 0
    assert np.allclose(out, [1.0, 1.0, 3.0, 0.0])  # parameter 3 is frozen
    # rank-one matrix: the scaled pivot collapses -> degenerate, step 0
    v = np.array([1.0, 2.0, 3.0, 4.0])
    out, st = orc.solve4(np.outer(v, v), g)
    assert st == 1 and not out.any()
    out, st = orc.solve4(np.full((4, 4), math.nan), g)
    assert st == 1 and not out.any()
