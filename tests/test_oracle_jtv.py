"""Pins for the oracle's JTV prior, IRLS algebra and PCG (Sec. 2.5-2.6).

The stencil operators are checked against an explicit sparse finite-difference
matrix G (6N x N, forward and backward differences, zero across the border)
built here from the definition; the IRLS identity is checked by finite
differences of the smoothed JTV; PCG is checked against a dense solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

DIMS = (5, 4, 3)


def explicit_G(dims):
    nx, ny, nz = dims
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    r = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                n = x + nx * (y + ny * z)
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                        m = xx + nx * (yy + ny * zz)
                        rows += [r, r]
                        cols += [m, n]
                        vals += [1.0, -1.0]
                    r += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(6 * N, N))


def test_weights_and_stencil_match_explicit_operator(orc):
    rng = np.random.default_rng(0)
    N = int(np.prod(DIMS))
    G = explicit_G(DIMS)
    Y = rng.normal(size=(4, N))
    lam = np.array([0.3, 1.7, 0.5, 2.2])
    eps = 0.05
    w, d, jtv = orc.jtv_weights(DIMS, Y, lam, eps)
    # q_n = sum_k lambda_k ||G_n y_k||^2 with the 6 rows of voxel n
    q = sum(lam[k] * (np.asarray(G @ Y[k]) ** 2).reshape(N, 6).sum(1) for k in range(4))
    assert np.allclose(w, 1 / np.sqrt(q + eps ** 2), rtol=1e-13)
    assert jtv == pytest.approx(np.sqrt(q + eps ** 2).sum(), rel=1e-13)
    W = sp.diags(np.repeat(w, 6))
    GWG = (G.T @ W @ G).toarray()
    assert np.allclose(d, np.diag(GWG), rtol=1e-13)
    V = rng.normal(size=(4, N))
    LV = orc.apply_L(DIMS, w, lam, V)
    for k in range(4):
        assert np.allclose(LV[k], lam[k] * GWG @ V[k], rtol=1e-12, atol=1e-12)
    # L annihilates constants and is positive semi-definite
    assert np.abs(orc.apply_L(DIMS, w, lam, np.ones((4, N)))).max() < 1e-12
    assert (V * LV).sum() >= 0


def test_irls_gradient_identity(orc):
    """At w = (q + eps^2)^(-1/2), grad of sum_n sqrt(q_n + eps^2) equals L_w y
    (the bound eq. bound is tight and has zero slope in w there)."""
    rng = np.random.default_rng(1)
    N = int(np.prod(DIMS))
    Y = rng.normal(size=(4, N))
    lam = np.array([0.5, 1.0, 2.0, 0.25])
    eps = 0.1
    w, _, _ = orc.jtv_weights(DIMS, Y, lam, eps)
    grad = orc.apply_L(DIMS, w, lam, Y)
    h = 1e-6
    for k, n in [(0, 0), (1, 7), (2, 31), (3, N - 1), (1, 22)]:
        Yp, Ym = Y.copy(), Y.copy()
        Yp[k, n] += h
        Ym[k, n] -= h
        fd = (orc.jtv_weights(DIMS, Yp, lam, eps)[2] - orc.jtv_weights(DIMS, Ym, lam, eps)[2]) / (2 * h)
        assert grad[k, n] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_pcg_matches_dense_solve(orc):
    dims = (4, 3, 2)
    N = int(np.prod(dims))
    rng = np.random.default_rng(2)
    P = np.empty((N, 4, 4))
    for n in range(N):
        A = rng.normal(size=(4, 4))
        P[n] = A @ A.T + 0.2 * np.eye(4)
    w = rng.uniform(0.1, 2.0, N)
    lam = np.array([0.5, 1.5, 0.7, 1.1])
    _, d, _ = orc.jtv_weights(dims, rng.normal(size=(4, N)), lam, 1.0)  # any d works as a preconditioner
    G = explicit_G(dims)
    GWG = (G.T @ sp.diags(np.repeat(w, 6)) @ G).toarray()
    d = np.diag(GWG).copy()
    # dense system in [4][N] ordering
    A = np.zeros((4 * N, 4 * N))
    for k in range(4):
        A[k * N:(k + 1) * N, k * N:(k + 1) * N] += lam[k] * GWG
        for j in range(4):
            A[k * N + np.arange(N), j * N + np.arange(N)] += P[:, k, j]
    b = rng.normal(size=(4, N))
    delta, it = orc.pcg(dims, P, w, d, lam, b, n_cg=400, cg_stop=1e-30)
    ref = np.linalg.solve(A, b.reshape(-1)).reshape(4, N)
    assert np.allclose(delta, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    assert it <= 400
