"""Pins for the rate and time representations (Sec. 3.1, the representation
comparison: the Newton-like steps act on (A, R1, R2*, MTsat) or on
(A, T1, T2*, MTsat) instead of the log/logit parameters, with the |H| 1
loading).

* the signal in either basis equals the log-parameter model at the same
  physical point, and its gradient and second derivatives follow from the
  (separately pinned) log-basis ones by the chain rule;
* both derivative sets match Richardson central differences, also at points
  outside the physical domain (the formula is evaluated as it is);
* the likelihood block's gradient and Gauss-Newton matrix transform by the
  same Jacobian;
* with the row-sum loading the loaded Hessian majorises the exact Hessian of
  the NLL (central differences of the oracle gradient) in both bases;
* noise-free echoes are recovered exactly;
* a step that would leave the domain moves halfway to its boundary (R-basis);
* on the experiment's random problems the log basis converges faster and the
  three bases reach the same optimum (Sec. 3.1, discussion of the figure).
"""
import numpy as np
import pytest

from paper_2102_01604_amd import synth

from test_oracle_voxelwise import _shape, _simulate_voxelwise


def _to_basis(y, basis):
    a, r1, r2, d = np.exp(y[0]), np.exp(y[1]), np.exp(y[2]), 1.0 / (1.0 + np.exp(-y[3]))
    if basis == "rate":
        return np.array([a, r1, r2, d])
    return np.array([a, 1.0 / r1, 1.0 / r2, d])


def _jac(th, basis):
    """d theta_k / d y_k and d2 theta_k / d y_k^2 (theta as a function of the
    log/logit parameter y_k)."""
    a, u1, u2, d = th
    if basis == "rate":
        return np.array([a, u1, u2, d * (1 - d)]), np.array([a, u1, u2, d * (1 - d) * (1 - 2 * d)])
    return np.array([a, -u1, -u2, d * (1 - d)]), np.array([a, u1, u2, d * (1 - d) * (1 - 2 * d)])


def _points(rng, n):
    for _ in range(n):
        y = np.array([rng.uniform(-2, 5), rng.uniform(-3, 2), rng.uniform(0, 5), rng.uniform(-5, 2)])
        yield y, rng.uniform(0.02, 1.2), np.exp(rng.uniform(-6, -1)), np.exp(rng.uniform(-6, -1)), int(rng.integers(2))


@pytest.mark.parametrize("basis", ["rate", "time"])
def test_basis_model_and_chain_rule(orc, basis):
    rng = np.random.default_rng(11)
    for y, al, tr, te, mt in _points(rng, 200):
        s, ds, d2s = orc.spgr_derivs(y, al, tr, te, mt)
        Hy = orc.spgr_hess(y, al, tr, te, mt)
        th = _to_basis(y, basis)
        sb, dsb, Hb = orc.spgr_basis(th, basis, al, tr, te, mt)
        assert abs(sb - s) <= 1e-13 * abs(s)
        J, J2 = _jac(th, basis)
        scale = np.abs(ds).max()
        assert np.abs(J * dsb - ds).max() <= 1e-12 * scale
        # d2s/dy_j dy_k = J_j J_k d2s/dth_j dth_k + [j = k] J2_k ds/dth_k
        Hc = J[:, None] * J[None, :] * Hb + np.diag(J2 * dsb)
        assert np.abs(Hc - Hy).max() <= 1e-11 * np.abs(Hy).max()
        assert np.array_equal(Hb, Hb.T)
        if not mt:
            assert dsb[3] == 0.0 and np.all(Hb[3] == 0.0)


def _richardson(f, x, k, h):
    def cd(hh):
        e = np.zeros_like(x)
        e[k] = hh
        return (f(x + e) - f(x - e)) / (2 * hh)
    return (4 * cd(h / 2) - cd(h)) / 3


@pytest.mark.parametrize("basis", ["rate", "time"])
def test_basis_derivatives_by_finite_differences(orc, basis):
    """Points inside and outside the physical domain (negative A, MTsat
    outside (0, 1), R1 TR slightly negative)."""
    rng = np.random.default_rng(12)
    for t in range(120):
        al, tr, te, mt = rng.uniform(0.05, 1.2), rng.uniform(0.005, 0.05), rng.uniform(0.0, 0.05), 1
        if t % 2:
            th = np.array([rng.uniform(-3, 3), rng.uniform(-2, 40), rng.uniform(-10, 60), rng.uniform(-0.3, 1.3)])
        else:
            th = _to_basis(np.array([rng.uniform(-1, 4), rng.uniform(-2, 2), rng.uniform(1, 4), rng.uniform(-4, 1)]),
                           basis)
        if basis == "time" and t % 2:
            th[1], th[2] = 1.0 / th[1], 1.0 / th[2]  # T = 1/R, both signs
        _, ds, H = orc.spgr_basis(th, basis, al, tr, te, mt)
        val = lambda v: orc.spgr_basis(v, basis, al, tr, te, mt)[0]  # noqa: E731
        grad = lambda v: orc.spgr_basis(v, basis, al, tr, te, mt)[1]  # noqa: E731
        for k in range(4):
            h = 1e-3 * max(abs(th[k]), 1e-2)
            fd = _richardson(val, th, k, h)
            assert abs(fd - ds[k]) <= 1e-7 * np.abs(ds).max() + 1e-12, (basis, t, k, fd, ds[k])
            fdh = _richardson(grad, th, k, h)
            assert np.abs(fdh - H[:, k]).max() <= 1e-6 * np.abs(H).max() + 1e-12, (basis, t, k)


@pytest.mark.parametrize("basis", ["rate", "time"])
def test_likelihood_block_transforms_with_the_jacobian(orc, basis):
    rng = np.random.default_rng(13)
    proto = synth.protocol()
    proto["sigma"] = [3.0] * 22
    truth = synth.maps_iid((1, 1, 20), rng)
    x = orc.simulate(proto, truth) + 3.0 * rng.normal(size=(22, 20))
    for n in range(20):
        y = truth[:, n] + rng.uniform(-0.3, 0.3, 4)
        th = _to_basis(y, basis)
        J, _ = _jac(th, basis)
        l0, g0, P0 = orc.lik_voxel_basis(proto, x[:, n], y, "log", "gn")
        l1, g1, P1 = orc.lik_voxel_basis(proto, x[:, n], th, basis, "gn")
        assert abs(l1 - l0) <= 1e-12 * l0
        assert np.abs(J * g1 - g0).max() <= 1e-11 * np.abs(g0).max()
        assert np.abs(J[:, None] * P1 * J[None, :] - P0).max() <= 1e-11 * np.abs(P0).max()


@pytest.mark.parametrize("basis", ["rate", "time"])
def test_row_sum_loading_majorises_the_nll_hessian(orc, basis):
    """Far from the optimum (start perturbed by up to 1.5 in each log
    parameter), P~ - H is positive semi-definite for the |H| 1 loading; the
    diagonal loading fails that test at some points."""
    rng = np.random.default_rng(14)
    proto = synth.protocol()
    proto["sigma"] = [4.0] * 22
    M = 150
    truth = synth.maps_iid((1, 1, M), rng)
    x = orc.simulate(proto, truth) + 4.0 * rng.normal(size=(22, M))
    fail_diag = 0
    for n in range(M):
        th = _to_basis(truth[:, n] + rng.uniform(-1.5, 1.5, 4), basis)
        grad = lambda v: orc.lik_voxel_basis(proto, x[:, n], v, basis, "gn")[1]  # noqa: E731
        Hx = np.empty((4, 4))
        for k in range(4):
            Hx[:, k] = _richardson(grad, th, k, 1e-4 * abs(th[k]))
        Hx = 0.5 * (Hx + Hx.T)
        _, _, Pp = orc.lik_voxel_basis(proto, x[:, n], th, basis, "plus")
        _, _, Pd = orc.lik_voxel_basis(proto, x[:, n], th, basis, "proposed")
        D = 1.0 / np.sqrt(np.diag(Pp))
        assert np.linalg.eigvalsh(D[:, None] * (Pp - Hx) * D[None, :]).min() >= -1e-6, (basis, n)
        Dd = 1.0 / np.sqrt(np.diag(Pd))
        fail_diag += np.linalg.eigvalsh(Dd[:, None] * (Pd - Hx) * Dd[None, :]).min() < -1e-6
    print(basis, "diagonal loading not a majoriser at", fail_diag, "of", M)
    assert fail_diag > 0


@pytest.mark.parametrize("basis", ["rate", "time"])
def test_noise_free_recovery(orc, basis):
    rng = np.random.default_rng(15)
    N = 200
    proto = synth.protocol()
    proto["sigma"] = [1.0] * 22
    truth = synth.maps_iid((1, 1, N), rng)
    x = orc.simulate(proto, truth)
    shape = {"n_echoes": proto["n_echoes"], "mt": proto["mt"], "sigma": proto["sigma"]}
    tr = np.repeat(np.asarray(proto["tr"])[:, None], N, axis=1)
    flip = np.repeat(np.asarray(proto["flip"])[:, None], N, axis=1)
    te = np.repeat(np.asarray(proto["te"])[:, None], N, axis=1)
    th_true = np.stack([_to_basis(truth[:, n], basis) for n in range(N)], axis=1)
    th0 = np.stack([_to_basis(truth[:, n] + rng.uniform(-0.3, 0.3, 4), basis) for n in range(N)], axis=1)
    # the row-sum loading is far more conservative in these bases: it needs
    # many more steps (the slower convergence Sec. 3.1 reports)
    for loading, steps in (("proposed", 200), ("gn", 200), ("plus", 20000)):
        m, _, nll, rep = orc.fit_voxelwise(shape, tr, flip, te, x, {"n_gn": steps, "loading": loading,
                                                                     "basis": basis}, maps0=th0)
        rel = np.abs(m - th_true) / np.abs(th_true)
        print(basis, loading, steps, "max rel error", rel.max(axis=1))
        assert rel.max() <= 1e-8
        assert rep["nonfinite_voxels"] == 0


@pytest.mark.parametrize("basis", ["rate", "time"])
def test_step_that_leaves_the_domain_goes_halfway(orc, basis):
    """One step from a start far from the optimum: each parameter moves by the
    solved step unless that would leave its domain, in which case it moves
    halfway to the boundary (reading R-basis)."""
    rng = np.random.default_rng(16)
    N = 400
    y, tr, flip, te = synth.e1_problems(N, rng)
    with np.errstate(all="ignore"):
        x = _simulate_voxelwise(orc, (5, 5, 5), (0, 0, 1), tr, flip, te, y) + rng.normal(size=(15, N))
    shape = _shape((5, 5, 5), (0, 0, 1), 1.0)
    th0 = np.stack([_to_basis(rng.uniform(-3, 3, 4), basis) for _ in range(N)], axis=1)
    m, _, _, _ = orc.fit_voxelwise(shape, tr, flip, te, x, {"n_gn": 1, "loading": "plus", "basis": basis},
                                   maps0=th0)
    crossed = 0
    for n in range(N):
        p = {"n_echoes": [5, 5, 5], "tr": list(tr[:, n]), "flip": list(flip[:, n]), "mt": [0, 0, 1],
             "te": list(te[:, n]), "sigma": [1.0] * 15}
        _, g, P = orc.lik_voxel_basis(p, x[:, n], th0[:, n], basis, "plus")
        step, degenerate = orc.solve4(P, g)
        for k in range(4):
            u, v = th0[k, n], th0[k, n] - step[k]
            if v <= 0:
                want, crossed = 0.5 * u, crossed + 1
            elif k == 3 and v >= 1:
                want, crossed = 0.5 * (1 + u), crossed + 1
            else:
                want = v
            assert m[k, n] == want, (n, k)
    print(basis, "parameters that would have left the domain:", crossed, "of", 4 * N)
    assert crossed > 0


def test_log_basis_converges_faster_to_the_same_optimum(orc):
    """Sec. 3.1 representation comparison on the experiment's random problems
    (three contrasts x five echoes, sigma = 1, 10,000 steps, |H| 1 loading,
    every basis started from the point log-parameters 0 give)."""
    rng = np.random.default_rng(2103)
    N = 300
    y, tr, flip, te = synth.e1_problems(N, rng)
    with np.errstate(all="ignore"):
        x = _simulate_voxelwise(orc, (5, 5, 5), (0, 0, 1), tr, flip, te, y) + rng.normal(size=(15, N))
    shape = _shape((5, 5, 5), (0, 0, 1), 1.0)
    checkpoints = [100, 1000, 10000]
    nll = {}
    final = {}
    for basis in ("log", "rate", "time"):
        start = [0.0] * 4 if basis == "log" else [1.0, 1.0, 1.0, 0.5]
        m, done, rows = None, 0, []
        for it in checkpoints:
            opts = {"n_gn": it - done, "loading": "plus", "basis": basis, "init": "const", "init_const": start}
            with np.errstate(all="ignore"):
                m, _, v, rep = orc.fit_voxelwise(shape, tr, flip, te, x, opts, maps0=m)
            done = it
            rows.append(v)
        nll[basis] = np.array(rows)
        final[basis] = m
        assert rep["nonfinite_voxels"] == 0
    best = np.min([nll[b][-1] for b in nll], axis=0)
    excess = {b: (nll[b] - best) / np.abs(best) for b in nll}
    for b in excess:
        print(b, "median relative NLL excess at", checkpoints, np.median(excess[b], axis=1),
              "| within 1e-6 of the best at the end:", np.mean(excess[b][-1] <= 1e-6))
    for b in ("rate", "time"):
        assert np.all(np.median(excess["log"], axis=1) < np.median(excess[b], axis=1))
        th = final[b]
        assert np.all(th[:3] >= 0.0) and np.all((th[3] >= 0.0) & (th[3] <= 1.0))  # the domain is kept
    # the log basis reaches the best optimum found by any basis in almost every voxel
    assert np.mean(excess["log"][-1] <= 1e-6) >= 0.9
