"""Pins for the oracle's spatial projection (Sec. 2.4, "Spatial projection";
reading R-proj: trilinear reslicing Psi with replicated borders, acquisition
voxels outside the reconstruction field of view carry no observation).

* pull and push are adjoint: <Psi u, v> = <u, Psi^T v>;
* trilinear pull reproduces affine functions exactly away from the border,
  constants everywhere in the field of view, and gives 0 outside it;
* with identity spaces the projected fit is the unprojected fit;
* the pushed gradient equals central differences of the projected NLL;
* with the Proposed+ loading the pushed blocks majorise the full (coupled)
  Hessian of the projected NLL, the block-diagonal majoriser Sec. 2.4 cites;
* a projected ML fit to noise-free echoes decreases the NLL monotonically.
"""
import numpy as np
import pytest

from conftest import f32
from paper_2102_01604_amd import synth


def _affine(rng, rot_deg=4.0, shift=1.0, scale=(1.0, 1.0, 1.0), centre=(0.0, 0.0, 0.0)):
    """A rigid motion (+ scaling) about `centre`, as acquisition index -> recon coordinate."""
    a, b, c = np.deg2rad(rng.uniform(-rot_deg, rot_deg, 3))
    Rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rz = np.array([[np.cos(c), -np.sin(c), 0], [np.sin(c), np.cos(c), 0], [0, 0, 1]])
    R = Rz @ Ry @ Rx @ np.diag(scale)
    t = np.asarray(centre) - R @ np.asarray(centre) + rng.uniform(-shift, shift, 3)
    return np.hstack([R, t[:, None]])


def _space(dims, A):
    return {"dims": tuple(int(v) for v in dims), "affine": np.asarray(A).reshape(3, 4)}


def test_pull_push_adjoint(orc):
    rng = np.random.default_rng(1)
    dims = (9, 7, 6)
    for _ in range(10):
        sp = _space((10, 6, 7), _affine(rng, 10.0, 2.0, scale=rng.uniform(0.8, 1.25, 3), centre=(4, 3, 3)))
        u = rng.normal(size=int(np.prod(dims)))
        v = rng.normal(size=int(np.prod(sp["dims"])))
        lhs, rhs = np.dot(orc.pull(dims, sp, u), v), np.dot(u, orc.push(dims, sp, v))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_pull_reproduces_affine_functions(orc):
    rng = np.random.default_rng(2)
    dims = (8, 9, 7)
    x, y, z = np.meshgrid(np.arange(dims[0]), np.arange(dims[1]), np.arange(dims[2]), indexing="ij")
    coef = rng.normal(size=4)
    u = (coef[0] + coef[1] * x + coef[2] * y + coef[3] * z).transpose(2, 1, 0).reshape(-1)  # x fastest
    for _ in range(5):
        A = _affine(rng, 6.0, 1.5, centre=(3.5, 4, 3))
        sp = _space((9, 8, 7), A)
        out = orc.pull(dims, sp, u)
        ones = orc.pull(dims, sp, np.ones(int(np.prod(dims))))
        ii, jj, kk = np.meshgrid(*[np.arange(n) for n in sp["dims"]], indexing="ij")
        idx = np.stack([ii, jj, kk, np.ones_like(ii)], -1).transpose(2, 1, 0, 3).reshape(-1, 4)
        r = idx @ A.T
        inside_fov = np.all((r >= -0.5) & (r <= np.asarray(dims) - 0.5), axis=1)
        interior = np.all((r >= 0) & (r <= np.asarray(dims) - 1), axis=1)
        assert interior.sum() > 100 and (~inside_fov).sum() > 0
        expect = coef[0] + r @ coef[1:]
        assert np.abs(out[interior] - expect[interior]).max() <= 1e-12 * np.abs(expect).max()
        assert np.allclose(ones[inside_fov], 1.0, atol=1e-14)
        assert np.all(out[~inside_fov] == 0.0) and np.all(ones[~inside_fov] == 0.0)


def _identity(dims):
    return _space(dims, np.hstack([np.eye(3), np.zeros((3, 1))]))


@pytest.mark.parametrize("mode", ["ml", "map"])
def test_identity_spaces_equal_the_unprojected_fit(orc, mode):
    c = synth.make_case("map_brain", dims=(12, 10, 6), seed=51)
    x = orc.simulate(c["proto"], c["truth"], c["b1"]) + c["sigma"] * c["eps"].astype(np.float64)
    opts = (dict(c["opts"], n_outer=3, n_gn=2, n_cg=8) if mode == "map" else {"mode": "ml", "n_gn": 8})
    spaces = [_identity(c["dims"])] * 3
    m0, r0, t0 = orc.fit(c["proto"], c["dims"], x, c["b1"], opts)
    m1, r1, t1 = orc.fit_projected(c["proto"], c["dims"], spaces, x.reshape(-1), c["b1"], opts)
    assert np.abs(m1 - m0).max() <= 1e-11 * np.abs(m0).max()
    assert np.allclose(t1, t0, rtol=1e-12, equal_nan=True)
    assert r1["gn_done"] == r0["gn_done"] and r1["nll"] == pytest.approx(r0["nll"], rel=1e-12)


@pytest.mark.parametrize("mode", ["ml", "map"])
def test_identity_spaces_equal_the_unprojected_uncertainty(orc, mode):
    """With every contrast acquired on the reconstruction grid the pushed
    blocks are the voxel blocks, so the projected Laplace variance is the plain
    one (itself pinned by sampling, test_oracle_map)."""
    c = synth.make_case("map_brain", dims=(12, 10, 6), seed=53)
    x = orc.simulate(c["proto"], c["truth"], c["b1"]) + c["sigma"] * c["eps"].astype(np.float64)
    opts = dict(c["opts"], mode=mode)
    maps = c["truth"] + 0.05
    v0 = orc.uncertainty(c["proto"], c["dims"], x, c["b1"], opts, maps)
    v1 = orc.uncertainty_projected(c["proto"], c["dims"], [_identity(c["dims"])] * 3, x.reshape(-1), c["b1"], opts,
                                   maps)
    assert np.all(np.isfinite(v0)) and np.all(v0 > 0)
    assert np.abs(v1 - v0).max() <= 1e-12 * np.abs(v0).max()


def _moved_problem(orc, dims=(10, 9, 6), seed=52, noise=True):
    """Three contrasts, each acquired on its own moved grid; echoes simulated
    by pulling the true maps (and b1) into each space."""
    rng = np.random.default_rng(seed)
    c = synth.make_case("map_brain", dims=dims, seed=seed)
    centre = (np.asarray(dims) - 1) / 2
    spaces = [_identity(dims)] + [_space((dims[0] + 1, dims[1], dims[2]), _affine(rng, 4.0, 0.8, centre=centre))
                                  for _ in range(2)]
    xs = []
    for ci, sp in enumerate(spaces):
        yp = np.stack([orc.pull(dims, sp, c["truth"][k]) for k in range(4)])
        bp = orc.pull(dims, sp, c["b1"])
        pc = dict(c["proto"])
        first = sum(c["proto"]["n_echoes"][:ci])
        ne = c["proto"]["n_echoes"][ci]
        pc.update(n_echoes=[ne], tr=[pc["tr"][ci]], flip=[pc["flip"][ci]], mt=[pc["mt"][ci]],
                  te=pc["te"][first:first + ne], sigma=pc["sigma"][first:first + ne])
        s = orc.simulate(pc, yp, np.where(bp > 0, bp, 1.0))
        if noise:
            s = s + c["sigma"] * rng.normal(size=s.shape)
        xs.append(s)
    return c, spaces, xs


def test_projected_gradient_matches_fd(orc):
    c, spaces, xs = _moved_problem(orc)
    N = int(np.prod(c["dims"]))
    rng = np.random.default_rng(3)
    y = c["truth"] + 0.05 * rng.normal(size=c["truth"].shape)
    _, g, _ = orc.proj_lik(c["proto"], c["dims"], spaces, xs, c["b1"], y)
    for n in rng.choice(N, 6, replace=False):
        for k in range(4):
            def f(h):
                yy = y.copy()
                yy[k, n] += h
                return orc.proj_lik(c["proto"], c["dims"], spaces, xs, c["b1"], yy)[0]
            fd = (8 * (f(1e-4) - f(-1e-4)) - (f(2e-4) - f(-2e-4))) / (12 * 1e-4)
            assert fd == pytest.approx(g[k, n], rel=1e-6, abs=1e-6 * np.abs(g).max())


def test_pushed_blocks_majorise_the_projected_hessian(orc):
    c, spaces, xs = _moved_problem(orc, dims=(4, 3, 3), seed=53)
    N = int(np.prod(c["dims"]))
    rng = np.random.default_rng(4)
    for _ in range(3):
        y = c["truth"] + 0.5 * rng.normal(size=c["truth"].shape)  # large residuals
        _, _, P = orc.proj_lik(c["proto"], c["dims"], spaces, xs, c["b1"], y, loading="plus")
        # exact Hessian of the projected NLL by central differences of its gradient, in [k][n] order
        H = np.zeros((4 * N, 4 * N))
        h = 1e-5
        for k in range(4):
            for n in range(N):
                yp, ym = y.copy(), y.copy()
                yp[k, n] += h
                ym[k, n] -= h
                gp = orc.proj_lik(c["proto"], c["dims"], spaces, xs, c["b1"], yp)[1]
                gm = orc.proj_lik(c["proto"], c["dims"], spaces, xs, c["b1"], ym)[1]
                H[:, k * N + n] = ((gp - gm) / (2 * h)).reshape(-1)
        H = 0.5 * (H + H.T)
        D = np.zeros_like(H)
        for n in range(N):
            for a in range(4):
                for b in range(4):
                    D[a * N + n, b * N + n] = P[n, a, b]
        scale = np.abs(D).max()
        assert np.linalg.eigvalsh(D - H).min() >= -1e-6 * scale
        assert np.abs(H - np.diag(np.diag(H))).max() > 1e-3 * scale  # the Hessian really is coupled
        # the unloaded (Gauss-Newton) blocks do not majorise it: the check can fail
        _, _, Pg = orc.proj_lik(c["proto"], c["dims"], spaces, xs, c["b1"], y, loading="gn")
        Dg = np.zeros_like(H)
        for n in range(N):
            for a in range(4):
                for b in range(4):
                    Dg[a * N + n, b * N + n] = Pg[n, a, b]
        assert np.linalg.eigvalsh(Dg - H).min() < -1e-3 * scale


def test_projected_ml_fit_noise_free(orc):
    c, spaces, xs = _moved_problem(orc, noise=False)
    y0 = orc.default_init_projected(c["proto"], c["dims"], spaces, xs, c["b1"])
    maps, rep, trace = orc.fit_projected(c["proto"], c["dims"], spaces, xs, c["b1"],
                                         {"mode": "ml", "n_gn": 40, "init": "const", "init_const": y0,
                                          "loading": "plus"})
    assert np.all(np.diff(trace) <= 1e-12 * trace[:-1])
    assert trace[-1] < 1e-3 * trace[0]
    assert rep["nonfinite_voxels"] == 0
