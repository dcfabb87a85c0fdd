"""Pins for the oracle's early stopping of the MAP fit (Sec. 2.7: a tolerance
on the gain between successive iterations; reading R-stop: the gain of a
step is the decrease it brings over the decrease since the first value of its
sequence -- F_w before the first Newton step of an outer loop, or the
objective at the end of the first outer loop).

* zero tolerances give the fixed-count fit;
* with a Newton tolerance, each outer loop stops after the first step whose
  gain, recomputed from the recorded objective values, is below it; the
  steps taken before are those of the fixed-count fit;
* with an outer tolerance, the loops stop after the first whose gain is below
  it, likewise.
"""
import numpy as np

from conftest import observations
from paper_2102_01604_amd import synth


def _problem(orc, seed=81):
    c = synth.make_case("map_brain", dims=(24, 20, 12), seed=seed)
    x = observations(orc, c).astype(np.float64)
    y0 = orc.default_init(c["proto"], x, c["b1"])
    return c, x, dict(c["opts"], init="const", init_const=[float(v) for v in y0])


def test_zero_tolerances_are_the_fixed_count_fit(orc):
    c, x, opts = _problem(orc)
    opts = dict(opts, n_outer=3, n_gn=4, n_cg=12)
    m0, r0, t0 = orc.fit(c["proto"], c["dims"], x, c["b1"], opts)
    m1, r1, t1 = orc.fit(c["proto"], c["dims"], x, c["b1"], dict(opts, tol_gn=0.0, tol_outer=0.0))
    assert np.array_equal(m0, m1) and np.array_equal(t0, t1, equal_nan=True) and r0 == r1


def _gains(f):
    """Gain of each step of the sequence f[0], f[1], ...: (f[j] - f[j+1]) / (f[0] - f[j+1])."""
    out = []
    for j in range(len(f) - 1):
        den = f[0] - f[j + 1]
        out.append((f[j] - f[j + 1]) / den if den > 0 else -np.inf)
    return np.array(out)


def test_newton_tolerance(orc):
    c, x, opts = _problem(orc)
    opts = dict(opts, n_outer=3, n_gn=8, n_cg=16)
    tol = 0.05
    _, rf, tf = orc.fit(c["proto"], c["dims"], x, c["b1"], opts)
    _, rs, ts = orc.fit(c["proto"], c["dims"], x, c["b1"], dict(opts, tol_gn=tol))
    S = opts["n_gn"] + 2
    stopped_early = 0
    taken = 0
    for t in range(opts["n_outer"]):
        seg = ts[t * S:t * S + opts["n_gn"] + 1]
        k = int(np.isfinite(seg).sum()) - 1  # steps taken in this loop
        assert np.all(np.isfinite(seg[:k + 1])) and np.all(np.isnan(seg[k + 1:]))
        g = _gains(seg[:k + 1])
        assert np.all(g[:-1] >= tol)  # every step before the last kept going
        if k < opts["n_gn"]:
            assert g[-1] < tol  # and the last one stopped the loop
            stopped_early += 1
        taken += k
        if t == 0:  # the same trajectory as the fixed-count fit up to the stop
            assert np.array_equal(seg[:k + 1], tf[:k + 1])
    assert stopped_early >= 1 and rs["gn_done"] == taken < rf["gn_done"]


def test_outer_tolerance(orc):
    c, x, opts = _problem(orc, seed=82)
    opts = dict(opts, n_outer=8, n_gn=2, n_cg=12)
    tol = 0.05
    _, rf, tf = orc.fit(c["proto"], c["dims"], x, c["b1"], opts)
    _, rs, ts = orc.fit(c["proto"], c["dims"], x, c["b1"], dict(opts, tol_outer=tol))
    S = opts["n_gn"] + 2
    objf = tf[S - 1::S]  # objective at the end of each loop, fixed count
    objs = ts[S - 1::S]
    T = rs["outer_done"]
    assert 1 <= T < opts["n_outer"]
    assert np.array_equal(objs[:T], objf[:T]) and np.all(np.isnan(objs[T:]))
    g = _gains(objf[:T])
    assert np.all(g[:-1] >= tol) and g[-1] < tol
