"""Resuming a MAP fit (option start_outer): the IRLS state between outer loops
is the maps and the loop index (Sec. 2.5-2.7: each loop re-weights from the
current maps, then takes its Newton steps), so a fit of T loops equals a fit
stopped after t loops followed by a fit that starts from its maps at loop t.

* the resumed fit reproduces the uninterrupted one exactly (maps, objective,
  the trace from loop t on, the step and CG counts of the remaining loops),
  also with gain-based early stopping inside the loops and with projection;
* restarting from the same maps at loop 0 instead (zero weights in its first
  loop, an ML warm start) does not, so the pin sees the re-weighting.
"""
import numpy as np
import pytest

from conftest import observations
from paper_2102_01604_amd import synth


def _case(dims=(12, 10, 8), seed=21):
    c = synth.make_case("map_brain", dims=dims, seed=seed)
    x = observations(__import__("oracle"), c).astype(np.float64)
    return c, x


def _resume(fit, T, t0, opts, y0):
    full, rf, tf = fit(dict(opts, n_outer=T), y0)
    part, rp, _ = fit(dict(opts, n_outer=t0), y0)
    res, rr, tr = fit(dict(opts, n_outer=T, start_outer=t0, init="maps"), part)
    return (full, rf, tf), (part, rp), (res, rr, tr)


def _check(T, t0, S, full, part, res):
    (yf, rf, tf), (_, rp), (yr, rr, tr) = full, part, res
    assert np.array_equal(yr, yf)
    assert np.all(np.isnan(tr[:t0 * S]))
    assert np.array_equal(tr[t0 * S:], tf[t0 * S:], equal_nan=True)
    assert rr["outer_done"] == T - t0
    assert rr["gn_done"] == rf["gn_done"] - rp["gn_done"]
    assert rr["cg_done"] == rf["cg_done"] - rp["cg_done"]
    assert rr["objective"] == rf["objective"] and rr["jtv"] == rf["jtv"]


@pytest.mark.parametrize("t0", [1, 3, 5])
def test_resumed_map_fit_equals_the_uninterrupted_fit(orc, t0):
    c, x = _case()
    opts = dict(c["opts"], n_gn=3, n_cg=12, lam=list(np.array(c["lam"]) * 20))
    y0 = orc.fit(c["proto"], c["dims"], x, c["b1"], {"mode": "ml", "n_gn": 0})[0]
    fit = lambda o, m: orc.fit(c["proto"], c["dims"], x, c["b1"], dict(o, init="maps"), maps0=m)
    T = 6
    full, part, res = _resume(fit, T, t0, opts, y0)
    _check(T, t0, opts["n_gn"] + 2, full, part, res)
    # restarting at loop 0 from the same maps is a different fit
    again, _, _ = fit(dict(opts, n_outer=T - t0), part[0])
    assert np.abs(again - full[0]).max() > 1e-6


def test_resume_with_early_stopping_inside_loops(orc):
    c, x = _case(seed=22)
    opts = dict(c["opts"], n_gn=6, n_cg=12, lam=list(np.array(c["lam"]) * 20), tol_gn=0.2)
    y0 = orc.fit(c["proto"], c["dims"], x, c["b1"], {"mode": "ml", "n_gn": 0})[0]
    fit = lambda o, m: orc.fit(c["proto"], c["dims"], x, c["b1"], dict(o, init="maps"), maps0=m)
    full, part, res = _resume(fit, 5, 2, opts, y0)
    assert full[1]["gn_done"] < 5 * 6  # the tolerance cut steps
    _check(5, 2, opts["n_gn"] + 2, full, part, res)


def test_resumed_projected_fit(orc):
    from test_oracle_proj import _moved_problem
    c, spaces, xs = _moved_problem(orc, dims=(8, 7, 5), seed=58)
    y0c = orc.default_init_projected(c["proto"], c["dims"], spaces, xs, c["b1"])
    y0 = np.repeat(np.asarray(y0c)[:, None], int(np.prod(c["dims"])), 1)
    opts = {"mode": "map", "n_gn": 3, "n_cg": 10, "lam": list(np.array(c["lam"]) * 20), "max_halvings": 4}
    fit = lambda o, m: orc.fit_projected(c["proto"], c["dims"], spaces, xs, c["b1"], dict(o, init="maps"),
                                         maps0=m)
    full, part, res = _resume(fit, 4, 2, opts, y0)
    _check(4, 2, opts["n_gn"] + 2, full, part, res)
