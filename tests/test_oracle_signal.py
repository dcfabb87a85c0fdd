"""Pins for the oracle's forward model (Sec. 2.1 eqs. 1-3, Sec. 2.4 eq.
spgr_signal and its printed derivatives).

The signal is pinned to a brute-force simulation of the spoiled steady state
(a longitudinal magnetisation recursion iterated to convergence), to the Ernst
angle and to the long-TR limit; the printed first and diagonal second
derivatives are pinned to finite differences of the signal itself.
"""
import math

import numpy as np
import pytest

from conftest import sigmoid


def bloch_steady_state(a, r1, r2, delta, alpha, tr, te, n_rep=20000):
    """Longitudinal magnetisation before each excitation, iterated over TRs.

    Each TR: an MT saturation pulse of angle alpha2 (cos alpha2 = 1 - delta)
    immediately before the excitation (TR2 = 0), excitation by alpha (perfect
    spoiling keeps only mz * cos alpha), then T1 recovery over TR towards a.
    The measured transverse signal is sin(alpha) * mz_after_MT, decayed by
    exp(-r2 * te)."""
    mz = a
    e1 = math.exp(-r1 * tr)
    cos2 = 1.0 - delta
    for _ in range(n_rep):
        mz_sat = mz * cos2
        mz = mz_sat * math.cos(alpha) * e1 + a * (1.0 - e1)
    mz_sat = mz * cos2
    return math.sin(alpha) * mz_sat * math.exp(-r2 * te)


@pytest.mark.parametrize("seed", range(6))
def test_signal_matches_bloch_recursion(orc, seed):
    rng = np.random.default_rng(seed)
    for mt in (0, 1):
        y = np.array([rng.uniform(5, 7), rng.uniform(-1, 0.5), rng.uniform(2, 4), rng.uniform(-5, -3)])
        a, r1, r2, dl = math.exp(y[0]), math.exp(y[1]), math.exp(y[2]), sigmoid(y[3])
        alpha, tr, te = rng.uniform(0.05, 0.6), rng.uniform(0.01, 0.05), rng.uniform(0.0, 0.02)
        s, _, _ = orc.spgr_derivs(y, alpha, tr, te, mt)
        ref = bloch_steady_state(a, r1, r2, dl if mt else 0.0, alpha, tr, te)
        assert s == pytest.approx(ref, rel=1e-11)


def test_ernst_angle_maximises_signal(orc):
    # delta = 0, TE = 0: dS/dalpha = 0 at cos(alpha_E) = exp(-R1 TR)
    y = np.array([math.log(800.0), math.log(1.1), math.log(20.0), 0.0])
    tr = 0.025
    alpha_e = math.acos(math.exp(-1.1 * tr))
    h = 1e-5
    sp, _, _ = orc.spgr_derivs(y, alpha_e + h, tr, 0.0, 0)
    sm, _, _ = orc.spgr_derivs(y, alpha_e - h, tr, 0.0, 0)
    s0, _, _ = orc.spgr_derivs(y, alpha_e, tr, 0.0, 0)
    assert abs(sp - sm) / (2 * h) < 1e-6 * s0
    for da in (-0.02, 0.02):
        s1, _, _ = orc.spgr_derivs(y, alpha_e + da, tr, 0.0, 0)
        assert s1 < s0


def test_long_tr_limit(orc):
    # TR -> infinity: full recovery, S = A sin(alpha) (1 - delta) exp(-R2* TE)
    y = np.array([math.log(700.0), math.log(0.9), math.log(30.0), -4.0])
    for mt in (0, 1):
        dl = sigmoid(y[3]) if mt else 0.0
        s, _, _ = orc.spgr_derivs(y, 0.3, 1e3, 0.01, mt)
        ref = 700.0 * math.sin(0.3) * (1 - dl) * math.exp(-30.0 * 0.01)
        assert s == pytest.approx(ref, rel=1e-13)


def _signal(orc, y, alpha, tr, te, mt):
    return orc.spgr_derivs(np.asarray(y, dtype=np.float64), alpha, tr, te, mt)[0]


@pytest.mark.parametrize("seed", range(8))
def test_derivatives_match_finite_differences(orc, seed):
    rng = np.random.default_rng(100 + seed)
    for mt in (0, 1):
        y = np.array([rng.uniform(5, 7), rng.uniform(-1, 0.5), rng.uniform(2, 4), rng.uniform(-5, -2)])
        alpha, tr, te = rng.uniform(0.05, 0.6), rng.uniform(0.01, 0.05), rng.uniform(0.001, 0.02)
        s, ds, d2s = orc.spgr_derivs(y, alpha, tr, te, mt)
        for k in range(4):
            e = np.zeros(4)
            h = 1e-6
            e[k] = h
            fd1 = (_signal(orc, y + e, alpha, tr, te, mt) - _signal(orc, y - e, alpha, tr, te, mt)) / (2 * h)

            def second(hh):
                e2 = np.zeros(4)
                e2[k] = hh
                return (_signal(orc, y + e2, alpha, tr, te, mt) - 2 * s
                        + _signal(orc, y - e2, alpha, tr, te, mt)) / (hh * hh)
            # Richardson extrapolation removes the O(h^2) truncation term
            fd2 = (4 * second(5e-4) - second(1e-3)) / 3
            scale = abs(s)
            assert abs(ds[k] - fd1) <= 1e-7 * scale
            assert abs(d2s[k] - fd2) <= 1e-6 * scale
        if not mt:
            assert ds[3] == 0.0 and d2s[3] == 0.0
