"""Pins for the paper's 1-D toy problems (Sec. 2.3) and the protocol fixture.

The toy problems are where the proposed loading (|residual| * |second
derivative| added to the Gauss-Newton curvature) is motivated.  Their printed
formulas are checked against finite differences, which exposes two typos the
implementation reads past:
  * toy 2: the true Hessian carries the residual (exp(-exp(y)) - x), not
    (exp(y) - x);
  * toy 1: r = g/p has derivative +x*exp(y), and the objective is non-convex
    for y > y* + ln 2 (on the side of large y).
The proposed step is then monotone from the non-convex side where
Gauss-Newton overshoots.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2102_01604_amd import synth

X = 0.5


def toy1(y):
    e = math.exp(-y)
    return 0.5 * (e - X) ** 2, -(e - X) * e, e * e + (e - X) * e, e * e, e * e + abs(e - X) * e


def toy2(y):
    ee = math.exp(-math.exp(y))
    j = math.exp(y - math.exp(y))
    res = ee - X
    g = -j * res
    h_true = j * j + (math.exp(2 * y) - math.exp(y)) * ee * res
    h_printed = j * j + (math.exp(2 * y) - math.exp(y)) * ee * (math.exp(y) - X)
    p = j * j
    pt = j * j + abs((math.exp(2 * y) - math.exp(y)) * ee * res)
    return 0.5 * (X - ee) ** 2, g, h_true, p, pt, h_printed


@pytest.mark.parametrize("y", [-1.5, -0.3, 0.2, 1.1, 2.5])
def test_toy_formulas_match_fd(y):
    h = 1e-6
    f1 = lambda v: toy1(v)[0]
    f2 = lambda v: toy2(v)[0]
    _, g1, h1, _, _ = toy1(y)
    assert g1 == pytest.approx((f1(y + h) - f1(y - h)) / (2 * h), rel=1e-6, abs=1e-10)
    assert h1 == pytest.approx((toy1(y + h)[1] - toy1(y - h)[1]) / (2 * h), rel=1e-6, abs=1e-10)
    _, g2, h2, _, _, h2p = toy2(y)
    assert g2 == pytest.approx((f2(y + h) - f2(y - h)) / (2 * h), rel=1e-6, abs=1e-10)
    fdh = (toy2(y + h)[1] - toy2(y - h)[1]) / (2 * h)
    assert h2 == pytest.approx(fdh, rel=1e-6, abs=1e-10)
    # the printed residual factor is wrong wherever exp(y) != exp(-exp(y))
    assert abs(h2p - fdh) > 1e-3 * abs(fdh) + 1e-9


def test_toy1_ratio_derivative_and_convexity():
    ystar = -math.log(X)
    for y in (-1.0, 0.0, 1.0, 2.0):
        r = lambda v: toy1(v)[1] / toy1(v)[3]
        h = 1e-6
        assert (r(y + h) - r(y - h)) / (2 * h) == pytest.approx(X * math.exp(y), rel=1e-6)
    # second derivative changes sign at y* + ln 2
    yc = ystar + math.log(2)
    assert toy1(yc - 0.01)[2] > 0 > toy1(yc + 0.01)[2]


@pytest.mark.parametrize("toy,y0", [(toy1, 3.0), (toy2, -3.0), (toy2, 1.5)])
def test_proposed_monotone_where_gauss_newton_fails(toy, y0):
    def run(kind, n=60):
        y, vals = y0, []
        for _ in range(n):
            t = toy(y)
            f, g, p, pt = t[0], t[1], t[3], t[4]
            vals.append(f)
            curv = pt if kind == "proposed" else p
            if curv <= 0.0:
                vals.append(math.inf)
                break
            y = y - g / curv
            if not math.isfinite(y) or abs(y) > 50:
                vals.append(math.inf)
                break
        else:
            vals.append(toy(y)[0] if math.isfinite(y) and abs(y) <= 50 else math.inf)
        return np.array(vals)

    prop = run("proposed")
    gn = run("gn")
    assert np.all(np.diff(prop) <= 1e-15)
    assert prop[-1] < 1e-10
    assert np.any(np.diff(gn) > 0) or not np.all(np.isfinite(gn))


def test_default_protocol_is_the_papers():
    here = os.path.dirname(os.path.abspath(__file__))
    gold = json.load(open(os.path.join(here, "golden", "paper_protocol.json")))
    p = synth.protocol()
    assert p["n_echoes"] == gold["n_echoes"]
    assert np.allclose(np.degrees(p["flip"]), gold["flip_deg"])
    assert p["mt"] == gold["mt_pulse"]
    assert np.allclose(p["tr"], gold["tr_ms"] * 1e-3)
    te = np.array(p["te"])
    k0 = 0
    for ne in p["n_echoes"]:
        assert np.allclose(np.diff(te[k0:k0 + ne]), gold["echo_spacing_ms"] * 1e-3)
        k0 += ne
