"""Pins of the oracle's extrapolation fits: exact recovery, closed forms and a
library cross-check (scipy)."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import curve_fit, minimize

from oracle import fits

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_poly_exact_and_lagrange():
    lam = np.array([1e-3, 2e-3, 4e-3, 8e-3])
    y = 0.7 - 30 * lam + 900 * lam ** 2
    v, coef = fits.fit_poly(lam, y, 2, 0.0)
    assert abs(v - 0.7) < 1e-12
    # three points: the quadratic fit is Lagrange interpolation
    x, yy = np.array([1.0, 2.0, 4.0]), np.array([0.3, -0.2, 0.9])
    t = 3.0
    lag = sum(yy[i] * np.prod([(t - x[j]) / (x[i] - x[j])
                               for j in range(3) if j != i]) for i in range(3))
    assert abs(fits.fit_poly(x, yy, 2, t)[0] - lag) < 1e-12


def test_exp3_exact_recovery_and_closed_form():
    lam = np.linspace(1e-3, 16e-3, 8)
    a, b, c = 0.6, 85.0, 0.05
    y = a * np.exp(-b * lam) + c
    v, coef = fits.fit_exp3(lam, y, 0.0)
    assert abs(v - (a + c)) < 1e-9
    assert np.max(np.abs(coef - [a, b, c])) < 1e-6
    # three equally spaced points: b = -ln((y3 - y2) / (y2 - y1)) / dlam
    l3 = np.array([0.1, 0.2, 0.3])
    y3 = np.array([0.9, 0.55, 0.4])
    b_cf = -np.log((y3[2] - y3[1]) / (y3[1] - y3[0])) / 0.1
    _, coef3 = fits.fit_exp3(l3, y3, 0.0)
    assert abs(coef3[1] - b_cf) < 1e-7


def test_exp3_vs_scipy_curve_fit():
    rng = np.random.default_rng(0)
    lam = np.linspace(1e-3, 16e-3, 8)
    y = 0.4 * np.exp(-60 * lam) - 0.02 + 1e-3 * rng.standard_normal(8)
    v, coef = fits.fit_exp3(lam, y, 1e-3)
    p, _ = curve_fit(lambda l, a, b, c: a * np.exp(-b * l) + c, lam, y,
                     p0=coef, maxfev=20000)
    rss = lambda q: np.sum((q[0] * np.exp(-q[1] * lam) + q[2] - y) ** 2)  # noqa
    assert rss(coef) <= rss(p) * (1 + 1e-9)
    assert abs(v - (p[0] * np.exp(-p[1] * 1e-3) + p[2])) < 1e-6


def test_loglin_exact_recovery():
    lam = np.array([0.0, 1e-3, 2e-3, 4e-3, 8e-3])
    fid = np.array([0.999, 0.3, 0.5, 0.8, 0.995])
    a, b = -0.35, 40.0
    y = a * np.exp(-b * lam)
    v, coef, used = fits.fit_loglin_weighted(lam, y, fid, 2e-3)
    assert used.all()
    assert abs(v - a * np.exp(-b * 2e-3)) < 1e-12
    assert np.max(np.abs(coef - [a, b])) < 1e-9


def test_loglin_criteria_and_weights_vs_direct_minimisation():
    lam = np.array([0.0, 1e-3, 2e-3, 3e-3, 5e-3, 8e-3, 12e-3])
    y = np.array([0.5, 0.47, 0.43, -0.01, 0.36, 5e-12, 0.21])
    fid = np.array([0.999, 0.4, 0.6, 0.7, 0.95, 0.992, 0.999])
    lt = 1e-3
    v, coef, used = fits.fit_loglin_weighted(lam, y, fid, lt)
    # criterion 3 drops the negative value, criterion 2 the 5e-12 one
    assert list(used) == [True, True, True, False, True, False, True]
    d = 8e-3                  # smallest lambda > 0 with F > 0.99 (App. B.2)
    assert fits.dip_size(lam, fid) == d
    w = fid ** 2 * np.exp(-20 * np.abs(lt - lam) / d)

    def loss(p):
        r = p[0] - p[1] * lam[used] - np.log(np.abs(y[used]))
        return np.sum(w[used] ** 2 * r ** 2)
    res = minimize(loss, x0=[np.log(0.5), 10.0], method="Nelder-Mead",
                   options={"xatol": 1e-13, "fatol": 1e-30, "maxiter": 40000})
    a_ref, b_ref = np.exp(res.x[0]), res.x[1]
    assert abs(coef[0] - a_ref) < 1e-6 * a_ref
    assert abs(coef[1] - b_ref) < 1e-4 * abs(b_ref) + 1e-6


def test_nzne_fallback_chain():
    lam = np.array([1e-3, 2e-3, 4e-3, 8e-3])
    fid = np.ones(4)
    # only one point with the reference sign -> direct exponential fit
    y = np.array([0.01, -0.02, -0.03, -0.035])
    v, method, coef, used = fits.nzne(lam, y, fid, 0.0)
    assert method == "exp3"
    # two points only, opposite signs -> nothing possible
    v, method, coef, used = fits.nzne(lam[:2], y[:2], fid[:2], 0.0)
    assert method == "none" and v is None


def test_fidelity_extrapolation_and_convergence():
    f = np.array([0.5, 0.7, 0.9])
    o = 0.2 + 0.1 * (1 - f)
    assert abs(fits.fidelity_extrapolation(o, f) - 0.2) < 1e-14
    # App. B.1: slope 0.1, (1 - F_k) = 0.1 -> 0.01 < |0.21| / 2
    assert fits.converged(o, f)
    assert not fits.converged([0.01, 0.2], [0.5, 0.6])


def test_golden_worked_examples():
    with open(os.path.join(GOLDEN, "fits_worked_examples.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        lam, y = np.array(case["lambda"]), np.array(case["value"])
        fid = np.array(case["fidelity"])
        if case["method"] == "loglin":
            v, _, _ = fits.fit_loglin_weighted(lam, y, fid,
                                               case["lambda_target"])
        elif case["method"] == "poly":
            v, _ = fits.fit_poly(lam, y, case["degree"], case["lambda_target"])
        else:
            v, _ = fits.fit_exp3(lam, y, case["lambda_target"])
        assert abs(v - case["expected"]) < case["tol"], case["name"]
