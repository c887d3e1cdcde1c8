"""Extrapolation fits of Sec. 2.2.2 and App. B.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``fit_poly``: least-squares polynomial in lambda (a low-degree fit; the
  quadratic is not from the paper, it is one of the synthetic workloads).
* ``fit_exp3``: the exponential Ansatz O(lambda) = a exp(-b lambda) + c
  (eq. ``exp_Ansatz``) fitted by unweighted mean-square error (the fallback of
  Sec. 2.2.2 (B) and App. D.1).  Variable projection: for a fixed b the model is
  linear in (a, c); the 1-D profile residual in b is minimised by a bracketed
  golden-section search and polished with Newton steps.  b is confined to
  [0, b_max].
* ``fit_loglin_weighted``: the primary log-linear fit of Sec. 2.2.2 (B) with
  c = 0, criteria 2 (|O| >= small) and 3 (same sign as at lambda = 0), and the
  weighted loss of App. B.2: sum_lambda w^2 (log|a| - b lambda - log|O|)^2,
  w = F^delta_f * exp(-delta_d |lambda* - lambda| / d), d the dip size.
* ``nzne``: the decision chain of Sec. 2.2.2 (B): log-linear if at least two
  points survive criteria 2-3, else the direct exponential fit on every point
  (criteria 2-3 dropped), else no extrapolation.
* ``fidelity_extrapolation`` / ``converged``: step (A) of Sec. 2.2.2 (straight
  line in emulation fidelity, evaluated at F = 1) and App. B.1's criterion 1.
"""
import numpy as np

GOLDEN = (np.sqrt(5.0) - 1.0) / 2.0


def fit_poly(lam, y, degree, lam_target):
    lam = np.asarray(lam, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if lam.size < degree + 1:
        raise ValueError("too few points")
    V = np.vander(lam, degree + 1, increasing=True)     # columns 1, l, l^2 ..
    coef, *_ = np.linalg.lstsq(V, y, rcond=None)
    value = float(np.polyval(coef[::-1], lam_target))
    return value, coef


def _exp3_linear(lam, y, b):
    """For fixed b: least-squares (a, c) and the residual sum of squares."""
    A = np.column_stack([np.exp(-b * lam), np.ones_like(lam)])
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    r = A @ coef - y
    return coef, float(r @ r)


def fit_exp3(lam, y, lam_target, b_max=None):
    lam = np.asarray(lam, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if lam.size < 3:
        raise ValueError("too few points")
    span = lam.max() - lam.min()
    if b_max is None:
        b_max = 50.0 / span
    # coarse scan to bracket the minimum of the profile residual
    grid = np.linspace(0.0, b_max, 401)
    rss = np.array([_exp3_linear(lam, y, b)[1] for b in grid])
    i = int(np.argmin(rss))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, grid.size - 1)]
    # golden-section search on [lo, hi]
    x1 = hi - GOLDEN * (hi - lo)
    x2 = lo + GOLDEN * (hi - lo)
    f1 = _exp3_linear(lam, y, x1)[1]
    f2 = _exp3_linear(lam, y, x2)[1]
    for _ in range(200):
        if hi - lo <= 1e-15 * max(1.0, abs(hi)):
            break
        if f1 < f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - GOLDEN * (hi - lo)
            f1 = _exp3_linear(lam, y, x1)[1]
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + GOLDEN * (hi - lo)
            f2 = _exp3_linear(lam, y, x2)[1]
    b = 0.5 * (lo + hi)
    # Newton polish on the profile residual (central differences)
    for _ in range(20):
        h = 1e-5 * max(1.0, abs(b))
        fm = _exp3_linear(lam, y, b - h)[1]
        f0 = _exp3_linear(lam, y, b)[1]
        fp = _exp3_linear(lam, y, b + h)[1]
        d2 = (fp - 2 * f0 + fm) / (h * h)
        if d2 <= 0:
            break
        step = -((fp - fm) / (2 * h)) / d2
        nb = min(max(b + step, 0.0), b_max)
        if _exp3_linear(lam, y, nb)[1] > f0:
            break
        if abs(nb - b) <= 1e-14 * max(1.0, abs(b)):
            b = nb
            break
        b = nb
    (a, c), _ = _exp3_linear(lam, y, b)
    value = float(a * np.exp(-b * lam_target) + c)
    return value, np.array([a, b, c])


def dip_size(lam, fid, threshold=0.99):
    """Smallest non-zero lambda whose emulation fidelity exceeds the
    threshold (App. B.2); the largest lambda if none does."""
    lam = np.asarray(lam, dtype=np.float64)
    fid = np.asarray(fid, dtype=np.float64)
    cand = [l for l, f in zip(lam, fid) if l > 0 and f > threshold]
    return float(min(cand)) if cand else float(lam.max())


def fit_loglin_weighted(lam, y, fid, lam_target, delta_f=2.0, delta_d=20.0,
                        small=1e-10, dip_threshold=0.99, ref_sign=0):
    """Returns (value, (a, b), used_mask) or raises ValueError if fewer than
    two points pass criteria 2-3."""
    lam = np.asarray(lam, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    fid = np.asarray(fid, dtype=np.float64)
    if ref_sign == 0:
        ref_sign = 1.0 if y[int(np.argmin(lam))] >= 0 else -1.0
    used = (np.abs(y) >= small) & (np.sign(y) == ref_sign)
    if used.sum() < 2:
        raise ValueError("too few points for the log-linear fit")
    d = dip_size(lam, fid, dip_threshold)
    w = fid ** delta_f * np.exp(-delta_d * np.abs(lam_target - lam) / d)
    lu, yu, wu = lam[used], np.log(np.abs(y[used])), w[used]
    # minimise sum w^2 (alpha - b l - log|y|)^2 over (alpha, b)
    A = np.column_stack([np.ones_like(lu), -lu]) * wu[:, None]
    sol, *_ = np.linalg.lstsq(A, yu * wu, rcond=None)
    alpha, b = sol
    a = ref_sign * np.exp(alpha)
    return float(a * np.exp(-b * lam_target)), np.array([a, b]), used


def nzne(lam, y, fid, lam_target, **kw):
    """Sec. 2.2.2 (B) decision chain.  Returns (value, method, coef, used)
    with method in {"loglin", "exp3", "none"}."""
    try:
        v, coef, used = fit_loglin_weighted(lam, y, fid, lam_target, **kw)
        return v, "loglin", coef, used
    except ValueError:
        pass
    lam = np.asarray(lam, dtype=np.float64)
    if lam.size >= 3:
        v, coef = fit_exp3(lam, y, lam_target)
        return v, "exp3", coef, np.ones(lam.size, dtype=bool)
    return None, "none", None, np.zeros(lam.size, dtype=bool)


def fidelity_extrapolation(values, fids):
    """Straight-line fit of <O>^(D_j) against F^(D_j), evaluated at F = 1."""
    f = np.asarray(fids, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    A = np.column_stack([np.ones_like(f), f])
    (c0, c1), *_ = np.linalg.lstsq(A, v, rcond=None)
    return float(c0 + c1)


def converged(values, fids):
    """App. B.1: |d<O>/dF| (1 - F_k) < |<O>_k| / 2 over the two largest D."""
    o1, o2 = values[-2], values[-1]
    f1, f2 = fids[-2], fids[-1]
    slope = abs((o2 - o1) / (f2 - f1))
    return bool(slope * (1.0 - f2) < abs(o2) / 2.0)
