"""Laplace quadrature of the energy denominator (eq. laplace_transform).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); never used by the product.

The paper replaces 1/D of the triples by a sum over quadrature points,
1/x = int_0^inf exp(-x t) dt ~ sum_k w_k exp(-t_k x) for x = |D| > 0, with
n_q = 3-4 points chosen per system by the scheme of its LaplaceT reference,
which it does not print.  The scheme used here is the minimax exponential sum
(Takatsuka, Ten-no and Hackbusch, J. Chem. Phys. 129, 044112 (2008)): on
[1, R], with R the ratio of the largest to the smallest |D|, the weights and
exponents that minimise max |1/x - sum_k w_k exp(-a_k x)|.  The best
approximation is characterised by an error curve that equioscillates at
2n + 1 points of [1, R] (Braess and Hackbusch, IMA J. Numer. Anal. 25, 685
(2005)); it is found by Remez exchange: Newton steps on the 2n + 1
alternation equations for a set of extremal points, then the points moved to
the extrema of the new error curve, until the two agree.  Its start: for
n = 1, 2, ... in turn, the exponents of n - 1 terms plus one more, locally
optimised by Nelder-Mead (scipy) with the weights that minimise the maximum
error on a dense grid for each trial (a linear program).  Where the exchange
does not converge (larger n at small R), that local fit is kept: then the
sum is close to, not exactly, minimax, and the error returned is the one
measured, which is what the pins use.  For denominators in [x_min, x_max]
the exponents and weights are scaled by 1 / x_min.
"""
from __future__ import annotations

import numpy as np


def _err(x, w, a):
    """1/x - sum_k w_k exp(-a_k x) on the points x."""
    return 1.0 / x - np.exp(-np.outer(x, a)) @ w


def _derr(x, w, a):
    """d/dx of _err."""
    return -1.0 / x**2 + np.exp(-np.outer(x, a)) @ (w * a)


def _lp_weights(a, x):
    """Weights minimising the maximum error on the grid x for exponents a
    (a linear program), and that maximum error."""
    from scipy.optimize import linprog
    B = np.exp(-np.outer(x, a))
    f = 1.0 / x
    m, n = B.shape
    c = np.zeros(n + 1)
    c[-1] = 1.0
    one = np.ones((m, 1))
    A = np.vstack([np.hstack([B, -one]), np.hstack([-B, -one])])
    b = np.concatenate([f, -f])
    res = linprog(c, A_ub=A, b_ub=b, bounds=[(None, None)] * n + [(0.0, None)], method="highs")
    if not res.success:
        return None, np.inf
    return res.x[:n], res.x[-1]


def _local_search(a0, R, n):
    """Exponents near a0 minimising the LP-optimal maximum error on a dense
    grid (Nelder-Mead on their logarithms), with their weights."""
    from scipy.optimize import minimize
    x = np.geomspace(1.0, R, 800)

    def obj(b):
        return _lp_weights(np.exp(np.sort(b)), x)[1]

    res = minimize(obj, np.log(a0), method="Nelder-Mead",
                   options={"xatol": 1e-7, "fatol": 1e-15, "maxiter": 300 * n, "maxfev": 400 * n})
    a = np.exp(np.sort(res.x))
    w, _ = _lp_weights(a, x)
    return w, a


def _extremal_set(w, a, R, n):
    """2n + 1 alternating extrema of the error curve on [1, R] (endpoints
    included), each refined by bisection on the derivative."""
    x = np.geomspace(1.0, R, 40000)
    e = _err(x, w, a)
    cand = [0]
    for k in range(1, len(x) - 1):
        if (e[k] - e[k - 1]) * (e[k + 1] - e[k]) <= 0.0 and e[k] != e[k - 1]:
            cand.append(k)
    cand.append(len(x) - 1)
    pts = []
    for k in cand:
        if k in (0, len(x) - 1):
            pts.append(x[k])
            continue
        lo, hi = x[k - 1], x[k + 1]
        dlo = _derr(np.array([lo]), w, a)[0]
        for _ in range(100):
            mid = 0.5 * (lo + hi)
            dm = _derr(np.array([mid]), w, a)[0]
            if dm == 0.0:
                break
            if (dm > 0) == (dlo > 0):
                lo, dlo = mid, dm
            else:
                hi = mid
        pts.append(0.5 * (lo + hi))
    pts = np.array(pts)
    ev = _err(pts, w, a)
    # merge neighbours of equal sign, keeping the larger magnitude
    keep_x, keep_e = [pts[0]], [ev[0]]
    for xx, ee in zip(pts[1:], ev[1:]):
        if np.sign(ee) == np.sign(keep_e[-1]):
            if abs(ee) > abs(keep_e[-1]):
                keep_x[-1], keep_e[-1] = xx, ee
        else:
            keep_x.append(xx)
            keep_e.append(ee)
    keep_x, keep_e = np.array(keep_x), np.array(keep_e)
    m = 2 * n + 1
    if len(keep_x) < m:
        return None
    # the window of m consecutive alternation points with the largest smallest error
    best, start = -1.0, 0
    for s0 in range(len(keep_x) - m + 1):
        v = np.min(np.abs(keep_e[s0:s0 + m]))
        if v > best:
            best, start = v, s0
    return keep_x[start:start + m]


def _newton(w, a, xs, iters=60):
    """Solve err(x_i) = (-1)^i E (i = 0..2n) for w, a, E from the given start."""
    n = len(w)
    sgn = (-1.0) ** np.arange(len(xs))
    E = float(np.mean(sgn * _err(xs, w, a)))
    z = np.concatenate([w, np.log(a), [E]])
    for _ in range(iters):
        w_, b_, E_ = z[:n], z[n:2 * n], z[-1]
        a_ = np.exp(b_)
        ex = np.exp(-np.outer(xs, a_))
        F = 1.0 / xs - ex @ w_ - sgn * E_
        J = np.hstack([-ex, ex * (w_ * a_)[None, :] * xs[:, None], -sgn[:, None]])
        try:
            dz = np.linalg.solve(J, -F)
        except np.linalg.LinAlgError:
            return None
        step = 1.0
        f0 = np.max(np.abs(F))
        while step > 1e-4:
            zt = z + step * dz
            at = np.exp(zt[n:2 * n])
            Ft = 1.0 / xs - np.exp(-np.outer(xs, at)) @ zt[:n] - sgn * zt[-1]
            if np.max(np.abs(Ft)) < f0 or f0 < 1e-15:
                break
            step *= 0.5
        z = z + step * dz
        if np.max(np.abs(step * dz)) < 1e-14 * max(1.0, np.max(np.abs(z))):
            break
    return z[:n], np.exp(z[n:2 * n]), z[-1]


def _remez(w, a, R, n, rounds=40):
    """Remez exchange from (w, a): the equioscillating curve, or None when
    the exchange does not converge."""
    grid = np.geomspace(1.0, R, 40000)
    xs = _extremal_set(w, a, R, n)
    if xs is None:
        i = np.arange(2 * n + 1)
        xs = R ** ((1.0 - np.cos(np.pi * i / (2 * n))) / 2.0)
    for _ in range(rounds):
        with np.errstate(over="ignore", invalid="ignore"):
            out = _newton(w, a, xs)
        if out is None:
            return None
        w2, a2, E2 = out
        if not (np.all(np.isfinite(a2)) and np.all(np.isfinite(w2)) and np.all(a2 > 0)):
            return None
        order = np.argsort(a2)
        w, a = w2[order], a2[order]
        if np.max(np.abs(_err(grid, w, a))) <= abs(E2) * (1.0 + 1e-9):
            return w, a
        xs = _extremal_set(w, a, R, n)
        if xs is None:
            return None
    return None


def _table(nmax, R):
    """Exponent sums for n = 1..nmax, each started from the previous one with
    one more exponent (the geometric continuation of the last two)."""
    out = {}
    grid = np.geomspace(1.0, R, 40000)
    a0 = np.array([1.0 / np.sqrt(R)])
    for n in range(1, nmax + 1):
        if n == 2:
            a0 = np.array([out[1][1][0] * 0.2, out[1][1][0] * 5.0])
        elif n > 2:
            ap = out[n - 1][1]
            a0 = np.concatenate([ap, [ap[-1] * ap[-1] / ap[-2]]])
        w, a = _local_search(a0, R, n)
        pol = _remez(w, a, R, n)
        if pol is not None and np.max(np.abs(_err(grid, *pol))) < np.max(np.abs(_err(grid, w, a))):
            w, a = pol
        out[n] = (w, a)
    return out


def minimax(n: int, R: float):
    """Exponential sum of 1/x on [1, R] with n terms, minimax where the
    exchange converges (otherwise the best local minimax-in-weights fit).

    Returns (a, w, emax): exponents (increasing), weights, and the maximum
    error over [1, R] on a grid of 200001 log-spaced points."""
    if n < 1 or not R > 1.0:
        raise ValueError("need n >= 1 and R > 1")
    w, a = _table(n, R)[n]
    grid = np.geomspace(1.0, R, 200001)
    return a, w, float(np.max(np.abs(_err(grid, w, a))))


def quadrature(n: int, xmin: float, xmax: float):
    """Points t_k and weights w_k with 1/x ~ sum_k w_k exp(-t_k x) on
    [xmin, xmax] (minimax in the absolute error of 1/x scaled to [1, R]);
    also returns the bound on |1/x - sum| over the interval."""
    R = xmax / xmin
    a, w, emax = minimax(n, max(R, 1.0 + 1e-9))
    return a / xmin, w / xmin, emax / xmin
