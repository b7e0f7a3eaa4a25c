"""Cluster-frame centre of Sec. 2.1 and the basis parameters (alpha, b) of
Sec. 2, in FP64.

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the product path.

The frame is placed where the monopole coefficient a_000 of the expansion is
largest.  About a centre c, a_000(c) = (Y_00 / sqrt(N_00)) sum_k w_k
g(|x_k - c|) with g(r) = (1 + (r/b)^(1/alpha))^(-alpha) (Eq. u00), so its
stationary points satisfy sum_k w_k omega_k (x_k - c) = 0 with
omega = -g'(r)/r = t (1 + t)^(-alpha-1) / r^2, t = (r/b)^(1/alpha).  The
paper leaves the search procedure to its companion paper; the one read here
is the fixed-point iteration of that condition,
    c <- sum_k w_k omega_k x_k / sum_k w_k omega_k,
which climbs a_000 monotonically (the kernel is convex in r^2), from the
current origin until the step is at most tol * b (at most maxit steps).
Particles closer than rmin * b to the current c are left out of a step (their
weight has no finite limit there).

The same objective tunes alpha and b (Eq. u00 and the text after it): about a
fixed centre, a_000 = sum_k w_k Y_00 f(r_k) / sqrt(N_00) with
f(r) = (1 + (r/b)^(1/alpha))^(-alpha) and the energy norm
N_00 = (b / 4 pi G) int s^2 f'(s)^2 ds = b alpha B(alpha + 2, alpha) / (4 pi G)
(B the Beta function; 1/(12 pi) at alpha = 1 and 3/64 at alpha = 1/2 for
b = G = 1).  The basis is orthonormal in that norm, so a_000 is the
projection of the cluster potential on the unit zeroth mode, and its maximum
over (alpha, b) is the zeroth mode closest to the potential.
"""
from __future__ import annotations

import numpy as np


def a000_kernel(B, r):
    """g(r) of the zeroth mode (Eq. u00), without its constant factor."""
    t = (np.asarray(r, dtype=np.float64) / B.b) ** (1.0 / B.alpha)
    return (1.0 + t) ** (-B.alpha)


def a000_about(B, pos, w, c):
    """sum_k w_k g(|x_k - c|): a_000 about c up to its constant factor."""
    d = np.asarray(pos, dtype=np.float64) - np.asarray(c, dtype=np.float64)[:, None]
    return float((np.asarray(w, dtype=np.float64) * a000_kernel(B, np.sqrt((d * d).sum(0)))).sum())


def recentre(B, pos, w, c0=(0.0, 0.0, 0.0), tol=1e-6, maxit=100, rmin=1e-9):
    """The fixed-point iteration above; returns (c, steps taken)."""
    pos = np.asarray(pos, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    c = np.array(c0, dtype=np.float64)
    for it in range(1, maxit + 1):
        d = pos - c[:, None]
        r = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        ok = (w > 0) & (r > rmin * B.b)
        if not ok.any():
            return c, it
        t = (r[ok] / B.b) ** (1.0 / B.alpha)
        om = w[ok] * t * (1.0 + t) ** (-B.alpha - 1.0) / (r[ok] * r[ok])
        cn = (om * pos[:, ok]).sum(1) / om.sum()
        step = np.sqrt(((cn - c) ** 2).sum())
        c = cn
        if step <= tol * B.b:
            return c, it
    return c, maxit


def n00(alpha, b, G=1.0):
    """Energy norm of the zeroth mode, b alpha B(alpha+2, alpha) / (4 pi G)."""
    from math import exp, lgamma, pi
    beta = exp(lgamma(alpha + 2.0) + lgamma(alpha) - lgamma(2.0 * alpha + 2.0))
    return b * alpha * beta / (4.0 * pi * G)


def a000_basis(pos, w, alpha, b, G=1.0):
    """a_000 of the particles about the origin for the basis (alpha, b)."""
    pos = np.asarray(pos, dtype=np.float64)
    r = np.sqrt((pos * pos).sum(0))
    f = (1.0 + (r / b) ** (1.0 / alpha)) ** (-alpha)
    return float((np.asarray(w, dtype=np.float64) * f).sum() / np.sqrt(4.0 * np.pi * n00(alpha, b, G)))


def tune_basis(pos, w, alpha0=1.0, b0=1.0, G=1.0, alpha_min=0.25):
    """(alpha, b) maximising a_000 of the particles about the origin, with
    alpha in [alpha_min, 1]: scipy's L-BFGS-B on (alpha, ln b) with
    finite-difference gradients, from a coarse grid's best point."""
    from scipy.optimize import minimize
    pos = np.asarray(pos, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    f = lambda v: -a000_basis(pos, w, v[0], np.exp(v[1]), G)
    lb0 = np.log(b0)
    grid = [(f((a, lb)), a, lb) for a in np.linspace(alpha_min, 1.0, 7)
            for lb in np.linspace(lb0 - 4.0, lb0 + 4.0, 17)]
    _, a_start, lb_start = min(grid)
    res = minimize(f, np.array([a_start, lb_start]), method="L-BFGS-B",
                   bounds=[(alpha_min, 1.0), (lb0 - 12.0, lb0 + 12.0)],
                   options={"ftol": 1e-16, "gtol": 1e-12, "maxiter": 10000, "eps": 1e-9})
    v = np.array(res.x, dtype=np.float64)
    # Newton polish from a quadratic fitted on a 3 x 3 stencil (the gradient
    # by finite differences above resolves the maximum only to ~1e-6)
    h = 1e-4
    for _ in range(4):
        F0 = f(v)
        g = np.zeros(2)
        Hm = np.zeros((2, 2))
        for i in range(2):
            e = np.zeros(2)
            e[i] = h
            fp, fm = f(v + e), f(v - e)
            g[i] = (fp - fm) / (2 * h)
            Hm[i, i] = (fp - 2 * F0 + fm) / (h * h)
        e0, e1 = np.array([h, 0.0]), np.array([0.0, h])
        Hm[0, 1] = Hm[1, 0] = (f(v + e0 + e1) - f(v + e0 - e1) - f(v - e0 + e1) + f(v - e0 - e1)) / (4 * h * h)
        step = -np.linalg.solve(Hm, g)
        vn = v + step
        vn[0] = min(max(vn[0], alpha_min), 1.0)
        if f(vn) > F0:
            break
        v = vn
    return float(v[0]), float(np.exp(v[1])), -float(f(v))
