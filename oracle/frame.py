"""Cluster-frame centre of Sec. 2.1, in FP64.

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
