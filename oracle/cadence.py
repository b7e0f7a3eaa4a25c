"""Refresh cadence of the SCF potential (Sec. 2.2), in FP64.

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the product path.
It builds on the FP64 oracle (``pyoracle``) and shares nothing with the GPU
library.

Between refreshes the particles move in a frozen SCF potential.  The paper
sets the length of these integration intervals from the host tidal tensor,
and refreshes the potential in two ways: completely every few intervals, and
with intermediate updates in between.  The pieces, in the paper's order:

* ``tidal_timestep``: Eq. tidal_timestep,
  Delta t_int = sqrt(eta) (|T|_F^2 / 6)^(-1/4), where T is the tidal tensor of
  Eq. tidal_tensor at the centre orbit's position at the start of the interval.
* ``specific_energy`` and ``select``: the bound test of the footnote to Sec. 2.2
  with the SCF potential in place of the direct pair sum and the usual kinetic
  factor 1/2 (bound iff |v|^2/2 + psi_SCF(x) < 0, in the cluster frame).  The
  energy Lagrange radius r_x is the smallest radius that encloses the fraction
  x of the bound particles: the k-th smallest bound radius, k = ceil(x N_b).
  Only bound particles with r <= r_99.9 enter the coefficient sum.
* ``n_samples``: the number of orbit samples, max(1, ceil(n_s Delta t_int /
  t_dyn)), with t_dyn = c_dyn M^(-1/2) r_hm^(3/2) from the bound mass and
  r_hm = r_50.
* ``evolve``: the driver.  Each interval is integrated by kick-drift-kick
  substeps of equal length h = Delta t_int / ceil(Delta t_int / dt_max) in the
  frozen potential.  Sample j (of N_s) is the positions after substep
  ceil((j+1) nsub / N_s), so the last one is the interval end.  At the end the
  selection is redone in the potential the particles moved in.  Every
  ``refresh_every``-th interval is a complete refresh: the coefficients of
  Eq. sumanlm over the selected particles, averaged over the samples.  The
  other intervals are intermediate refreshes: the contributions of the
  particles whose selection weight changed, with weights w' - w, are added
  over the same samples.

The radii are compared through their squares.  The caller picks the precision
of the squares (``key_dtype``): float32 keys reproduce the decisions of a
single-precision run, which computes |x|^2 as ((x x + y y) + z z) with every
operation rounded.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import frame as F
from oracle import pyoracle as O

# t_dyn / 4.3451 Myr = (M / 1e5 Msun)^(-1/2) (r_hm / 10 pc)^(3/2) (Sec. 2.2),
# written as t_dyn = C_DYN sqrt(r_hm^3 / (G M)) in any units with G explicit:
# G = 4.30091727e-3 pc (km/s)^2 / Msun and 1 pc / (km/s) = 0.977792222 Myr.
_T_UNIT_MYR = 3.0856775814913673e13 / 3.15576e13
C_DYN = 4.3451 / (math.sqrt(1000.0 / (4.30091727e-3 * 1e5)) * _T_UNIT_MYR)


def tidal_timestep(H, R, eta):
    """Eq. tidal_timestep at the host-frame position R."""
    T = O.tidal_norm(H, np.asarray(R, dtype=np.float64))
    return math.sqrt(eta) * (T * T / 6.0) ** -0.25


def specific_energy(B, coef, state):
    """|v|^2/2 + psi_SCF(x) per particle (cluster frame)."""
    st = np.asarray(state, dtype=np.float64)
    pot, _ = O.field(B, coef, st[0], st[1], st[2], pot=True, acc=False)
    return 0.5 * (st[3] ** 2 + st[4] ** 2 + st[5] ** 2) + pot


def squared_radii(state, key_dtype=np.float64):
    """|x|^2 evaluated as ((x x + y y) + z z) in key_dtype."""
    x, y, z = (np.asarray(state[i], dtype=key_dtype) for i in range(3))
    return (x * x + y * y) + z * z


def energy_radius2(r2, bound, frac):
    """Squared r_x: the k-th smallest bound squared radius, k = ceil(frac N_b)
    clamped to [1, N_b].  Returns (r_x^2, k, N_b); r_x^2 = -inf when N_b = 0."""
    rb = np.sort(np.asarray(r2)[np.asarray(bound, dtype=bool)])
    nb = len(rb)
    if nb == 0:
        return -np.inf, 0, 0
    k = min(max(int(math.ceil(frac * float(nb))), 1), nb)
    return rb[k - 1], k, nb


def rank_gap(r2, bound, k):
    """Relative distance of the k-th smallest bound squared radius to its
    neighbours (inf when it has none): how far the selection is from a tie."""
    rb = np.sort(np.asarray(r2, dtype=np.float64)[np.asarray(bound, dtype=bool)])
    if k < 1 or k > len(rb):
        return np.inf
    c = rb[k - 1]
    g = np.inf
    if k >= 2:
        g = min(g, (c - rb[k - 2]) / c)
    if k < len(rb):
        g = min(g, (rb[k] - c) / c)
    return g


def select(B, coef, state, m, frac, key_dtype=np.float64):
    """Bound flags, selection weights w = m [bound and r <= r_x] and the
    quantities the next interval needs (N_b, r_x, r_50, bound mass).  The info
    also reports how close the decisions are to their thresholds: the smallest
    |e| relative to the largest, and the rank gaps of r_x and r_50."""
    m = np.asarray(m, dtype=np.float64)
    e = specific_energy(B, coef, state)
    bound = e < 0.0
    r2 = squared_radii(state, key_dtype)
    rx2, kx, nb = energy_radius2(r2, bound, frac)
    rh2, kh, _ = energy_radius2(r2, bound, 0.5)
    w = np.where(bound & (r2 <= rx2), m, 0.0)
    ae = np.abs(e)
    info = {"nbound": nb, "rx": math.sqrt(float(rx2)) if nb else 0.0,
            "rhm": math.sqrt(float(rh2)) if nb else 0.0, "mbound": float(m[bound].sum()),
            "energy": e, "emargin": float(ae.min() / ae.max()) if len(e) else np.inf,
            "gap": min(rank_gap(r2, bound, kx), rank_gap(r2, bound, kh))}
    return w, bound, info


def n_samples(dt_int, mbound, rhm, n_samples_tdyn, c_dyn=C_DYN, G=1.0):
    """max(1, ceil(n_s Delta t_int / t_dyn)); 1 when sampling is off or the
    bound set is empty."""
    if n_samples_tdyn <= 0 or mbound <= 0.0 or rhm <= 0.0:
        return 1
    tdyn = c_dyn * math.sqrt(rhm ** 3 / (G * mbound))
    return max(1, int(math.ceil(n_samples_tdyn * dt_int / tdyn)))


def sample_ends(nsub, ns):
    """Substep index after which sample j (0-based) is taken."""
    return [-(-(j + 1) * nsub // ns) for j in range(ns)]


def complete_refresh(B, snaps, w):
    """Coefficients over the selected particles, averaged over the samples."""
    c = sum(O.coeffs(B, s[0], s[1], s[2], w) for s in snaps)
    return c / len(snaps)


def intermediate_refresh(B, coef, snaps, w_old, w_new):
    """coef plus the changed particles' contributions, weights w_new - w_old."""
    dw = np.asarray(w_new, dtype=np.float64) - np.asarray(w_old, dtype=np.float64)
    sel = dw != 0.0
    if not sel.any():
        return np.array(coef, dtype=np.float64, copy=True), 0
    c = sum(O.coeffs(B, s[0][sel], s[1][sel], s[2][sel], dw[sel]) for s in snaps)
    return np.asarray(coef, dtype=np.float64) + c / len(snaps), int(sel.sum())


def initial_refresh(B, state, m, frac, key_dtype=np.float64):
    """Start of a run: coefficients of all particles, the selection in their
    potential, then a complete refresh over the selected particles."""
    st = np.asarray(state, dtype=np.float64)
    c_all = O.coeffs(B, st[0], st[1], st[2], m)
    w, _, info = select(B, c_all, st, m, frac, key_dtype)
    coef = complete_refresh(B, [st[:3]], w)
    return coef, w, info


def evolve(B, H, state, m, centre, coef, w, nint, *, eta, dt_max, frac=0.999,
           refresh_every=5, n_samples_tdyn=0, c_dyn=C_DYN, ns_max=8, since=0, mbound=0.0,
           rhm=0.0, key_dtype=np.float64, recentre=False, retune=False, alpha_min=0.25):
    """nint integration intervals of the cadence.  Returns the state, centre,
    coefficients, weights, the cadence state (since, mbound, rhm) and one log
    entry per interval.  With recentre, a complete refresh first moves the
    frame origin to the a_000 maximum of the selected particles (Sec. 2.1;
    positions, samples and the centre shift), computes the coefficients, then
    moves the frame velocity to the core velocity of the new potential.  With
    retune, the complete refresh (after any recentring) first sets the basis
    (alpha, b) to the a_000 maximum over the selected particles; the basis in
    force at the end is returned as the last item."""
    st = np.array(state, dtype=np.float64, copy=True)
    cen = np.array(centre, dtype=np.float64, copy=True)
    coef = np.array(coef, dtype=np.float64, copy=True)
    w = np.array(w, dtype=np.float64, copy=True)
    m = np.asarray(m, dtype=np.float64)
    log = []
    for _ in range(nint):
        dti = tidal_timestep(H, cen[:3], eta)
        nsub = max(1, int(math.ceil(dti / dt_max)))
        h = dti / nsub
        ns = min(n_samples(dti, mbound, rhm, n_samples_tdyn, c_dyn, B.G), nsub, ns_max)
        ratio = (n_samples_tdyn * dti / (c_dyn * math.sqrt(rhm ** 3 / (B.G * mbound)))
                 if n_samples_tdyn > 0 and mbound > 0.0 and rhm > 0.0 else 0.0)
        snaps, done = [], 0
        for end in sample_ends(nsub, ns):
            st, cen = O.step_frozen(B, H, st, coef, cen, h, end - done)
            done = end
            snaps.append(st[:3].copy())
        w_new, _, info = select(B, coef, st, m, frac, key_dtype)
        since += 1
        dx, dv = np.zeros(3), np.zeros(3)
        if since >= refresh_every:
            nchanged = int((w_new != w).sum())
            if recentre:
                dx, _ = F.recentre(B, st[:3], w_new, tol=1e-6, maxit=100)
                st[:3] -= dx[:, None]
                snaps = [s - dx[:, None] for s in snaps[:-1]] + [st[:3].copy()]
                cen[:3] += dx
            if retune:
                a, b, _ = F.tune_basis(st[:3], w_new, B.alpha, B.b, B.G, alpha_min)
                B = O.basis(B.nmax, B.lmax, alpha=a, b=b, G=B.G)
            coef = complete_refresh(B, snaps, w_new)
            if recentre:
                _, dv, _ = O.core(B, coef, st, m, w_new)
                st[3:] -= dv[:, None]
                cen[3:] += dv
            since, kind = 0, "complete"
        else:
            coef, nchanged = intermediate_refresh(B, coef, snaps, w, w_new)
            kind = "intermediate"
        w = w_new
        mbound, rhm = info["mbound"], info["rhm"]
        log.append({"dt_int": dti, "nsub": nsub, "nsamples": ns, "kind": kind,
                    "nbound": info["nbound"], "nchanged": nchanged, "rx": info["rx"],
                    "rhm": rhm, "mbound": mbound, "emargin": info["emargin"],
                    "gap": info["gap"], "ns_ratio": ratio, "dx": dx, "dv": dv,
                    "alpha": B.alpha, "b": B.b})
    if retune:
        return st, cen, coef, w, (since, mbound, rhm), log, B
    return st, cen, coef, w, (since, mbound, rhm), log
