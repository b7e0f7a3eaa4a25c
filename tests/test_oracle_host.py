"""Pins of the oracle's host potentials and centre orbit.

Appendix A gives potentials, forces and tidal terms; forces must be minus the
finite-difference gradient and the Hessian the finite difference of the
gradient.  The paper's MilkyWayPotential2022 orbit table (Sec. 2.3, integrated
for 5 Gyr at 0.1 Myr) pins the host model and the leapfrog together.
"""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
G_ASTRO = 4.300917270e-6  # kpc (km/s)^2 / Msun (the paper does not print G)
KPC_KMS_GYR = 0.9777922216807891  # 1 kpc / (km/s) in Gyr


def _hosts(O):
    return {
        "log": O.host([(O.HOST_LOG, (1.5, 1.0))]),
        "hernquist": O.host([(O.HOST_HERNQUIST, (2.0, 1.5))], G=0.8),
        "nfw": O.host([(O.HOST_NFW, (232.98, 20.0))]),
        "mn": O.host([(O.HOST_MN, (11.8, 3.0, 0.28))]),
        "plummer": O.host([(O.HOST_PLUMMER, (5.0, 2.0))]),
        "composite": O.host([(O.HOST_HERNQUIST, (1.11955, 1.0)), (O.HOST_MN, (11.8372, 3.0, 0.28)),
                             (O.HOST_NFW, (124.107, 15.626))]),
    }


@pytest.mark.parametrize("name", ["log", "hernquist", "nfw", "mn", "plummer", "composite"])
def test_host_gradient_and_hessian_by_differences(O, name):
    H = _hosts(O)[name]
    rng = np.random.default_rng(4)
    for _ in range(6):
        p = rng.normal(0, 8.0, 3)
        _, g, hs = O.host_eval(H, p)
        h = 1e-4
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            # fourth-order central differences
            v = [O.host_eval(H, p + k * e) for k in (2, 1, -1, -2)]
            fd_g = (-v[0][0] + 8 * v[1][0] - 8 * v[2][0] + v[3][0]) / (12 * h)
            fd_h = (-v[0][1] + 8 * v[1][1] - 8 * v[2][1] + v[3][1]) / (12 * h)
            assert g[i] == pytest.approx(fd_g, rel=1e-8, abs=1e-11)
            assert np.allclose(hs[:, i], fd_h, rtol=1e-7, atol=1e-11)
        assert np.allclose(hs, hs.T, atol=1e-14)


@pytest.mark.parametrize("name", ["log", "hernquist", "nfw", "mn", "plummer"])
def test_host_parameter_derivatives_by_differences(O, name):
    H = _hosts(O)[name]
    rng = np.random.default_rng(7)
    p = rng.normal(0, 8.0, 3)
    d = O.host_dgrad_dparam(H, p)[0]
    kinds = {"log": 2, "hernquist": 2, "nfw": 2, "mn": 3, "plummer": 2}
    for k in range(kinds[name]):
        comp = H.comp[0]
        base = comp.p[k]
        hstep = 1e-6 * abs(base)
        comp.p[k] = base + hstep
        _, gp, _ = O.host_eval(H, p)
        comp.p[k] = base - hstep
        _, gm, _ = O.host_eval(H, p)
        comp.p[k] = base
        assert np.allclose(d[k], (gp - gm) / (2 * hstep), rtol=1e-6, atol=1e-12)


def test_paper_tidal_terms_hernquist_nfw(O):
    # the paper's d f_r / d r for Hernquist: 2 G M / r^3 (r/a)^3 / (1 + r/a)^3
    H = O.host([(O.HOST_HERNQUIST, (3.0, 1.3))], G=1.0)
    r = 2.7
    _, _, hs = O.host_eval(H, np.array([r, 0.0, 0.0]))
    assert -hs[0, 0] == pytest.approx(2 * 3.0 / r ** 3 * (r / 1.3) ** 3 / (1 + r / 1.3) ** 3, rel=1e-13)
    # NFW: 2 G M g / r^3 (1 - (x/(1+x))^2 / (2 g)),  g = ln(1+x) - x/(1+x)
    H = O.host([(O.HOST_NFW, (100.0, 15.0))])
    x = r / 15.0
    g = math.log1p(x) - x / (1 + x)
    _, _, hs = O.host_eval(H, np.array([0.0, r, 0.0]))
    assert -hs[1, 1] == pytest.approx(2 * 100.0 * g / r ** 3 * (1 - (x / (1 + x)) ** 2 / (2 * g)),
                                      rel=1e-12)


def _load_mw2022(O):
    comps = []
    with open(os.path.join(HERE, "golden", "mw2022_host.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, M, a, b = line.split()
            k = {"hernquist": O.HOST_HERNQUIST, "mn": O.HOST_MN, "nfw": O.HOST_NFW}[kind]
            comps.append((k, (float(M), float(a), float(b))))
    H = O.host(comps, G=G_ASTRO)
    rows = []
    with open(os.path.join(HERE, "golden", "mw2022_orbits.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([float(v) for v in line.split()])
    return H, np.array(rows)


def test_mw2022_orbit_table(O):
    H, rows = _load_mw2022(O)
    dt = 1e-4 / KPC_KMS_GYR  # 0.1 Myr
    nsteps = int(round(5.0 / KPC_KMS_GYR / dt))
    for row in rows:
        ic = row[1:7]
        tr = O.orbit(H, ic, dt, nsteps)
        r = np.sqrt((tr[:, :3] ** 2).sum(1))
        rp, ra = r.min(), r.max()
        e = (ra - rp) / (ra + rp)
        Lz = ic[0] * ic[4] - ic[1] * ic[3]
        E = 0.5 * (ic[3:] ** 2).sum() + O.host_eval(H, ic[:3])[0]
        got = [rp, ra, e, Lz / 1e3, E / 1e5]
        for g, ref in zip(got, row[7:12]):
            assert abs(g - ref) <= 0.005 + 1e-9, (row[0], got, row[7:12])
        # the leapfrog conserves the host energy along the orbit
        Eend = 0.5 * (tr[-1, 3:] ** 2).sum() + O.host_eval(H, tr[-1, :3])[0]
        assert abs(Eend - E) < 1e-4 * abs(E)
