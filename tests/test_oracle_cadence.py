"""Pins of the refresh-cadence oracle (Sec. 2.2).

* Eq. tidal_timestep: the Kepler limit (a Hernquist host of vanishing scale
  radius, |T|^2 = 6 (GM/r^3)^2, so Delta t_int = sqrt(eta r^3 / GM)) and the
  closed-form Hessian of the logarithmic host.
* Energy Lagrange radius: brute force over candidate radii.
* Bound test: the SCF potential of quadrature particles of a Hernquist sphere
  is -1/(1 + r) exactly, so points moving at f v_esc have e = (f^2 - 1)/(1 + r).
* Frozen-potential leapfrog: a kick-drift-kick written out here with the
  closed-form Hernquist cluster force and a Hernquist host's differential
  field.
* Refreshes: linearity identities; the driver's schedule (interval lengths
  from the centre orbit, complete refresh every k-th interval, coefficients
  after a complete refresh equal those of the selected particles).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import cadence as K
from paper_2602_13385_amd import inputs as I


def _host(O, comps, G=1.0):
    kinds = {"log": O.HOST_LOG, "hernquist": O.HOST_HERNQUIST, "nfw": O.HOST_NFW, "mn": O.HOST_MN}
    return O.host([(kinds[k], p) for k, p in comps], G)


def test_tidal_timestep_kepler_limit(O):
    GM, eta = 2.5, 1.0 / 400.0
    H = _host(O, [("hernquist", (GM, 1e-9, 0.0))])
    for R in ([13.0, 0.0, 0.0], [3.0, 4.0, 12.0], [-7.0, 2.0, 5.0]):
        r = math.sqrt(sum(c * c for c in R))
        assert K.tidal_timestep(H, R, eta) == pytest.approx(math.sqrt(eta * r ** 3 / GM), rel=1e-8)


def test_tidal_timestep_log_host_closed_form(O):
    v0, rc, eta = 1.5, 1.0, 1.0 / 400.0
    H = _host(O, [("log", (v0, rc, 0.0))])
    for R in ([20.0, 0.0, 0.0], [0.3, -0.4, 0.2], [5.0, 5.0, -1.0]):
        r2 = sum(c * c for c in R)
        s = r2 + rc * rc
        # psi = v0^2/2 ln(r^2 + rc^2): Hessian eigenvalues v0^2 (rc^2 - r^2)/s^2
        # (radial) and v0^2/s (twice, tangential)
        t2 = v0 ** 4 * (((rc * rc - r2) / (s * s)) ** 2 + 2.0 / (s * s))
        assert K.tidal_timestep(H, R, eta) == pytest.approx(math.sqrt(eta) * (t2 / 6.0) ** -0.25,
                                                            rel=1e-12)


@pytest.mark.parametrize("frac", [0.5, 0.999, 0.9, 1.0, 0.1, 0.25])
def test_energy_radius_brute_force(frac):
    rng = np.random.default_rng(7)
    for n in (1, 2, 7, 100, 1000, 2345):
        r2 = rng.uniform(0.0, 10.0, n)
        bound = rng.uniform(size=n) < 0.8
        rx2, k, nb = K.energy_radius2(r2, bound, frac)
        assert nb == bound.sum()
        if nb == 0:
            assert rx2 == -np.inf
            continue
        # smallest candidate radius enclosing at least the fraction frac
        # (as the decimal it is written as) of the bound particles
        want = Fraction(str(frac)) * nb
        best = min(c for c in r2[bound] if (bound & (r2 <= c)).sum() >= want)
        assert rx2 == best


def test_bound_flags_and_selection_on_hernquist_quadrature(O):
    """Potential: Hernquist (M = a = 1) exactly, through the coefficients of
    quadrature particles; state: a random ball with speeds f v_esc(r)."""
    B = O.basis(6, 2)
    q = I.quadrature_sphere("hernquist", 1.0, nr=24, nmu=8, nphi=8)
    coef = O.coeffs(B, *q.pos, q.mass)
    p = I.uniform_ball(600, 4, radius=8.0)
    n = p.n
    r = np.sqrt((p.pos ** 2).sum(0))
    f = np.array([0.5, 0.8, 1.2, 1.5, 0.95, 1.05])[np.arange(n) % 6]
    u = np.stack([np.cos(np.arange(n)), np.sin(np.arange(n)), np.zeros(n)])
    vel = f * np.sqrt(2.0 / (1.0 + r)) * u
    st = np.concatenate([p.pos, vel])
    e = K.specific_energy(B, coef, st)
    np.testing.assert_allclose(e, (f * f - 1.0) / (1.0 + r), rtol=1e-10, atol=1e-12)
    w, bound, info = K.select(B, coef, st, p.mass, 0.9)
    assert np.array_equal(bound, f < 1.0)
    rb = np.sort(r[f < 1.0])
    kk = int(math.ceil(0.9 * len(rb)))
    assert info["rx"] == pytest.approx(rb[kk - 1], rel=1e-14)
    assert np.array_equal(w > 0, (f < 1.0) & (r <= rb[kk - 1]))
    assert np.array_equal(w[w > 0], p.mass[w > 0])
    assert info["mbound"] == pytest.approx(p.mass[f < 1.0].sum(), rel=1e-14)
    assert info["rhm"] == pytest.approx(rb[int(math.ceil(0.5 * len(rb))) - 1], rel=1e-14)


def test_frozen_step_is_the_closed_form_leapfrog(O):
    """Cluster: Hernquist (M = 1, a = 1) exactly through quadrature
    coefficients; host: Hernquist (M_h, a_h); KDK written out here."""
    B = O.basis(6, 2)
    q = I.quadrature_sphere("hernquist", 1.0, nr=24, nmu=8, nphi=8)
    coef = O.coeffs(B, *q.pos, q.mass)
    Mh, ah = 50.0, 3.0
    H = _host(O, [("hernquist", (Mh, ah, 0.0))])
    p = I.uniform_ball(40, 3, radius=3.0)
    st0 = np.concatenate([p.pos, p.vel])
    cen0 = np.array([12.0, 1.0, -2.0, 0.1, 1.8, 0.2])
    dt, nsteps = 0.01, 7

    def g_hern(x, M, a):  # -grad(-M/(r + a))
        r = np.sqrt((x ** 2).sum(0))
        return -M * x / (r * (r + a) ** 2)

    def acc(x, R):
        return g_hern(x, 1.0, 1.0) + g_hern(R[:, None] + x, Mh, ah) - g_hern(R[:, None], Mh, ah)

    x, v = st0[:3].copy(), st0[3:].copy()
    R, V = cen0[:3].copy(), cen0[3:].copy()
    for _ in range(nsteps):
        v = v + 0.5 * dt * acc(x, R)
        V = V + 0.5 * dt * g_hern(R[:, None], Mh, ah)[:, 0]
        x = x + dt * v
        R = R + dt * V
        v = v + 0.5 * dt * acc(x, R)
        V = V + 0.5 * dt * g_hern(R[:, None], Mh, ah)[:, 0]
    st, cen = O.step_frozen(B, H, st0, coef, cen0, dt, nsteps)
    np.testing.assert_allclose(st[:3], x, rtol=0, atol=1e-11)
    np.testing.assert_allclose(st[3:], v, rtol=0, atol=1e-11)
    np.testing.assert_allclose(cen, np.concatenate([R, V]), rtol=0, atol=1e-12)


def test_refresh_identities(O):
    B = O.basis(4, 2)
    p = I.plummer(300, 5)
    st = np.asarray(p.state(), dtype=np.float64)
    m = np.asarray(p.mass, dtype=np.float64)
    rng = np.random.default_rng(1)
    w_old = np.where(rng.uniform(size=p.n) < 0.7, m, 0.0)
    w_new = np.where(rng.uniform(size=p.n) < 0.7, m, 0.0)
    c_old = K.complete_refresh(B, [st[:3]], w_old)
    c_inc, nch = K.intermediate_refresh(B, c_old, [st[:3]], w_old, w_new)
    c_full = K.complete_refresh(B, [st[:3]], w_new)
    assert nch == (w_old != w_new).sum()
    assert np.abs(c_inc - c_full).max() <= 1e-13 * np.abs(c_full).max()
    # identical samples average to one sample
    c3 = K.complete_refresh(B, [st[:3]] * 3, w_new)
    assert np.abs(c3 - c_full).max() <= 1e-14 * np.abs(c_full).max()
    # unchanged weights: nothing to add
    c_same, n0 = K.intermediate_refresh(B, c_old, [st[:3]], w_old, w_old)
    assert n0 == 0 and np.array_equal(c_same, c_old)


def test_sample_schedule_and_count():
    for nsub in (1, 2, 5, 13, 40):
        for ns in range(1, nsub + 1):
            ends = K.sample_ends(nsub, ns)
            assert len(ends) == ns and ends[-1] == nsub
            assert all(b > a for a, b in zip([0] + ends[:-1], ends))
    # t_dyn = C M^-1/2 r^3/2: with M = r = 1 it is C itself
    C = K.C_DYN
    assert K.n_samples(2.5 * C, 1.0, 1.0, 1) == 3
    assert K.n_samples(2.5 * C, 1.0, 1.0, 2) == 5
    assert K.n_samples(0.3 * C, 1.0, 1.0, 1) == 1
    assert K.n_samples(10.0, 1.0, 1.0, 0) == 1
    assert K.n_samples(10.0, 0.0, 1.0, 1) == 1
    # the paper's normalisation: M = 1e5 Msun, r_hm = 10 pc gives 4.3451 Myr
    G = 4.30091727e-3  # pc (km/s)^2 / Msun
    t_pc_kms = C * math.sqrt(10.0 ** 3 / (G * 1e5))
    assert t_pc_kms * 3.0856775814913673e13 / 3.15576e13 == pytest.approx(4.3451, rel=1e-12)


def test_evolve_schedule(O):
    """Plummer (N = 400) at R = 20 in the logarithmic host: interval lengths
    follow the centre orbit, a complete refresh comes every 3rd interval and
    gives the coefficients of the selected particles at the interval end."""
    B = O.basis(4, 2)
    p = I.plummer(400, 9)
    H = _host(O, [("log", (1.5, 1.0, 0.0))])
    st0 = np.asarray(p.state(), dtype=np.float64)
    m = np.asarray(p.mass, dtype=np.float64)
    cen0 = np.array([20.0, 0.0, 0.0, 0.0, I.LOG_VC_20, 0.0])
    coef0, w0, info0 = K.initial_refresh(B, st0, m, 0.999)
    eta, dt_max, every = 1.0 / 400.0, 0.02, 3
    st, cen, coef, w, cs, log = K.evolve(B, H, st0, m, cen0, coef0, w0, 7, eta=eta,
                                         dt_max=dt_max, refresh_every=every)
    assert [e["kind"] for e in log] == ["intermediate", "intermediate", "complete"] * 2 + \
        ["intermediate"]
    assert cs[0] == 1
    c = cen0.copy()
    for e in log:
        assert e["dt_int"] == pytest.approx(K.tidal_timestep(H, c[:3], eta), rel=1e-14)
        assert e["nsub"] == math.ceil(e["dt_int"] / dt_max)
        c = O.orbit(H, c, e["dt_int"] / e["nsub"], e["nsub"])[-1]
    np.testing.assert_allclose(cen, c, rtol=0, atol=1e-12)
    # the complete refresh of the 6th interval: replay intervals 1..6 and
    # compare with the coefficients of the selected particles
    st6, _, coef6, w6, _, _ = K.evolve(B, H, st0, m, cen0, coef0, w0, 6, eta=eta,
                                       dt_max=dt_max, refresh_every=every)
    c_sel = O.coeffs(B, *st6[:3], w6)
    assert np.abs(coef6 - c_sel).max() <= 1e-13 * np.abs(c_sel).max()
    assert 0 < log[-1]["nbound"] <= p.n
