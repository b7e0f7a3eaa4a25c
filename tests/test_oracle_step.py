"""Pins of the oracle's leapfrog in the accelerating cluster frame.

An isolated SCF system integrated with kick-drift-kick is Hamiltonian with
H = K - (1/2) sum_t w_t a_t^2, so the energy error is bounded and scales as
dt^2; the angular momentum about the centre is conserved to roundoff (the
truncated expansion keeps every m for each l, so it is rotation covariant);
the map is time-reversible.  In a host, a massless tracer at the frame origin
stays there and the frame follows the host orbit.
"""
import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I


def _w(nmax, lmax):
    return np.array([1.0 if j == 0 else 2.0 for n in range(nmax + 1) for l in range(lmax + 1)
                     for j in range(2 * l + 1)])


def _energy(O, B, st, m):
    c = O.coeffs(B, *st[:3], m)
    return 0.5 * (m * (st[3:] ** 2).sum(0)).sum() - 0.5 * (_w(B.nmax, B.lmax) * c * c).sum()


def test_energy_error_scales_as_dt_squared(O):
    p = I.plummer(1500, 31)
    B = O.basis(6, 4)
    st0 = p.state()
    E0 = _energy(O, B, st0, p.mass)
    errs = []
    for dt, n in ((0.04, 25), (0.02, 50), (0.01, 100)):
        st, _, _ = O.step(B, None, st0, p.mass, np.zeros(6), dt, n)
        errs.append(abs(_energy(O, B, st, p.mass) - E0) / abs(E0))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs


def test_angular_momentum_conserved(O):
    p = I.plummer(800, 32)
    B = O.basis(6, 4)
    st, _, _ = O.step(B, None, p.state(), p.mass, np.zeros(6), 0.01, 40)
    L0 = (p.mass * np.cross(p.pos.T, p.vel.T).T).sum(1)
    L1 = (p.mass * np.cross(st[:3].T, st[3:].T).T).sum(1)
    scale = (p.mass * np.linalg.norm(p.pos, axis=0) * np.linalg.norm(p.vel, axis=0)).sum()
    assert np.abs(L1 - L0).max() < 1e-12 * scale


def test_time_reversibility(O):
    p = I.plummer(500, 33)
    B = O.basis(4, 3)
    H = O.host([(O.HOST_NFW, (232.98, 20.0))])
    cen = np.array([20.0, 0.0, 0.0, 0.1, 1.4, 0.3])
    st, c1, _ = O.step(B, H, p.state(), p.mass, cen, 0.01, 30)
    st[3:] *= -1
    c1[3:] *= -1
    back, c0, _ = O.step(B, H, st, p.mass, c1, 0.01, 30)
    assert np.abs(back[:3] - p.pos).max() < 1e-10
    assert np.abs(-back[3:] - p.vel).max() < 1e-10
    assert np.abs(c0[:3] - cen[:3]).max() < 1e-10


def test_frame_follows_host_orbit_and_origin_tracer(O):
    p = I.plummer(400, 34)
    # a massless tracer at the frame origin
    pos = np.concatenate([p.pos, np.zeros((3, 1))], axis=1)
    vel = np.concatenate([p.vel, np.zeros((3, 1))], axis=1)
    m = np.concatenate([p.mass, [0.0]])
    B = O.basis(4, 2)
    H = O.host([(O.HOST_LOG, (1.5, 1.0))])
    cen = np.array([20.0, 0.0, 0.0, 0.0, I.LOG_VC_20, 0.0])
    st, c1, _ = O.step(B, H, np.concatenate([pos, vel]), m, cen, 0.005, 50)
    tr = O.orbit(H, cen, 0.005, 50)
    assert np.allclose(c1, tr[-1], rtol=0, atol=1e-13)
    # the tracer only feels the (tiny) SCF force at the centre; without
    # the cluster it would not move at all
    st2, _, _ = O.step(B, H, np.zeros((6, 1)), np.zeros(1), cen, 0.005, 50)
    assert np.abs(st2).max() < 1e-12


def test_batched_equals_per_cluster(O):
    B = O.basis(4, 2)
    H = O.host([(O.HOST_HERNQUIST, (1.11955, 1.0)), (O.HOST_MN, (11.8372, 3.0, 0.28)),
                (O.HOST_NFW, (124.107, 15.626))])
    cl = [I.plummer(n, 40 + i) for i, n in enumerate((150, 300, 90))]
    cens = [np.array([15.0 + 5 * i, 0.0, 1.0, 0.0, 1.3, 0.2]) for i in range(3)]
    off = np.cumsum([0] + [c.n for c in cl])
    st = np.concatenate([c.state() for c in cl], axis=1)
    m = np.concatenate([c.mass for c in cl])
    sb, cb, coefb = O.step_batched(B, H, off, st, m, np.stack(cens), 0.01, 5)
    for i, c in enumerate(cl):
        s1, c1, k1 = O.step(B, H, c.state(), c.mass, cens[i], 0.01, 5)
        assert np.array_equal(s1, sb[:, off[i]:off[i + 1]])
        assert np.array_equal(c1, cb[i])
        assert np.array_equal(k1, coefb[i])


def test_nsteps_zero_returns_input_and_acceleration(O):
    p = I.plummer(200, 35)
    B = O.basis(4, 2)
    st, cen, coef, acc = O.step(B, None, p.state(), p.mass, np.zeros(6), 0.01, 0, want_acc=True)
    assert np.array_equal(st, p.state())
    _, g = O.field(B, O.coeffs(B, *p.pos, p.mass), *p.pos)
    assert np.allclose(acc, g, rtol=0, atol=0)
