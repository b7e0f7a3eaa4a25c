"""Pins of the oracle's coefficients, potential and accelerations.

Closed forms: a Hernquist sphere is exactly the alpha = 1 zeroth mode
(a_000 = 1/sqrt(3), psi = -GM/(r+a)); a Plummer sphere is exactly the
alpha = 1/2 zeroth mode (a_000 = sqrt(12 pi)/8, psi = -GM/sqrt(r^2+a^2)).
Deterministic "quadrature particles" make the particle sum of Eq. (sumanlm)
an exact quadrature of Eq. (a_nlm).  Invariants: W = (1/2) sum m psi equals
-(1/2) sum |a|^2; per-l power is rotation invariant; forces are minus the
finite-difference gradient of the potential.
"""
import math

import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I


def _weights(nmax, lmax):
    w = []
    for n in range(nmax + 1):
        for l in range(lmax + 1):
            for j in range(2 * l + 1):
                w.append(1.0 if j == 0 else 2.0)
    return np.array(w)


def test_hernquist_quadrature_coefficients(O):
    B = O.basis(16, 10)
    q = I.quadrature_sphere("hernquist", 1.0, nr=40, nmu=24, nphi=24)
    c = O.coeffs(B, *q.pos, q.mass)
    assert c[0] == pytest.approx(1 / math.sqrt(3), rel=1e-12)
    assert np.abs(c[1:]).max() < 1e-12


def test_plummer_quadrature_coefficients_alpha_half(O):
    B = O.basis(10, 6, alpha=0.5)
    q = I.quadrature_sphere("plummer", 0.5, nr=40, nmu=16, nphi=16)
    c = O.coeffs(B, *q.pos, q.mass)
    assert c[0] == pytest.approx(math.sqrt(12 * math.pi) / 8, rel=1e-12)
    assert np.abs(c[1:]).max() < 1e-12


def test_closed_form_potential_and_force(O):
    pts = I.uniform_ball(300, 11, radius=5.0).pos
    r = np.sqrt((pts ** 2).sum(0))
    B = O.basis(8, 4)
    q = I.quadrature_sphere("hernquist", 1.0, nr=32, nmu=16, nphi=16)
    c = O.coeffs(B, *q.pos, q.mass)
    P, g = O.field(B, c, *pts)
    assert np.allclose(P, -1 / (1 + r), rtol=1e-11, atol=1e-13)
    assert np.allclose(g, -pts / (r * (1 + r) ** 2), rtol=1e-11, atol=1e-13)
    B2 = O.basis(8, 4, alpha=0.5)
    q2 = I.quadrature_sphere("plummer", 0.5, nr=32, nmu=16, nphi=16)
    c2 = O.coeffs(B2, *q2.pos, q2.mass)
    P2, g2 = O.field(B2, c2, *pts)
    assert np.allclose(P2, -1 / np.sqrt(1 + r * r), rtol=1e-11, atol=1e-13)
    assert np.allclose(g2, -pts / (1 + r * r) ** 1.5, rtol=1e-11, atol=1e-13)


def test_scale_radius_and_G(O):
    # Hernquist sphere of mass M, scale a in a basis with b = a and constant G:
    # a_000 scales as M sqrt(G / b) and psi = -G M / (r + a)
    M, a, G = 3.0, 2.0, 0.5
    q = I.quadrature_sphere("hernquist", 1.0, nr=32, nmu=8, nphi=8, M=M, a=a)
    B = O.basis(4, 2, b=a, G=G)
    c = O.coeffs(B, *q.pos, q.mass)
    assert c[0] == pytest.approx(M * math.sqrt(G / a) / math.sqrt(3), rel=1e-12)
    pts = I.uniform_ball(50, 2, radius=6.0).pos
    r = np.sqrt((pts ** 2).sum(0))
    P, g = O.field(B, c, *pts)
    assert np.allclose(P, -G * M / (r + a), rtol=1e-11)
    assert np.allclose(g, -G * M * pts / (r * (r + a) ** 2), rtol=1e-11)


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_potential_energy_identity(O, alpha):
    p = I.uniform_ball(400, 7)
    B = O.basis(6, 4, alpha=alpha)
    c = O.coeffs(B, *p.pos, p.mass)
    P, _ = O.field(B, c, *p.pos, acc=False)
    W = 0.5 * (p.mass * P).sum()
    assert W == pytest.approx(-0.5 * (_weights(6, 4) * c * c).sum(), rel=1e-13)


def test_force_is_minus_gradient(O):
    p = I.plummer(300, 3)
    B = O.basis(6, 4)
    c = O.coeffs(B, *p.pos, p.mass)
    pts = I.uniform_ball(40, 9, radius=3.0).pos
    _, g = O.field(B, c, *pts)
    h = 1e-5
    for i in range(3):
        dp = np.zeros((3, 1))
        dp[i] = h
        Pp, _ = O.field(B, c, *(pts + dp), acc=False)
        Pm, _ = O.field(B, c, *(pts - dp), acc=False)
        fd = -(Pp - Pm) / (2 * h)
        assert np.allclose(g[i], fd, rtol=1e-7, atol=1e-9)


def test_force_at_poles_is_finite_and_consistent(O):
    p = I.plummer(200, 4)
    B = O.basis(6, 6)
    c = O.coeffs(B, *p.pos, p.mass)
    pts = np.array([[0.0, 0.0], [0.0, 0.0], [0.7, -1.3]])
    _, g = O.field(B, c, *pts)
    assert np.isfinite(g).all()
    eps = 1e-7
    near = pts + np.array([[eps, -eps], [eps, eps], [0.0, 0.0]])
    _, gn = O.field(B, c, *near)
    assert np.allclose(g, gn, atol=1e-5)


def _power(c, nmax, lmax):
    w = _weights(nmax, lmax)
    El = np.zeros(lmax + 1)
    k = 0
    for n in range(nmax + 1):
        for l in range(lmax + 1):
            for j in range(2 * l + 1):
                El[l] += w[k] * c[k] ** 2
                k += 1
    return El


def test_power_is_rotation_invariant(O):
    p = I.plummer(500, 8)
    # squash it so that the l > 0 power is not just noise
    pos = p.pos * np.array([[1.0], [0.6], [0.3]])
    B = O.basis(6, 5)
    c = O.coeffs(B, *pos, p.mass)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    c2 = O.coeffs(B, *(Q @ pos), p.mass)
    assert np.allclose(_power(c, 6, 5), _power(c2, 6, 5), rtol=1e-12, atol=1e-15)


def test_monte_carlo_a000_statistics(O):
    B = O.basis(2, 0)
    errs = []
    for n in (10_000, 100_000):
        p = I.hernquist(n, 21)
        c = O.coeffs(B, *p.pos, p.mass)
        sigma = math.sqrt(1 / 18 - 1 / 36) * math.sqrt(12 * math.pi) * (1 / math.sqrt(4 * math.pi)) / math.sqrt(n)
        # Var[1/(1+r)] for Hernquist = E[1/(1+r)^2] - 1/9 = 1/6 - 1/9 = 1/18
        sigma = math.sqrt(1 / 18) * math.sqrt(3) / math.sqrt(n)
        errs.append(abs(c[0] - 1 / math.sqrt(3)))
        assert errs[-1] < 5 * sigma


def test_spherical_limit_approaches_enclosed_mass(O):
    # l_max = 0 (the paper's spherically symmetric variant): the radial force
    # converges to -G M(<r)/r^2 of the particle distribution as nmax grows
    q = I.quadrature_sphere("plummer", 1.0, nr=64, nmu=8, nphi=8)
    pts = np.array([[0.5, 1.0, 2.0, 4.0], [0.0] * 4, [0.0] * 4])
    menc = pts[0] ** 3 / (1 + pts[0] ** 2) ** 1.5
    errs = []
    for nmax in (4, 12, 24):
        B = O.basis(nmax, 0)
        c = O.coeffs(B, *q.pos, q.mass)
        _, g = O.field(B, c, *pts)
        errs.append(np.abs(g[0] / (-menc / pts[0] ** 2) - 1).max())
    assert errs[2] < errs[0] and errs[2] < 2e-3


def test_direct_summation_sign_and_normalisation(O):
    # A handful of particles: the expansion converges (slowly, it is a
    # truncated Green's function) to the direct-summation potential away from
    # the particles; this pins the overall sign and normalisation only.
    rng = np.random.default_rng(3)
    src = rng.normal(0, 0.3, (3, 4))
    m = np.array([0.3, 0.2, 0.4, 0.1])
    B = O.basis(40, 8)
    c = O.coeffs(B, *src, m)
    pts = np.array([[2.5, -2.0, 0.3], [0.5, 1.5, -2.2], [1.0, -0.7, 2.4]])
    P, _ = O.field(B, c, *pts, acc=False)
    direct = np.array([-(m / np.sqrt(((pts[:, k:k + 1] - src) ** 2).sum(0))).sum() for k in range(3)])
    assert np.allclose(P, direct, rtol=2e-2)


def test_zero_radius_returns_zero_force(O):
    p = I.plummer(100, 2)
    B = O.basis(4, 2)
    c = O.coeffs(B, *p.pos, p.mass)
    P, g = O.field(B, c, np.zeros(1), np.zeros(1), np.zeros(1))
    assert np.isfinite(P).all() and (g == 0).all()
