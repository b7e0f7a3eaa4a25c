"""Pins of the oracle's basis functions (radial Zhao family, harmonics).

Each check compares the oracle with something other than itself: scipy's
special functions, closed forms of the Hernquist-Ostriker normalisation,
independent quadrature (scipy.integrate.quad), finite differences.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp


def test_gegenbauer_matches_scipy(O):
    for lam in (0.75, 1.5, 2.0, 5.5, 21.5):
        for n in range(0, 17):
            for x in (-0.99, -0.4, 0.0, 0.3, 0.97):
                ref = sp.eval_gegenbauer(n, lam, x)
                got = O.gegenbauer(n, lam, x)
                assert got == pytest.approx(ref, rel=1e-12, abs=1e-12 * max(1.0, abs(ref)))


def _closed_form_norm_alpha1(n, l, b=1.0, G=1.0):
    # Hernquist & Ostriker (1992) normalisation of the alpha = 1 family in the
    # energy inner product:  (b/G) K_nl Gamma(n+4l+3) /
    #   (2^(8l+6) n! (n+2l+3/2) Gamma(2l+3/2)^2),  K_nl = n(n+4l+3)/2 + (l+1)(2l+1)
    K = 0.5 * n * (n + 4 * l + 3) + (l + 1) * (2 * l + 1)
    lg = math.lgamma(n + 4 * l + 3) - math.lgamma(n + 1) - 2 * math.lgamma(2 * l + 1.5)
    return b / G * K * math.exp(lg) / (2.0 ** (8 * l + 6) * (n + 2 * l + 1.5))


@pytest.mark.parametrize("b,G", [(1.0, 1.0), (2.5, 0.7)])
def test_norm_alpha1_closed_form(O, b, G):
    B = O.basis(16, 10, alpha=1.0, b=b, G=G)
    N = O.norms(B)
    for n in range(17):
        for l in range(11):
            assert N[n, l] == pytest.approx(_closed_form_norm_alpha1(n, l, b, G), rel=1e-10)
    assert N[0, 0] == pytest.approx(b / G / (12 * math.pi), rel=1e-12)


def test_norm_alpha_half_hand_value(O):
    B = O.basis(6, 4, alpha=0.5)
    assert O.norms(B)[0, 0] == pytest.approx(3.0 / 64.0, rel=1e-12)


def _scipy_energy_inner(O, alpha, l, n1, n2):
    """Independent quadrature of int [s^2 f1' f2' + l(l+1) f1 f2] ds / (4 pi)
    with f built from scipy's Gegenbauer polynomials and scipy's derivative."""
    lam = (2 * l + 1) * alpha + 0.5

    def f(s, n):
        t = s ** (1 / alpha)
        xi = (t - 1) / (t + 1)
        return -s ** l * (1 + t) ** (-alpha * (2 * l + 1)) * sp.eval_gegenbauer(n, lam, xi)

    def df(s, n, h=1e-6):
        hh = h * max(s, 1e-3)
        return (f(s + hh, n) - f(s - hh, n)) / (2 * hh)

    def integrand(v):
        s = math.exp(v)
        return (s * s * df(s, n1) * df(s, n2) + l * (l + 1) * f(s, n1) * f(s, n2)) * s

    val, _ = si.quad(integrand, -40, 40, limit=400, epsabs=1e-14, epsrel=1e-11)
    return val / (4 * math.pi)


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_energy_orthonormality_independent(O, alpha):
    B = O.basis(6, 3, alpha=alpha)
    N = O.norms(B)
    for l in (0, 1, 3):
        for n1, n2 in ((0, 0), (2, 2), (3, 1), (5, 0), (4, 2)):
            ref = _scipy_energy_inner(O, alpha, l, n1, n2)
            got = O.energy_inner(B, l, n1, n2)
            scale = math.sqrt(N[n1, l] * N[n2, l])
            assert abs(got - ref) < 1e-6 * scale
            if n1 != n2:
                assert abs(got) < 1e-12 * scale


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.8])
def test_radial_derivative_matches_finite_difference(O, alpha):
    for l in (0, 2, 5):
        for s in (0.05, 0.7, 3.0, 20.0):
            f, df = O.radial_raw(alpha, l, 8, s)
            h = 1e-6 * s
            fp, _ = O.radial_raw(alpha, l, 8, s + h)
            fm, _ = O.radial_raw(alpha, l, 8, s - h)
            fd = (fp - fm) / (2 * h)
            assert np.allclose(df, fd, rtol=1e-6, atol=1e-9 * np.abs(f).max())


def test_zeroth_mode_is_paper_u00(O):
    # Eq. (u00): U_0^0 is proportional to (1 + (r/b)^(1/alpha))^(-alpha)
    for alpha in (1.0, 0.5, 0.7):
        s = np.array([0.01, 0.3, 1.0, 4.0, 50.0])
        f0 = np.array([O.radial_raw(alpha, 0, 0, si_)[0][0] for si_ in s])
        ref = (1 + s ** (1 / alpha)) ** (-alpha)
        ratio = f0 / ref
        assert np.allclose(ratio, ratio[0], rtol=1e-13)


def test_ylm_matches_scipy(O):
    rng = np.random.default_rng(5)
    for _ in range(20):
        th = rng.uniform(0, math.pi)
        ph = rng.uniform(0, 2 * math.pi)
        Y = O.ylm(10, th, ph)
        for l in range(11):
            for m in range(l + 1):
                ref = sp.sph_harm_y(l, m, th, ph)
                assert abs(Y[l * (l + 1) // 2 + m] - ref) < 1e-13
                # negative m follows from the Condon-Shortley convention
                refm = sp.sph_harm_y(l, -m, th, ph)
                assert abs((-1) ** m * np.conj(Y[l * (l + 1) // 2 + m]) - refm) < 1e-13


def test_addition_theorem(O):
    for th in (0.0, 0.3, 1.2, math.pi):
        Y = O.ylm(10, th, 0.7)
        for l in range(11):
            tot = abs(Y[l * (l + 1) // 2]) ** 2 + 2 * sum(
                abs(Y[l * (l + 1) // 2 + m]) ** 2 for m in range(1, l + 1))
            assert tot == pytest.approx((2 * l + 1) / (4 * math.pi), rel=1e-13)
