"""Pins of the oracle's coefficient and potential assembly for l > 0.

Eq. (a_nlm)/(sumanlm) of Sec. 2: one particle of mass m at x gives
a_nlm = -m U_nl(r) conj(Y_lm(theta, phi)); Eq. (psi_nlm) and the total
potential give, for a coefficient vector with a single non-zero stored entry,
psi = w U_nl(r) {Y_l0, Re Y_lm, Im Y_lm} with w = 1 (Re a_nl0), 2 (Re a_nlm)
and -2 (Im a_nlm), since the m < 0 terms are the complex conjugates.  Here
U_nl and Y_lm are built independently of the oracle: the radial function
from scipy's Gegenbauer polynomials and, for alpha = 1, the closed-form
Hernquist-Ostriker energy norm; the harmonics from scipy.special.sph_harm_y
(Condon-Shortley phase, theta polar).  A per-degree scale error, a wrong
b^-l factor at b != 1, a wrong G scaling or a conjugated imaginary part would
each fail these checks.

The Monte-Carlo pin: for a Hernquist sphere sampled with N particles the
estimate of a_000 = 1/sqrt(3) has variance Var[sqrt(3)/(1+r)]/N = 1/(6N); the
root-mean-square error over seeds follows sigma_N and falls with slope -1/2
in log N.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from paper_2602_13385_amd import inputs as I


def _closed_norm_alpha1(n, l, b, G):
    K = 0.5 * n * (n + 4 * l + 3) + (l + 1) * (2 * l + 1)
    lg = math.lgamma(n + 4 * l + 3) - math.lgamma(n + 1) - 2 * math.lgamma(2 * l + 1.5)
    return b / G * K * math.exp(lg) / (2.0 ** (8 * l + 6) * (n + 2 * l + 1.5))


def _U_independent(O, B, l, r):
    """U_nl(r), n = 0..nmax: -s^l (1+s^(1/alpha))^(-alpha(2l+1)) C_n^lambda(xi) / sqrt(N_nl)
    with scipy's C_n^lambda; N_nl in closed form for alpha = 1, else the oracle's
    quadrature norms (pinned against scipy quadrature in test_oracle_basis)."""
    a = B.alpha
    s = r / B.b
    t = s ** (1.0 / a)
    xi = (t - 1.0) / (t + 1.0)
    lam = (2 * l + 1) * a + 0.5
    pref = -s ** l * (1.0 + t) ** (-a * (2 * l + 1))
    N = O.norms(B)
    out = np.empty(B.nmax + 1)
    for n in range(B.nmax + 1):
        Nn = _closed_norm_alpha1(n, l, B.b, B.G) if a == 1.0 else N[n, l]
        out[n] = pref * sp.eval_gegenbauer(n, lam, xi) / math.sqrt(Nn)
    return out


def _sph(x):
    r = math.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
    th = math.acos(x[2] / r)
    ph = math.atan2(x[1], x[0]) % (2 * math.pi)
    return r, th, ph


POINTS = [np.array([0.83, -1.21, 0.47]), np.array([-2.9, 0.35, -1.6]), np.array([0.05, 0.11, -0.09])]
BASES = [(1.0, 1.7, 0.6), (0.5, 1.7, 0.6), (0.8, 1.7, 0.6), (1.0, 1.0, 1.0)]


@pytest.mark.parametrize("alpha,b,G", BASES)
def test_single_particle_coefficients_match_scipy(O, alpha, b, G):
    nmax, lmax = 16, 10
    B = O.basis(nmax, lmax, alpha=alpha, b=b, G=G)
    L2 = (lmax + 1) ** 2
    mass = 0.37
    for x in POINTS:
        r, th, ph = _sph(x)
        c = O.coeffs(B, x[:1], x[1:2], x[2:], np.array([mass]))
        ref = np.zeros_like(c)
        for l in range(lmax + 1):
            U = _U_independent(O, B, l, r)
            for m in range(l + 1):
                Y = complex(sp.sph_harm_y(l, m, th, ph))
                a = -mass * U * np.conj(Y)
                if m == 0:
                    ref[np.arange(nmax + 1) * L2 + l * l] = a.real
                else:
                    ref[np.arange(nmax + 1) * L2 + l * l + 2 * m - 1] = a.real
                    ref[np.arange(nmax + 1) * L2 + l * l + 2 * m] = a.imag
        scale = np.abs(ref).max()
        assert np.abs(c - ref).max() <= 1e-13 * scale
        # per degree as well, so that a small block is not hidden by a_000
        for l in range(lmax + 1):
            idx = np.concatenate([np.arange(nmax + 1) * L2 + l * l + j for j in range(2 * l + 1)])
            bs = np.abs(ref[idx]).max()
            assert np.abs(c[idx] - ref[idx]).max() <= 1e-12 * bs, (l, x)


@pytest.mark.parametrize("alpha,b,G", BASES[:3])
def test_unit_coefficient_potential_matches_scipy(O, alpha, b, G):
    nmax, lmax = 6, 10
    B = O.basis(nmax, lmax, alpha=alpha, b=b, G=G)
    L2 = (lmax + 1) ** 2
    T = O.ncoef(nmax, lmax)
    pts = np.stack(POINTS, axis=1)
    rng = np.random.default_rng(7)
    picks = rng.choice(T, 40, replace=False)
    for t in picks:
        n, rem = divmod(int(t), L2)
        l = int(math.isqrt(rem))
        j = rem - l * l
        e = np.zeros(T)
        e[t] = 1.0
        P, _ = O.field(B, e, *pts, acc=False)
        for k in range(pts.shape[1]):
            r, th, ph = _sph(pts[:, k])
            U = _U_independent(O, B, l, r)[n]
            if j == 0:
                ref = U * sp.sph_harm_y(l, 0, th, ph).real
            else:
                m = (j + 1) // 2
                Y = complex(sp.sph_harm_y(l, m, th, ph))
                ref = 2 * U * Y.real if j % 2 == 1 else -2 * U * Y.imag
            assert P[k] == pytest.approx(ref, rel=1e-12, abs=1e-14 * abs(U)), (n, l, j, k)


def test_unit_coefficient_force_matches_scipy_gradient(O):
    # -grad of the independent psi (central differences) for a few l > 0 terms
    nmax, lmax = 4, 6
    B = O.basis(nmax, lmax, alpha=0.8, b=1.7, G=0.6)
    L2 = (lmax + 1) ** 2
    T = O.ncoef(nmax, lmax)

    def psi_ref(t, x):
        n, rem = divmod(t, L2)
        l = int(math.isqrt(rem))
        j = rem - l * l
        r, th, ph = _sph(x)
        U = _U_independent(O, B, l, r)[n]
        if j == 0:
            return U * sp.sph_harm_y(l, 0, th, ph).real
        m = (j + 1) // 2
        Y = complex(sp.sph_harm_y(l, m, th, ph))
        return 2 * U * Y.real if j % 2 == 1 else -2 * U * Y.imag

    x = POINTS[0]
    h = 1e-5
    for t in (3 * L2 + 4 + 2, 1 * L2 + 25 + 7, 2 * L2 + 9 + 4, 4 * L2 + 36 + 12):
        e = np.zeros(T)
        e[t] = 1.0
        _, g = O.field(B, e, x[:1], x[1:2], x[2:])
        fd = np.array([-(psi_ref(t, x + h * d) - psi_ref(t, x - h * d)) / (2 * h) for d in np.eye(3)])
        assert np.allclose(g[:, 0], fd, rtol=1e-7, atol=1e-9 * np.abs(fd).max())


def test_monte_carlo_error_slope(O):
    # RMS of a_000 - 1/sqrt(3) over seeds at N = 1e4, 1e5, 1e6; Hernquist
    # particles, alpha = 1 basis.  Var of one particle's term is 1/6.
    B = O.basis(0, 0)
    exact = 1.0 / math.sqrt(3.0)
    sizes = (10_000, 100_000, 1_000_000)
    seeds = {10_000: 256, 100_000: 256, 1_000_000: 64}
    rms = []
    for n in sizes:
        errs = []
        for s in range(seeds[n]):
            p = I.hernquist(n, 500_000 + 1000 * int(math.log10(n)) + s)
            errs.append(O.coeffs(B, *p.pos, p.mass)[0] - exact)
        errs = np.asarray(errs)
        rms.append(math.sqrt((errs ** 2).mean()))
        sigma = math.sqrt(1.0 / 6.0 / n)
        # chi-square with K degrees of freedom: the mean square lies within
        # a few sqrt(2/K) of sigma^2; a biased estimator fails this at 1e6
        K = len(errs)
        assert abs(rms[-1] ** 2 / sigma ** 2 - 1.0) < 4.0 * math.sqrt(2.0 / K), (n, rms[-1], sigma)
        assert abs(errs.mean()) < 4.0 * sigma / math.sqrt(K), (n, errs.mean())
    slope = np.polyfit(np.log10(sizes), np.log10(rms), 1)[0]
    assert abs(slope + 0.5) <= 0.05, slope
