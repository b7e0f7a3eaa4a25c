"""The identity behind the matrix-core field pass, checked on the CPU.

That pass forms the xi-derivative sums sum_n W_n p_n'(xi) as sums over the
basis itself, sum_k W'_k p_k(xi), for the monic Gegenbauer polynomials
p_n = C_n^lam / kappa_n (kappa_n = 2^n (lam)_n / n!, the leading coefficient):

  p_n' = sum_{k = n-1, n-3, ...} D_nk p_k,   D_nk = 2 (k + lam) kappa_k / kappa_n,
  W'_k = sum_n D_nk W_n = 2 (k + lam) kappa_k S_k,
  S_k = W_{k+1} / kappa_{k+1} + S_{k+2}.

Here both sides come from independent constructions: the polynomials and
their derivatives from scipy's Gegenbauer coefficients with numpy's
polynomial calculus, and the suffix recurrence against the plain double sum.
(The GPU parity tests check the kernels that use it against the oracle.)
"""
import math

import numpy as np
import pytest
import scipy.special as sp
from numpy.polynomial import polynomial as P


def _kappa(n, lam):
    # leading coefficient of C_n^lam: 2^n Gamma(lam + n) / (Gamma(lam) n!)
    return math.exp(n * math.log(2.0) + math.lgamma(lam + n) - math.lgamma(lam)
                    - math.lgamma(n + 1))


def _monic(n, lam):
    """Monomial coefficients (lowest first) of C_n^lam / kappa_n, from scipy."""
    c = np.asarray(sp.gegenbauer(n, lam).coeffs, dtype=np.float64)[::-1]
    return c / c[-1]


# lam = (2 l + 1) alpha + 1/2 for the degrees and alphas the plans use
LAMS = [1.5, 3.5, 21.5, 1.0, 5.5, (2 * 4 + 1) * 0.8 + 0.5]


@pytest.mark.parametrize("lam", LAMS)
def test_leading_coefficient(lam):
    for n in range(0, 13):
        c = np.asarray(sp.gegenbauer(n, lam).coeffs, dtype=np.float64)
        assert c[0] == pytest.approx(_kappa(n, lam), rel=1e-10)


@pytest.mark.parametrize("lam", LAMS)
def test_derivative_in_the_same_basis(lam):
    xs = np.linspace(-0.98, 0.98, 23)
    for n in range(1, 13):
        lhs = P.polyval(xs, P.polyder(_monic(n, lam)))
        rhs = np.zeros_like(xs)
        for k in range(n - 1, -1, -2):
            rhs += 2.0 * (k + lam) * _kappa(k, lam) / _kappa(n, lam) * P.polyval(xs, _monic(k, lam))
        scale = np.abs(lhs).max() + 1e-300
        assert np.abs(lhs - rhs).max() <= 1e-9 * scale, (lam, n)


@pytest.mark.parametrize("lam", LAMS)
def test_suffix_recurrence_equals_the_double_sum(lam):
    rng = np.random.default_rng(int(lam * 100))
    nmax = 16
    W = rng.normal(size=nmax + 1)
    kap = [_kappa(n, lam) for n in range(nmax + 1)]
    direct = np.array([sum(2.0 * (k + lam) * kap[k] / kap[n] * W[n]
                           for n in range(k + 1, nmax + 1, 2)) for k in range(nmax + 1)])
    s1 = s2 = 0.0  # S_{k+1}, S_{k+2}
    rec = np.zeros(nmax + 1)
    for k in range(nmax, -1, -1):
        v = W[k + 1] / kap[k + 1] if k < nmax else 0.0
        sk = v + s2
        s2, s1 = s1, sk
        rec[k] = 2.0 * (k + lam) * kap[k] * sk
    assert np.allclose(rec, direct, rtol=1e-12, atol=1e-12 * np.abs(direct).max())
    assert rec[nmax] == 0.0  # the top polynomial has no higher term to feed its derivative


def test_derivative_sums_match_for_a_weight_vector():
    """sum_n W_n p_n'(xi) == sum_k W'_k p_k(xi) at lam = 21.5 (l = 10, alpha = 1)."""
    lam, nmax = 21.5, 16
    rng = np.random.default_rng(7)
    W = rng.normal(size=nmax + 1)
    kap = [_kappa(n, lam) for n in range(nmax + 1)]
    Wd = np.array([sum(2.0 * (k + lam) * kap[k] / kap[n] * W[n]
                       for n in range(k + 1, nmax + 1, 2)) for k in range(nmax + 1)])
    xs = np.linspace(-0.95, 0.95, 17)
    lhs = sum(W[n] * P.polyval(xs, P.polyder(_monic(n, lam))) for n in range(1, nmax + 1))
    rhs = sum(Wd[k] * P.polyval(xs, _monic(k, lam)) for k in range(nmax + 1))
    assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(lhs).max()
