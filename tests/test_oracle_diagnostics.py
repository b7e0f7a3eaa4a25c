"""Pins of the oracle's diagnostics: the power per degree E_l = sum_{n,m}
|a_nlm|^2 and the Frobenius norm of the host's tidal tensor (Sec. 3.5 and
Fig. power_spectrum_time_series; Sec. 2.2, Eq. tidal_tensor)."""
import math

import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I


def test_power_sums_to_minus_twice_the_potential_energy(O):
    # W = 1/2 sum_k m_k psi(x_k) = -1/2 sum_{nlm} |a_nlm|^2 = -1/2 sum_l E_l
    p = I.plummer(3000, 71)
    pos = p.pos * np.array([[1.0], [0.7], [0.4]])
    B = O.basis(8, 6)
    c = O.coeffs(B, *pos, p.mass)
    pot, _ = O.field(B, c, *pos, acc=False)
    W = 0.5 * np.sum(p.mass * pot)
    E = O.power(8, 6, c)
    assert E.sum() == pytest.approx(-2 * W, rel=1e-12)
    assert np.all(E > 0)


def test_power_of_a_spherical_system_is_monopole_only(O):
    q = I.quadrature_sphere("hernquist", 1.0, nr=32, nmu=16, nphi=16)
    B = O.basis(10, 6)
    E = O.power(10, 6, O.coeffs(B, *q.pos, q.mass))
    assert E[0] == pytest.approx(1.0 / 3.0, rel=1e-12)  # a_000 = 1/sqrt(3)
    assert np.abs(E[1:]).max() < 1e-24


def test_power_is_invariant_under_rotations_and_sees_a_quadrupole(O):
    p = I.plummer(2000, 72)
    pos = p.pos * np.array([[1.0], [1.0], [0.5]])  # oblate: l = 2 power dominates l > 0
    B = O.basis(6, 4)
    E1 = O.power(6, 4, O.coeffs(B, *pos, p.mass))
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    E2 = O.power(6, 4, O.coeffs(B, *(Q @ pos), p.mass))
    assert np.allclose(E1, E2, rtol=1e-11, atol=0)
    assert E1[2] > 10 * max(E1[1], E1[3])


@pytest.mark.parametrize("kind,params", [("hernquist", (3.0, 1.3)), ("nfw", (100.0, 15.0)),
                                         ("plummer", (2.0, 0.7)), ("log", (1.5, 1.0))])
def test_tidal_norm_of_a_spherical_host(O, kind, params):
    # for psi(r): ||T||^2 = psi''^2 + 2 (psi'/r)^2; psi', psi'' by central differences
    kinds = {"hernquist": O.HOST_HERNQUIST, "nfw": O.HOST_NFW, "plummer": O.HOST_PLUMMER,
             "log": O.HOST_LOG}
    H = O.host([(kinds[kind], params)])
    r = 2.3
    u = np.array([0.48, -0.6, 0.64])
    u /= np.linalg.norm(u)

    def psi(rr):
        return O.host_eval(H, rr * u)[0]
    h = 1e-3
    d1 = (psi(r + h) - psi(r - h)) / (2 * h)
    d2 = (psi(r + h) - 2 * psi(r) + psi(r - h)) / (h * h)
    ref = math.sqrt(d2 ** 2 + 2 * (d1 / r) ** 2)
    assert O.tidal_norm(H, r * u) == pytest.approx(ref, rel=1e-5)
