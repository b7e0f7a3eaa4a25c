"""Pins of the SCF density (Eq. total_dens) and the frame's core velocity
(Sec. 2.1) in the oracle.

* The density basis is defined by Poisson's equation, nabla^2 psi^(nlm) =
  4 pi G rho^(nlm): for random coefficients the oracle's rho_SCF equals the
  Laplacian of its psi_SCF taken by Richardson-extrapolated central
  differences.
* Quadrature particles of a Hernquist sphere (alpha = 1) and a Plummer sphere
  (alpha = 1/2) give the closed-form densities M a / (2 pi r (r + a)^3) and
  3 M / (4 pi a^3) (1 + r^2/a^2)^(-5/2).
* r_core and the core velocity against their definitions on a hand-made set.
"""
import math

import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I


def _laplacian(O, B, coef, pts, h):
    def pot(p):
        P, _ = O.field(B, coef, p[0], p[1], p[2], acc=False)
        return P
    lap = -6.0 * pot(pts)
    for d in range(3):
        e = np.zeros((3, 1))
        e[d] = h
        lap = lap + pot(pts + e) + pot(pts - e)
    return lap / (h * h)


@pytest.mark.parametrize("alpha,b,G", [(1.0, 1.0, 1.0), (0.5, 2.0, 1.0), (0.8, 1.5, 0.7)])
def test_density_is_the_laplacian_of_the_potential(O, alpha, b, G):
    B = O.basis(5, 3, alpha=alpha, b=b, G=G)
    rng = np.random.default_rng(17)
    coef = rng.normal(size=O.ncoef(5, 3)) / (1.0 + np.arange(O.ncoef(5, 3)) % 16)
    pts = I.uniform_ball(40, 8, radius=4.0 * b).pos
    pts = pts[:, np.sqrt((pts ** 2).sum(0)) > 0.3 * b]
    h = 2e-3 * b
    # Richardson: (4 L(h/2) - L(h)) / 3 removes the h^2 term
    lap = (4.0 * _laplacian(O, B, coef, pts, h / 2) - _laplacian(O, B, coef, pts, h)) / 3.0
    rho = O.density(B, coef, *pts)
    ref = lap / (4.0 * math.pi * G)
    assert np.abs(rho - ref).max() <= 2e-6 * np.abs(ref).max()


def test_density_of_quadrature_spheres(O):
    pts = I.uniform_ball(200, 12, radius=6.0).pos
    r = np.sqrt((pts ** 2).sum(0))
    B = O.basis(8, 4)
    q = I.quadrature_sphere("hernquist", 1.0, nr=32, nmu=16, nphi=16)
    c = O.coeffs(B, *q.pos, q.mass)
    np.testing.assert_allclose(O.density(B, c, *pts), 1.0 / (2 * math.pi * r * (1 + r) ** 3),
                               rtol=1e-10)
    B2 = O.basis(8, 4, alpha=0.5)
    q2 = I.quadrature_sphere("plummer", 0.5, nr=32, nmu=16, nphi=16)
    c2 = O.coeffs(B2, *q2.pos, q2.mass)
    np.testing.assert_allclose(O.density(B2, c2, *pts),
                               3.0 / (4 * math.pi) * (1 + r * r) ** -2.5, rtol=1e-10)


def test_core_radius_and_velocity_definitions(O):
    """Hernquist potential (quadrature coefficients): rho is known, so r_core
    and the core's mean velocity follow from their definitions directly."""
    B = O.basis(6, 2)
    q = I.quadrature_sphere("hernquist", 1.0, nr=24, nmu=8, nphi=8)
    c = O.coeffs(B, *q.pos, q.mass)
    p = I.uniform_ball(500, 21, radius=5.0)
    m = p.mass
    w = np.where(np.arange(p.n) % 7 == 3, 0.0, m)
    r = np.sqrt((p.pos ** 2).sum(0))
    rho = 1.0 / (2 * math.pi * r * (1 + r) ** 3)
    sel = w > 0
    rc = math.sqrt((rho[sel] ** 2 * r[sel] ** 2).sum() / (rho[sel] ** 2).sum())
    inc = sel & (r <= rc)
    v = (p.vel[:, inc] * m[inc]).sum(1) / m[inc].sum()
    rc_o, v_o, mc = O.core(B, c, np.concatenate([p.pos, p.vel]), m, w)
    assert rc_o == pytest.approx(rc, rel=1e-9)
    np.testing.assert_allclose(v_o, v, rtol=1e-9, atol=1e-12)
    assert mc == pytest.approx(m[inc].sum(), rel=1e-12)
