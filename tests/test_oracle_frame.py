"""Pins of the frame-centre search (Sec. 2.1) in the oracle.

* A smooth kernel (alpha = 1/2): the fixed point equals the maximum of
  a_000(c) found by an independent optimiser (scipy's Nelder-Mead on the
  objective itself).
* A quadrature sphere shifted by a known vector: the maximum sits at the
  shift, by symmetry.
* alpha = 1 (a cusp at every particle): the result is a local maximum of
  a_000 at the scale of 1e-3, and the iteration never lowers a_000.
* The basis parameters: the closed-form energy norm of the zeroth mode equals
  the oracle's quadrature of it; the potential of a Hernquist sphere is the
  alpha = 1 zeroth mode and that of a Plummer sphere the alpha = 1/2 one, so
  a_000 is largest there (b = their scale radius); scaling the positions
  scales b.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import frame as F
from paper_2602_13385_amd import inputs as I


def test_smooth_kernel_matches_an_independent_optimiser(O):
    B = O.basis(6, 2, alpha=0.5, b=1.3)
    p = I.plummer(4000, 71)
    pos = p.pos + np.array([[0.4], [-0.2], [0.1]])
    w = p.mass
    c, it = F.recentre(B, pos, w, tol=1e-12, maxit=2000)
    res = minimize(lambda c: -F.a000_about(B, pos, w, c), np.zeros(3), method="Nelder-Mead",
                   options={"xatol": 1e-10, "fatol": 1e-16, "maxiter": 20000})
    assert np.abs(c - res.x).max() <= 1e-6
    assert F.a000_about(B, pos, w, c) >= -res.fun - 1e-14


@pytest.mark.parametrize("alpha,profile", [(1.0, "hernquist"), (0.5, "plummer")])
def test_shifted_quadrature_sphere(O, alpha, profile):
    B = O.basis(4, 2, alpha=alpha)
    q = I.quadrature_sphere(profile, alpha, nr=24, nmu=12, nphi=12)
    shift = np.array([0.3, -0.7, 0.25])
    c, _ = F.recentre(B, q.pos + shift[:, None], q.mass, tol=1e-13, maxit=5000)
    assert np.abs(c - shift).max() <= 1e-9


def test_cusped_kernel_local_maximum_and_ascent(O):
    B = O.basis(6, 2)
    p = I.hernquist(20000, 72)
    pos = p.pos + np.array([[0.05], [0.02], [-0.03]])
    w = p.mass
    c0 = np.zeros(3)
    vals = [F.a000_about(B, pos, w, c0)]
    c = c0
    for _ in range(30):
        c, _ = F.recentre(B, pos, w, c0=c, tol=0.0, maxit=1)
        vals.append(F.a000_about(B, pos, w, c))
    assert all(b >= a - 1e-15 for a, b in zip(vals, vals[1:]))
    c, it = F.recentre(B, pos, w)
    g0 = F.a000_about(B, pos, w, c)
    for e in np.vstack([np.eye(3), -np.eye(3)]):
        assert F.a000_about(B, pos, w, c + 1e-3 * e) <= g0


@pytest.mark.parametrize("alpha,b,G", [(1.0, 1.0, 1.0), (0.5, 1.0, 1.0), (0.8, 1.7, 0.6)])
def test_zeroth_mode_norm_closed_form(O, alpha, b, G):
    B = O.basis(1, 0, alpha=alpha, b=b, G=G)
    assert F.n00(alpha, b, G) == pytest.approx(O.norms(B)[0], rel=1e-10)
    q = I.quadrature_sphere("hernquist", 1.0, nr=24, nmu=8, nphi=8)
    assert F.a000_basis(q.pos, q.mass, alpha, b, G) == pytest.approx(
        O.coeffs(B, *q.pos, q.mass)[0], rel=1e-12)


@pytest.mark.parametrize("profile,alpha_true", [("hernquist", 1.0), ("plummer", 0.5)])
def test_tuned_basis_of_exact_profiles(O, profile, alpha_true):
    q = I.quadrature_sphere(profile, alpha_true, nr=40, nmu=8, nphi=8, a=1.0)
    for scale in (1.0, 2.5):
        a, b, _ = F.tune_basis(q.pos * scale, q.mass, alpha0=0.7, b0=0.8)
        assert a == pytest.approx(alpha_true, abs=1e-6)
        assert b == pytest.approx(scale, rel=1e-6)
