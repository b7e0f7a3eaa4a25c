"""GPU parity of the SCF density (Eq. total_dens) and the frame core
(Sec. 2.1) against the FP64 oracle.

The density weights the potential's terms by K_nl, which grows like n^2, so
its FP32 rounding is larger relative to the result than the potential's (up
to 2e-6 here); the bar is the FP32 bar of the other fields, in their metric
(max |d rho| / (|rho| + median |rho|)).
"""
import math

import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I

pytestmark = pytest.mark.gpu

RHO_TOL = {"f32": 1e-5, "f64": 1e-11}


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def S():
    from paper_2602_13385_amd import scf
    scf.lib()
    return scf


def _rounded(arr, dtype):
    a = np.asarray(arr, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if dtype == "f32" else a


def _dev(torch, arr, dtype):
    td = torch.float32 if dtype == "f32" else torch.float64
    return torch.as_tensor(np.ascontiguousarray(arr), dtype=td, device="cuda")


def _err(g, ref):
    return (np.abs(g - ref) / (np.abs(ref) + np.median(np.abs(ref)))).max()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("nmax,lmax,alpha", [(10, 6, 1.0), (16, 10, 1.0), (6, 4, 0.5), (10, 6, 0.8)])
def test_density_matches_oracle(torch, S, O, dtype, nmax, lmax, alpha):
    print(f"[density] {dtype} n{nmax} l{lmax} alpha={alpha}", flush=True)
    p = I.plummer(20000, 61) if alpha != 1.0 else I.hernquist(20000, 61)
    st = _rounded(p.state(), dtype)
    m = _rounded(p.mass, dtype)
    B = O.basis(nmax, lmax, alpha=alpha)
    coef = O.coeffs(B, *st[:3], m)
    pts = _rounded(I.uniform_ball(3001, 62, radius=6.0).pos, dtype)
    ref = O.density(B, coef, *pts)
    plan = S.Plan(nmax, lmax, alpha=alpha, dtype=dtype)
    c = torch.as_tensor(coef, dtype=torch.float64, device="cuda")
    rho = plan.density(*[_dev(torch, pts[i], dtype) for i in range(3)], c)
    torch.cuda.synchronize()
    e = _err(rho.cpu().numpy().astype(np.float64), ref)
    print(f"    density error {e:.2e}", flush=True)
    assert e <= RHO_TOL[dtype], e


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_density_of_hernquist_quadrature_closed_form(torch, S, O, dtype):
    q = I.quadrature_sphere("hernquist", 1.0, nr=40, nmu=24, nphi=24)
    B = O.basis(16, 10)
    coef = O.coeffs(B, *q.pos, q.mass)
    pts = _rounded(I.uniform_ball(2000, 63, radius=8.0).pos, dtype)
    r = np.sqrt((pts ** 2).sum(0))
    plan = S.Plan(16, 10, dtype=dtype)
    c = torch.as_tensor(coef, dtype=torch.float64, device="cuda")
    rho = plan.density(*[_dev(torch, pts[i], dtype) for i in range(3)], c).cpu().numpy()
    exact = 1.0 / (2 * math.pi * r * (1 + r) ** 3)
    assert _err(rho.astype(np.float64), exact) <= (1e-5 if dtype == "f32" else 1e-10)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_core_matches_oracle(torch, S, O, dtype):
    p = I.plummer(30000, 64)
    st0 = _rounded(p.state(), dtype)
    st0[3:] += np.array([[0.3], [-0.1], [0.05]])  # a bulk motion for the core to find
    st0 = _rounded(st0, dtype)
    m = _rounded(p.mass, dtype)
    w = np.where(np.arange(p.n) % 11 == 5, 0.0, m)
    B = O.basis(10, 6)
    coef = O.coeffs(B, *st0[:3], w)
    rc, v, mc = O.core(B, coef, st0, m, w)
    r2 = (st0[:3] ** 2).sum(0)
    sel = w > 0
    # no selected particle within rounding of the core boundary
    assert np.abs(r2[sel] / (rc * rc) - 1.0).min() > 1e-5
    plan = S.Plan(10, 6, dtype=dtype)
    c = torch.as_tensor(coef, dtype=torch.float64, device="cuda")
    rc_g, v_g, mc_g = plan.core([_dev(torch, st0[i], dtype) for i in range(6)], _dev(torch, m, dtype),
                                _dev(torch, w, dtype), c)
    tol = 1e-5 if dtype == "f32" else 1e-11
    assert rc_g == pytest.approx(rc, rel=tol)
    assert mc_g == pytest.approx(mc, rel=1e-12)
    assert np.abs(v_g - v).max() <= 1e-12 * np.abs(v).max() + 1e-14
    # nothing selected: all zero
    z = _dev(torch, np.zeros(p.n), dtype)
    assert plan.core([_dev(torch, st0[i], dtype) for i in range(6)], _dev(torch, m, dtype), z, c)[2] == 0.0
