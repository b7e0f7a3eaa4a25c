"""Pin of the oracle's discrete adjoint against central finite differences of
the forward oracle (a separate code path: the forward step never calls the
adjoint's Hessian or vector-Jacobian routines)."""
import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I


def _setup(O, n=200, nsteps=8):
    p = I.plummer(n, 51)
    B = O.basis(4, 3)
    H = O.host([(O.HOST_NFW, (232.98, 20.0))])
    cen = np.array([20.0, 0.0, 0.0, 0.1, 1.4, 0.3])
    rng = np.random.default_rng(2)
    w_state = rng.normal(size=(6, n))
    w_cen = rng.normal(size=6)
    return p, B, H, cen, w_state, w_cen, nsteps


def _loss(O, B, H, st0, m, cen, dt, nsteps, w_state, w_cen):
    st, c1, _ = O.step(B, H, st0, m, cen, dt, nsteps)
    return (w_state * st).sum() + (w_cen * c1).sum()


def test_adjoint_matches_finite_differences(O):
    p, B, H, cen, ws, wc, nsteps = _setup(O)
    dt = 0.01
    lam0, lc0, gh = O.step_adjoint(B, H, p.state(), p.mass, cen, dt, nsteps, ws, wc)

    def fd(fun, h):
        return (fun(h) - fun(-h)) / (2 * h)

    # host parameters
    for k, h in ((0, 1e-3), (1, 1e-4)):
        def f(eps, k=k):
            Hc = O.host([(O.HOST_NFW, (232.98 + (eps if k == 0 else 0), 20.0 + (eps if k == 1 else 0)))])
            return _loss(O, B, Hc, p.state(), p.mass, cen, dt, nsteps, ws, wc)
        assert gh[0, k] == pytest.approx(fd(f, h), rel=1e-6, abs=1e-9)
    # centre initial conditions
    for k in range(6):
        def f(eps, k=k):
            c = cen.copy()
            c[k] += eps
            return _loss(O, B, H, p.state(), p.mass, c, dt, nsteps, ws, wc)
        assert lc0[k] == pytest.approx(fd(f, 1e-5), rel=1e-6, abs=1e-8)
    # a few particle initial conditions
    for (row, i) in ((0, 3), (2, 17), (4, 101), (5, 5)):
        def f(eps, row=row, i=i):
            st = p.state().copy()
            st[row, i] += eps
            return _loss(O, B, H, st, p.mass, cen, dt, nsteps, ws, wc)
        assert lam0[row, i] == pytest.approx(fd(f, 1e-5), rel=1e-6, abs=1e-8)


def test_adjoint_zero_steps_is_identity(O):
    p, B, H, cen, ws, wc, _ = _setup(O, n=50)
    lam0, lc0, gh = O.step_adjoint(B, H, p.state(), p.mass, cen, 0.01, 0, ws, wc)
    assert np.array_equal(lam0, ws) and np.array_equal(lc0, wc) and (gh == 0).all()
