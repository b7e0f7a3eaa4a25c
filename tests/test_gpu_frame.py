"""GPU parity of the frame-centre search (Sec. 2.1) and of the refresh
cadence with recentring, against the FP64 oracle."""
import numpy as np
import pytest

from oracle import cadence as K
from oracle import frame as F
from paper_2602_13385_amd import inputs as I

pytestmark = pytest.mark.gpu

LOG_HOST = [("log", (1.5, 1.0, 0.0))]


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


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("alpha,profile", [(1.0, "hernquist"), (0.5, "plummer")])
def test_recentre_matches_oracle(torch, S, O, dtype, alpha, profile):
    print(f"[frame] recentre {dtype} alpha={alpha}", flush=True)
    p = I.hernquist(20000, 81) if profile == "hernquist" else I.plummer(20000, 81)
    pos = _rounded(p.pos + np.array([[0.05], [0.02], [-0.03]]), dtype)
    w = _rounded(np.where(np.arange(p.n) % 9 == 2, 0.0, p.mass), dtype)
    B = O.basis(6, 2, alpha=alpha)
    c_ref, it_ref = F.recentre(B, pos, w, tol=1e-8, maxit=200)
    plan = S.Plan(6, 2, alpha=alpha, dtype=dtype)
    c, it = plan.recentre(*[_dev(torch, pos[i], dtype) for i in range(3)], _dev(torch, w, dtype),
                          tol=1e-8, maxit=200)
    assert it == it_ref
    assert np.abs(c - c_ref).max() <= 1e-10
    # from a given start, a fixed number of steps
    c5, it5 = plan.recentre(*[_dev(torch, pos[i], dtype) for i in range(3)], _dev(torch, w, dtype),
                            centre=(0.1, 0.0, 0.0), tol=0.0, maxit=5)
    c5_ref, _ = F.recentre(B, pos, w, c0=(0.1, 0.0, 0.0), tol=0.0, maxit=5)
    assert it5 == 5 and np.abs(c5 - c5_ref).max() <= 1e-10


def test_evolve_with_recentre_matches_oracle(torch, S, O):
    """Plummer (N = 2000) offset from the frame origin and drifting, at R = 20
    in the logarithmic host; complete refresh every 2nd interval with
    recentring: frame shifts, state, centre and coefficients (FP64)."""
    p = I.plummer(2000, 83)
    st0 = p.state()
    st0[:3] += np.array([[0.2], [-0.1], [0.05]])
    st0[3:] += np.array([[0.05], [0.02], [-0.01]])
    m = p.mass
    B = O.basis(10, 6)
    H = O.host([(O.HOST_LOG, (1.5, 1.0, 0.0))])
    cen0 = np.array([20.0, 0.0, 0.0, 0.0, I.LOG_VC_20, 0.0])
    coef0, w0, i0 = K.initial_refresh(B, st0, m, 0.999)
    st_ref, cen_ref, coef_ref, w_ref, cs_ref, log_ref = K.evolve(
        B, H, st0, m, cen0, coef0, w0, 4, eta=1.0 / 400.0, dt_max=0.05, refresh_every=2,
        n_samples_tdyn=8, mbound=i0["mbound"], rhm=i0["rhm"], recentre=True)
    assert np.abs(log_ref[1]["dx"]).max() > 1e-3 and np.abs(log_ref[1]["dv"]).max() > 1e-3
    plan = S.Plan(10, 6, dtype="f64")
    st = [_dev(torch, st0[i], "f64") for i in range(6)]
    md = _dev(torch, m, "f64")
    coef, w, state = plan.cadence_init(st, md, 0.999)
    cad = S.Cadence(eta=1.0 / 400.0, dt_max=0.05, frac=0.999, refresh_every=2, n_samples_tdyn=8,
                    ns_max=8, recentre=True)
    cen, state, log = plan.evolve(st, md, 4, cad, (LOG_HOST, 1.0), cen0, coef, w, state)
    torch.cuda.synchronize()
    for g, r in zip(log, log_ref):
        for k in ("nsub", "nsamples", "kind", "nbound", "nchanged"):
            assert g[k] == r[k], (k, g, r)
        assert np.abs(g["dx"] - r["dx"]).max() <= 1e-10
        assert np.abs(g["dv"] - r["dv"]).max() <= 1e-10
    out = np.stack([t.cpu().numpy() for t in st])
    for rows in (slice(0, 3), slice(3, 6)):
        assert np.abs(out[rows] - st_ref[rows]).max() <= 1e-11 * np.abs(st_ref[rows]).max()
    assert np.abs(cen - cen_ref).max() <= 1e-11 * np.abs(cen_ref).max()
    assert np.abs(coef.cpu().numpy() - coef_ref).max() <= 1e-11 * np.abs(coef_ref).max()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("profile", ["hernquist", "plummer"])
def test_tune_basis_matches_oracle(torch, S, O, dtype, profile):
    """The a_000 maximum over (alpha, b) against the oracle's independent
    optimiser; both resolve the maximum to about 1e-8."""
    print(f"[frame] tune {dtype} {profile}", flush=True)
    p = I.hernquist(20000, 85) if profile == "hernquist" else I.plummer(20000, 85)
    pos = _rounded(p.pos * 1.7, dtype)
    w = _rounded(p.mass, dtype)
    a_ref, b_ref, v_ref = F.tune_basis(pos, w, alpha0=1.0, b0=1.0)
    plan = S.Plan(6, 2, dtype=dtype)
    a, b, v = plan.tune_basis(*[_dev(torch, pos[i], dtype) for i in range(3)], _dev(torch, w, dtype))
    assert abs(a - a_ref) <= 1e-6 and abs(b / b_ref - 1.0) <= 1e-6, (a, a_ref, b, b_ref)
    assert v >= v_ref - 1e-12 * abs(v_ref)
    assert plan.alpha == 1.0 and plan.b == 1.0  # the plan itself is unchanged


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_set_basis_equals_a_new_plan(torch, S, dtype):
    p = I.plummer(8000, 86)
    st = [_dev(torch, p.state()[i], dtype) for i in range(6)]
    m = _dev(torch, p.mass, dtype)
    plan = S.Plan(10, 6, dtype=dtype)
    plan.coeffs(st[0], st[1], st[2], m)
    plan.set_basis(0.7, 1.3)
    assert plan.alpha == 0.7 and plan.b == 1.3
    ref = S.Plan(10, 6, alpha=0.7, b=1.3, dtype=dtype)
    c1 = plan.coeffs(st[0], st[1], st[2], m)
    c2 = ref.coeffs(st[0], st[1], st[2], m)
    assert torch.equal(c1, c2)
    # every field variant (the matrix-core ones read the derivative table
    # that set_basis rebuilds)
    for fv in range(plan.num_field_variants):
        plan.field_variant = fv
        ref.field_variant = fv
        a1 = plan.forces(st[0], st[1], st[2], c1)
        a2 = ref.forces(st[0], st[1], st[2], c2)
        assert all(torch.equal(u, v) for u, v in zip(a1, a2)), fv


def test_evolve_with_retune_matches_oracle(torch, S, O):
    """Plummer (N = 2000) in the logarithmic host, starting from the
    alpha = 1, b = 1 basis, with recentring and retuning at every 2nd
    interval (FP64).  The two optimisers agree to about 1e-8 in (alpha, b),
    which bounds the agreement of the runs; they are compared at 1e-5."""
    p = I.plummer(2000, 87)
    st0 = p.state()
    st0[:3] += np.array([[0.1], [0.0], [-0.05]])
    m = p.mass
    B = O.basis(10, 6)
    H = O.host([(O.HOST_LOG, (1.5, 1.0, 0.0))])
    cen0 = np.array([20.0, 0.0, 0.0, 0.0, I.LOG_VC_20, 0.0])
    coef0, w0, i0 = K.initial_refresh(B, st0, m, 0.999)
    st_ref, cen_ref, coef_ref, w_ref, cs_ref, log_ref, B_ref = K.evolve(
        B, H, st0, m, cen0, coef0, w0, 4, eta=1.0 / 400.0, dt_max=0.05, refresh_every=2,
        mbound=i0["mbound"], rhm=i0["rhm"], recentre=True, retune=True)
    assert abs(B_ref.alpha - 1.0) > 1e-2  # the basis really moved
    plan = S.Plan(10, 6, dtype="f64")
    st = [_dev(torch, st0[i], "f64") for i in range(6)]
    md = _dev(torch, m, "f64")
    coef, w, state = plan.cadence_init(st, md, 0.999)
    cad = S.Cadence(eta=1.0 / 400.0, dt_max=0.05, frac=0.999, refresh_every=2, recentre=True,
                    retune=True)
    cen, state, log = plan.evolve(st, md, 4, cad, (LOG_HOST, 1.0), cen0, coef, w, state)
    torch.cuda.synchronize()
    for g, r in zip(log, log_ref):
        for k in ("nsub", "kind", "nbound", "nchanged"):
            assert g[k] == r[k], (k, g, r)
        assert abs(g["alpha"] - r["alpha"]) <= 1e-6 and abs(g["b"] / r["b"] - 1.0) <= 1e-6
    assert abs(plan.alpha - B_ref.alpha) <= 1e-6
    out = np.stack([t.cpu().numpy() for t in st])
    for rows in (slice(0, 3), slice(3, 6)):
        assert np.abs(out[rows] - st_ref[rows]).max() <= 1e-5 * np.abs(st_ref[rows]).max()
    assert np.abs(coef.cpu().numpy() - coef_ref).max() <= 1e-5 * np.abs(coef_ref).max()
