"""GPU checks of scf_step_adjoint and the checkpointed autograd wrapper.

  * against the FP64 oracle's exact discrete adjoint of the same leapfrog map
    (same FP32-representable inputs): FP64 to 1e-9, FP32 to the gradient bar
    1e-3 (componentwise for the host-parameter and centre gradients);
  * against central finite differences of the GPU's own FP64 forward map,
    through the torch.autograd.Function with recomputation from checkpoints;
  * checkpointed and single-segment backward passes agree.
"""
import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I

pytestmark = pytest.mark.gpu

NFW = [("nfw", (232.98, 20.0))]
CEN = np.array([20.0, 0.0, 0.0, 0.1, 1.4, 0.3])


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


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# fv: the plan's field variant (3 = the matrix-core field pass of FP32 plans,
# which the segment's forward recompute uses; 5 in FP32 and 3 in FP64 = the
# degrees of each particle split over 4 waves, in the forward recompute and
# the accumulation pass)
@pytest.mark.parametrize("dtype,host,fv", [("f64", True, 0), ("f32", True, 0), ("f64", False, 0),
                                           ("f32", False, 0), ("f32", True, 3), ("f32", True, 5),
                                           ("f64", True, 3)])
def test_adjoint_matches_oracle(torch, S, O, dtype, host, fv):
    n, nmax, lmax, dt, nsteps = 3000, 10, 6, 0.005, 4
    print(f"[adjoint parity] {dtype} host={host} field variant {fv}", flush=True)
    p = I.plummer(n, 5501)
    st0 = _rounded(p.state(), dtype)
    m = _rounded(p.mass, dtype)
    rng = np.random.default_rng(5502)
    lam = _rounded(rng.normal(size=(6, n)), dtype)
    lamc = rng.normal(size=6)
    B = O.basis(nmax, lmax)
    Ho = O.host([(O.HOST_NFW, NFW[0][1])]) if host else None
    cen = CEN if host else np.zeros(6)
    lam_ref, lc_ref, gh_ref = O.step_adjoint(B, Ho, st0, m, cen, dt, nsteps, lam, lamc)
    plan = S.Plan(nmax, lmax, dtype=dtype)
    plan.field_variant = fv
    st = [_dev(torch, st0[i], dtype) for i in range(6)]
    lt = [_dev(torch, lam[i], dtype) for i in range(6)]
    lc, gh = plan.step_adjoint(st, _dev(torch, m, dtype), dt, nsteps, lt, lamc,
                               host=(NFW, 1.0) if host else None, centre0=cen)
    torch.cuda.synchronize()
    lg = np.stack([t.cpu().numpy() for t in lt]).astype(np.float64)
    # the state is not modified
    assert np.array_equal(np.stack([t.cpu().numpy() for t in st]).astype(np.float64), st0)
    tol = 1e-9 if dtype == "f64" else 1e-3
    assert _rel(lg[:3], lam_ref[:3]) <= tol, _rel(lg[:3], lam_ref[:3])
    assert _rel(lg[3:], lam_ref[3:]) <= tol, _rel(lg[3:], lam_ref[3:])
    for q in range(6):
        assert abs(lc[q] - lc_ref[q]) <= tol * max(abs(lc_ref[q]), 1e-6 * np.abs(lc_ref).max()), q
    if host:
        assert gh.shape == (1, 3)
        for k in range(2):
            assert abs(gh[0, k] - gh_ref[0, k]) <= tol * abs(gh_ref[0, k]), (k, gh, gh_ref)


def test_adjoint_zero_steps_is_identity(torch, S):
    p = I.plummer(500, 5503)
    plan = S.Plan(6, 4, dtype="f64")
    st = [_dev(torch, p.state()[i], "f64") for i in range(6)]
    lam = [torch.randn(500, dtype=torch.float64, device="cuda") for _ in range(6)]
    ref = [t.clone() for t in lam]
    lc, gh = plan.step_adjoint(st, _dev(torch, p.mass, "f64"), 0.01, 0, lam, np.arange(6.0),
                               host=(NFW, 1.0), centre0=CEN)
    assert np.array_equal(lc, np.arange(6.0))
    assert np.all(gh == 0.0)
    for a, b in zip(lam, ref):
        assert torch.equal(a, b)


def _functional(torch, n, seed):
    rng = np.random.default_rng(seed)
    w = torch.as_tensor(rng.normal(size=(6, n)), dtype=torch.float64, device="cuda")
    c = torch.as_tensor(rng.normal(size=6), dtype=torch.float64)
    return w, c


def test_autograd_checkpoints_match_finite_differences(torch, S):
    from paper_2602_13385_amd import adjoint as A
    n, dt, nsteps = 2000, 0.005, 5
    p = I.plummer(n, 5504)
    plan = S.Plan(10, 6, dtype="f64")
    m = _dev(torch, p.mass, "f64")
    st0 = _dev(torch, p.state(), "f64")
    w, c = _functional(torch, n, 5505)

    def loss(theta, cen0, checkpoint=2, grad=False):
        s0 = st0.clone().requires_grad_(grad)
        sT, cT = A.trajectory(plan, s0, m, theta, cen0, ["nfw"], dt, nsteps, checkpoint)
        return (w * sT).sum() + (c * cT).sum(), s0

    theta = torch.tensor([[232.98, 20.0, 0.0]], dtype=torch.float64, requires_grad=True)
    cen0 = torch.tensor(CEN, dtype=torch.float64, requires_grad=True)
    L, s0 = loss(theta, cen0, grad=True)
    L.backward()
    g_theta = theta.grad.numpy().copy()
    g_cen = cen0.grad.numpy().copy()
    g_s0 = s0.grad.detach().cpu().numpy()
    # single segment gives the same gradient
    theta2 = theta.detach().clone().requires_grad_(True)
    cen2 = cen0.detach().clone().requires_grad_(True)
    L2, _ = loss(theta2, cen2, checkpoint=nsteps)
    L2.backward()
    assert np.abs(theta2.grad.numpy() - g_theta).max() <= 1e-10 * np.abs(g_theta).max()
    assert np.abs(cen2.grad.numpy() - g_cen).max() <= 1e-10 * np.abs(g_cen).max()
    # central differences of the FP64 forward map
    with torch.no_grad():
        def Lnum(th, ce):
            return float(loss(th, ce)[0])
        for k, hrel in ((0, 1e-6), (1, 1e-6)):
            h = hrel * abs(float(theta[0, k]))
            tp, tm = theta.detach().clone(), theta.detach().clone()
            tp[0, k] += h
            tm[0, k] -= h
            fd = (Lnum(tp, cen0.detach()) - Lnum(tm, cen0.detach())) / (2 * h)
            assert abs(fd - g_theta[0, k]) <= 1e-5 * abs(g_theta[0, k]) + 1e-9, (k, fd, g_theta)
        for q in range(6):
            h = 1e-5
            cp, cm = cen0.detach().clone(), cen0.detach().clone()
            cp[q] += h
            cm[q] -= h
            fd = (Lnum(theta.detach(), cp) - Lnum(theta.detach(), cm)) / (2 * h)
            assert abs(fd - g_cen[q]) <= 1e-5 * np.abs(g_cen).max(), (q, fd, g_cen)
        # one particle coordinate
        for (row, i) in ((0, 17), (4, 1234)):
            h = 1e-6
            base = st0.clone()
            sp, sm = base.clone(), base.clone()
            sp[row, i] += h
            sm[row, i] -= h

            def Ls(s):
                sT, cT = A.trajectory(plan, s, m, theta.detach(), cen0.detach(), ["nfw"], dt,
                                      nsteps, 2)
                return float((w * sT).sum() + (c * cT).sum())
            fd = (Ls(sp) - Ls(sm)) / (2 * h)
            assert abs(fd - g_s0[row, i]) <= 1e-5 * max(abs(g_s0[row, i]), 1e-3), (row, i, fd)


def test_track_loss_gradient_over_full_horizon(torch, S):
    """The adjoint workload at its own size and horizon (Plummer N = 1e5, NFW
    host, 2000 steps of 0.005, checkpoints every 100): the FP64 adjoint
    gradient of the track loss with respect to (M_s, r_s, R0, V0) against
    FP64 central differences of the same loss (escaper set and nearest track
    points frozen at the FP64 base trajectory), and the FP32 adjoint against
    the FP64 one at the 1e-3 gradient bar, componentwise."""
    from paper_2602_13385_amd import adjoint as A
    w = I.config5()
    p = w.clusters[0]
    H, ck = w.nsteps, w.extra["checkpoint"]
    kinds = [w.host[0][0]]
    theta0 = np.array([list(w.host[0][1])])
    cen0 = np.array(w.centres[0])
    track = w.extra["track"]

    def setup(dtype):
        td = torch.float32 if dtype == "f32" else torch.float64
        return (S.Plan(w.nmax, w.lmax, dtype=dtype), torch.as_tensor(p.mass, dtype=td, device="cuda"),
                torch.as_tensor(p.state(), dtype=td, device="cuda").contiguous())

    def grad(plan, m, s0, mask, idx):
        th = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
        c = torch.tensor(cen0, dtype=torch.float64, requires_grad=True)
        sT, cT = A.trajectory(plan, s0.clone(), m, th, c, kinds, w.dt, H, ck)
        A.track_loss(sT, cT, track, mask, idx).backward()
        return np.concatenate([th.grad.numpy()[0][:2], c.grad.numpy()])

    plan, m, s0 = setup("f64")
    print(f"[adjoint horizon] N={p.n} steps={H}", flush=True)
    with torch.no_grad():
        sT, cT = A.trajectory(plan, s0, m, torch.as_tensor(theta0), torch.as_tensor(cen0), kinds,
                              w.dt, H, ck)
        mask = plan.escaped(sT, m)
        idx = A.nearest_track_points(sT, cT.numpy(), track, mask)
    assert int(mask.sum()) > 100
    g64 = grad(plan, m, s0, mask, idx)

    def loss(theta, cen):
        with torch.no_grad():
            sT, cT = A.trajectory(plan, s0, m, torch.as_tensor(theta), torch.as_tensor(cen), kinds,
                                  w.dt, H, ck)
            return float(A.track_loss(sT, cT, track, mask, idx).item())

    fd = np.zeros(8)
    for q in range(8):
        th, c = theta0.copy(), cen0.copy()
        if q < 2:
            h = 1e-5 * abs(th[0, q])
            th[0, q] += h
            lp = loss(th, c)
            th[0, q] -= 2 * h
            lm = loss(th, c)
        else:
            h = 1e-5 * max(1.0, abs(c[q - 2]))
            c[q - 2] += h
            lp = loss(th, c)
            c[q - 2] -= 2 * h
            lm = loss(th, c)
        fd[q] = (lp - lm) / (2 * h)
    assert (np.abs(g64 - fd) <= 1e-5 * np.abs(g64)).all(), (g64, fd)
    plan32, m32, s032 = setup("f32")
    g32 = grad(plan32, m32, s032, mask, idx)
    rel = np.abs(g32 - g64) / np.abs(g64)
    print(f"  FP32 vs FP64 gradient, componentwise max {rel.max():.1e}", flush=True)
    assert (rel <= 1e-3).all(), rel


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_kept_weights_replay_equals_recompute(torch, S, dtype):
    """scf_step_keep_weights advances the state exactly as scf_step does, and
    scf_step_adjoint from the kept weights returns exactly what it returns when
    it recomputes the coefficients (the same kernels on the same positions)."""
    n, dt, nsteps = 3000, 0.005, 5
    print(f"[kept weights] {dtype}", flush=True)
    p = I.plummer(n, 5511)
    st0 = _rounded(p.state(), dtype)
    m = _dev(torch, _rounded(p.mass, dtype), dtype)
    plan = S.Plan(10, 6, dtype=dtype)
    host = (NFW, 1.0)
    a = [_dev(torch, st0[i], dtype) for i in range(6)]
    b = [_dev(torch, st0[i], dtype) for i in range(6)]
    wsz = plan.weights_size
    assert wsz == 11 * 49
    hist = torch.full(((nsteps + 1) * wsz,), float("nan"), dtype=a[0].dtype, device="cuda")
    ca, acc_a = plan.step(a, m, dt, nsteps, host=host, centre=CEN)
    cb, acc_b = plan.step(b, m, dt, nsteps, host=host, centre=CEN, w_hist=hist)
    torch.cuda.synchronize()
    assert np.array_equal(ca, cb)
    for u, v in zip(a + acc_a, b + acc_b):
        assert torch.equal(u, v)
    assert bool(torch.isfinite(hist).all())  # every kick's row, the start-up one included
    # with the accelerations carried in, row 0 is left as it is
    h2 = torch.full_like(hist, float("nan"))
    plan.step(b, m, dt, nsteps, host=host, centre=cb, acc=acc_b, w_hist=h2)
    torch.cuda.synchronize()
    assert bool(torch.isnan(h2[:wsz]).all()) and bool(torch.isfinite(h2[wsz:]).all())

    rng = np.random.default_rng(5512)
    lam0 = _rounded(rng.normal(size=(6, n)), dtype)
    lamc = rng.normal(size=6)
    st = [_dev(torch, st0[i], dtype) for i in range(6)]
    l1 = [_dev(torch, lam0[i], dtype) for i in range(6)]
    l2 = [_dev(torch, lam0[i], dtype) for i in range(6)]
    lc1, gh1 = plan.step_adjoint(st, m, dt, nsteps, l1, lamc, host=host, centre0=CEN)
    lc2, gh2 = plan.step_adjoint(st, m, dt, nsteps, l2, lamc, host=host, centre0=CEN, w_hist=hist)
    torch.cuda.synchronize()
    assert np.array_equal(lc1, lc2) and np.array_equal(gh1, gh2)
    for u, v in zip(l1, l2):
        assert torch.equal(u, v)
