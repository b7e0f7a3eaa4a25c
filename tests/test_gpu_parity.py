"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars (fixed before the kernels were written):
  coefficients  max_t |da_t| / max_t |a_t|                  <= 1e-5 (FP32), 1e-11 (FP64)
  forces        max_i |dg_i| / (|g_i| + median_j |g_j|)     <= 1e-5 (FP32), 1e-11 (FP64)
The oracle is fed the same FP32-representable inputs, upcast to double.
"""
import math

import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-11}


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


def _dev(torch, arr, dtype):
    td = torch.float32 if dtype == "f32" else torch.float64
    return torch.as_tensor(np.ascontiguousarray(arr), dtype=td, device="cuda")


def _rounded(arr, dtype):
    return np.asarray(arr, dtype=np.float32).astype(np.float64) if dtype == "f32" else np.asarray(arr, np.float64)


def coef_err(a, ref):
    return np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300)


# Per degree: |da| <= TOL * max|a_l-block| + FLOOR * max|a|.  Single-precision
# evaluation of the basis leaves an absolute error of order 1e-8 |a_000| in
# every coefficient, so a block whose own size is below about 1e-3 |a_000|
# (the noise-level l > 0 blocks of a near-spherical sample) is resolved only
# to that floor.
FLOOR = {"f32": 2e-8, "f64": 1e-15}


def block_errs(a, ref, nmax, lmax, dtype):
    """Per-l ratio of the error to its bound (<= 1 passes)."""
    L2 = (lmax + 1) ** 2
    A = np.asarray(a).reshape(nmax + 1, L2)
    Rf = np.asarray(ref).reshape(nmax + 1, L2)
    top = np.abs(Rf).max()
    out = []
    for l in range(lmax + 1):
        sl = slice(l * l, (l + 1) ** 2)
        bound = TOL[dtype] * np.abs(Rf[:, sl]).max() + FLOOR[dtype] * top
        out.append(np.abs(A[:, sl] - Rf[:, sl]).max() / bound)
    return np.array(out)


def force_err(g, ref):
    mag = np.sqrt((ref ** 2).sum(0))
    d = np.sqrt(((g - ref) ** 2).sum(0))
    return (d / (mag + np.median(mag))).max()


def _gpu_coeffs(torch, S, plan, pos, m, dtype):
    x, y, z = (_dev(torch, pos[i], dtype) for i in range(3))
    c = plan.coeffs(x, y, z, _dev(torch, m, dtype))
    torch.cuda.synchronize()
    return c.cpu().numpy()


CASES = [  # (nmax, lmax, alpha, n, generator)
    (6, 4, 1.0, 10_000, "plummer"),
    (10, 6, 1.0, 20_011, "plummer"),
    (16, 10, 1.0, 30_001, "hernquist"),
    (10, 5, 1.0, 4_099, "ball"),
    (8, 3, 1.0, 3_001, "ball"),  # generic instance (runtime nmax < compiled bound)
    (20, 10, 1.0, 2_003, "hernquist"),  # generic instance at its compiled bound
    (12, 0, 1.0, 1_001, "plummer"),  # monopole only (generic, lmax 0)
    (5, 1, 1.0, 1_003, "plummer"),  # lmax 1 and 2: split-degree parts left empty
    (7, 2, 1.0, 1_009, "ball"),
    (9, 7, 1.0, 2_011, "ball"),  # generic instances of odd degree bounds
    (14, 9, 1.0, 2_017, "hernquist"),
    (6, 4, 0.5, 5_003, "plummer"),
    (10, 6, 0.8, 5_003, "plummer"),
]


def _gen(kind, n, seed):
    if kind == "plummer":
        return I.plummer(n, seed)
    if kind == "hernquist":
        return I.hernquist(n, seed)
    return I.uniform_ball(n, seed)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}l{c[1]}a{c[2]}N{c[3]}")
def test_coeffs_and_forces_match_oracle(torch, S, O, case, dtype):
    nmax, lmax, alpha, n, kind = case
    print(f"[parity] nmax={nmax} lmax={lmax} alpha={alpha} N={n} {dtype}", flush=True)
    p = _gen(kind, n, 700 + n % 97)
    pos = _rounded(p.pos, dtype)
    m = _rounded(p.mass, dtype)
    B = O.basis(nmax, lmax, alpha=alpha)
    ref = O.coeffs(B, *pos, m)
    plan = S.Plan(nmax, lmax, alpha=alpha, dtype=dtype)
    for v in range(plan.num_variants):
        plan.variant = v
        c = _gpu_coeffs(torch, S, plan, pos, m, dtype)
        assert coef_err(c, ref) <= TOL[dtype], (v, coef_err(c, ref))
        be = block_errs(c, ref, nmax, lmax, dtype)
        assert (be <= 1.0).all(), (v, be)
    # forces from the reference coefficients, at a sample of the particles
    # (a ragged count), for every field variant
    k = min(n, 2000)
    sub = pos[:, :k]
    Pref, gref = O.field(B, ref, *sub)
    x, y, z = (_dev(torch, sub[i], dtype) for i in range(3))
    for fv in range(plan.num_field_variants):
        plan.field_variant = fv
        ax, ay, az, pot = plan.forces(x, y, z, torch.as_tensor(ref, device="cuda"), pot=True)
        torch.cuda.synchronize()
        g = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()]).astype(np.float64)
        assert force_err(g, gref) <= TOL[dtype], (fv, force_err(g, gref))
        P = pot.cpu().numpy().astype(np.float64)
        assert np.abs(P - Pref).max() / np.abs(Pref).max() <= TOL[dtype], fv


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_forces_with_host_tidal_field(torch, S, O, dtype):
    p = I.plummer(3000, 31)
    pos = _rounded(p.pos, dtype)
    m = _rounded(p.mass, dtype)
    comps = [("hernquist", (1.11955, 1.0)), ("mn", (11.8372, 3.0, 0.28)), ("nfw", (124.107, 15.626))]
    Hc = O.host([(O.HOST_HERNQUIST, (1.11955, 1.0)), (O.HOST_MN, (11.8372, 3.0, 0.28)),
                 (O.HOST_NFW, (124.107, 15.626))])
    centre = np.array([18.0, -4.0, 2.5])
    B = O.basis(10, 6)
    ref = O.coeffs(B, *pos, m)
    _, gscf = O.field(B, ref, *pos)
    _, g0, _ = O.host_eval(Hc, centre)
    gh = np.stack([O.host_eval(Hc, centre + pos[:, i])[1] for i in range(pos.shape[1])], axis=1)
    gref = gscf - gh + g0[:, None]
    plan = S.Plan(10, 6, dtype=dtype)
    x, y, z = (_dev(torch, pos[i], dtype) for i in range(3))
    for fv in range(plan.num_field_variants):
        plan.field_variant = fv
        ax, ay, az = plan.forces(x, y, z, torch.as_tensor(ref, device="cuda"), host=(comps, 1.0),
                                 centre=centre)
        torch.cuda.synchronize()
        g = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()]).astype(np.float64)
        assert force_err(g, gref) <= TOL[dtype], (fv, force_err(g, gref))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_edge_cases(torch, S, O, dtype):
    plan = S.Plan(6, 4, dtype=dtype)
    B = O.basis(6, 4)
    td = torch.float32 if dtype == "f32" else torch.float64
    e = torch.empty(0, dtype=td, device="cuda")
    c = plan.coeffs(e, e, e, e)
    torch.cuda.synchronize()
    assert (c.cpu().numpy() == 0).all()
    ax, ay, az = plan.forces(e, e, e, c)
    assert ax.numel() == 0
    # one particle; a particle exactly at the origin; particles on the poles
    pos = np.array([[0.0, 0.0, 0.0, 0.3, 1.0], [0.0, 0.0, 0.0, -0.2, 0.5], [0.0, 1.5, -2.0, 0.1, -0.7]])
    m = np.array([0.2, 0.3, 0.1, 0.25, 0.15])
    for k in (1, 5):
        ref = O.coeffs(B, *pos[:, :k], m[:k])
        for v in range(plan.num_variants):
            plan.variant = v
            cg = _gpu_coeffs(torch, S, plan, _rounded(pos[:, :k], dtype), _rounded(m[:k], dtype), dtype)
            assert coef_err(cg, ref) <= TOL[dtype]
    ref = O.coeffs(B, *pos, m)
    _, gref = O.field(B, ref, *pos)
    x, y, z = (_dev(torch, pos[i], dtype) for i in range(3))
    for fv in range(plan.num_field_variants):
        plan.field_variant = fv
        ax, ay, az = plan.forces(x, y, z, torch.as_tensor(ref, device="cuda"))
        torch.cuda.synchronize()
        g = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()]).astype(np.float64)
        assert np.isfinite(g).all(), fv
        assert (g[:, 0] == 0).all(), fv  # the origin gets zero SCF force
        assert force_err(g, gref) <= TOL[dtype], fv


def test_coefficients_are_deterministic(torch, S):
    p = I.plummer(50_000, 5)
    plan = S.Plan(10, 6)
    x, y, z, m = (_dev(torch, a, "f32") for a in (*p.pos, p.mass))
    for v in range(plan.num_variants):
        plan.variant = v
        c1 = plan.coeffs(x, y, z, m).cpu().numpy()
        c2 = plan.coeffs(x, y, z, m).cpu().numpy()
        assert np.array_equal(c1, c2)


def test_autotune_picks_a_valid_variant(torch, S, O):
    p = I.plummer(40_000, 6)
    plan = S.Plan(10, 6)
    x, y, z, m = (_dev(torch, a, "f32") for a in (*p.pos, p.mass))
    v, ms = plan.autotune(x, y, z, m)
    assert 0 <= v < plan.num_variants and ms > 0
    ref = O.coeffs(O.basis(10, 6), *_rounded(p.pos, "f32"), _rounded(p.mass, "f32"))
    c = plan.coeffs(x, y, z, m).cpu().numpy()
    assert coef_err(c, ref) <= TOL["f32"]


def test_hernquist_quadrature_closed_form(torch, S):
    # the exact pin, through the GPU path: a_000 = 1/sqrt(3), others 0
    q = I.quadrature_sphere("hernquist", 1.0, nr=40, nmu=24, nphi=24)
    plan = S.Plan(16, 10, dtype="f64")
    c = _gpu_coeffs(torch, S, plan, q.pos, q.mass, "f64")
    assert c[0] == pytest.approx(1 / math.sqrt(3), rel=1e-12)
    assert np.abs(c[1:]).max() < 1e-12
    plan32 = S.Plan(16, 10, dtype="f32")
    c32 = _gpu_coeffs(torch, S, plan32, _rounded(q.pos, "f32"), _rounded(q.mass, "f32"), "f32")
    assert abs(c32[0] - 1 / math.sqrt(3)) < 1e-5 and np.abs(c32[1:]).max() < 1e-5


STEP_CASES = [  # (nmax, lmax, n, host, centre, dt, nsteps)
    (6, 4, 10_000, None, np.zeros(6), 0.01, 3),
    (10, 6, 20_000, [("log", (1.5, 1.0))], np.array([20.0, 0, 0, 0, I.LOG_VC_20, 0]), 0.005, 3),
    (10, 6, 8_000, [("nfw", (232.98, 20.0))], np.array([20.0, 0, 0, 0.1, 1.4, 0.3]), 0.005, 4),
]


def _ohost(O, comps):
    if comps is None:
        return None
    kinds = {"log": O.HOST_LOG, "hernquist": O.HOST_HERNQUIST, "nfw": O.HOST_NFW, "mn": O.HOST_MN,
             "plummer": O.HOST_PLUMMER}
    return O.host([(kinds[k], p) for k, p in comps])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: f"n{c[0]}l{c[1]}N{c[2]}")
def test_step_matches_oracle(torch, S, O, case, dtype):
    nmax, lmax, n, comps, centre, dt, nsteps = case
    print(f"[step parity] nmax={nmax} lmax={lmax} N={n} {dtype} host={comps}", flush=True)
    p = I.plummer(n, 900 + nsteps)
    st0 = _rounded(p.state(), dtype)
    m = _rounded(p.mass, dtype)
    B = O.basis(nmax, lmax)
    Ho = _ohost(O, comps)
    st_ref, cen_ref, coef_ref, acc_ref = O.step(B, Ho, st0, m, centre, dt, nsteps, want_acc=True)
    plan = S.Plan(nmax, lmax, dtype=dtype)
    st = [_dev(torch, st0[i], dtype) for i in range(6)]
    md = _dev(torch, m, dtype)
    coef = torch.empty(plan.T, dtype=torch.float64, device="cuda")
    cen, acc = plan.step(st, md, dt, nsteps, host=(comps, 1.0) if comps else None, centre=centre,
                         coef_last=coef)
    torch.cuda.synchronize()
    out = np.stack([t.cpu().numpy() for t in st]).astype(np.float64)
    a = np.stack([t.cpu().numpy() for t in acc]).astype(np.float64)
    assert np.allclose(cen, cen_ref, rtol=0, atol=1e-12)
    tol = TOL[dtype]
    for rows in (slice(0, 3), slice(3, 6)):
        d = np.abs(out[rows] - st_ref[rows]).max() / np.abs(st_ref[rows]).max()
        assert d <= tol, d
    assert coef_err(coef.cpu().numpy(), coef_ref) <= tol
    assert force_err(a, acc_ref) <= 2 * tol, force_err(a, acc_ref)
    # a second call continuing with the returned accelerations equals one
    # longer call
    st2 = [_dev(torch, st0[i], dtype) for i in range(6)]
    cenA, accA = plan.step(st2, md, dt, 1, host=(comps, 1.0) if comps else None, centre=centre)
    cenB, accB = plan.step(st2, md, dt, nsteps - 1, host=(comps, 1.0) if comps else None,
                           centre=cenA, acc=accA)
    torch.cuda.synchronize()
    out2 = np.stack([t.cpu().numpy() for t in st2]).astype(np.float64)
    split_tol = 1e-6 if dtype == "f32" else 1e-13
    assert np.abs(out2 - out).max() <= split_tol * np.abs(out).max()


@pytest.mark.parametrize("fv", [2, 3, 4, 5])
@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: f"n{c[0]}l{c[1]}N{c[2]}")
def test_step_with_other_field_variants_matches_oracle(torch, S, O, case, fv):
    """The fused kick-drift of the step (host field included) through the
    matrix-core field variants (2, 3) and the split-degree ones (4, 5),
    against the oracle's steps."""
    nmax, lmax, n, comps, centre, dt, nsteps = case
    print(f"[step parity, field variant {fv}] nmax={nmax} lmax={lmax} N={n}", flush=True)
    p = I.plummer(n, 900 + nsteps)
    st0 = _rounded(p.state(), "f32")
    m = _rounded(p.mass, "f32")
    B = O.basis(nmax, lmax)
    st_ref, cen_ref, coef_ref, acc_ref = O.step(B, _ohost(O, comps), st0, m, centre, dt, nsteps,
                                                want_acc=True)
    plan = S.Plan(nmax, lmax, dtype="f32")
    plan.field_variant = fv
    st = [_dev(torch, st0[i], "f32") for i in range(6)]
    cen, acc = plan.step(st, _dev(torch, m, "f32"), dt, nsteps,
                         host=(comps, 1.0) if comps else None, centre=centre)
    torch.cuda.synchronize()
    out = np.stack([t.cpu().numpy() for t in st]).astype(np.float64)
    a = np.stack([t.cpu().numpy() for t in acc]).astype(np.float64)
    assert np.allclose(cen, cen_ref, rtol=0, atol=1e-12)
    for rows in (slice(0, 3), slice(3, 6)):
        d = np.abs(out[rows] - st_ref[rows]).max() / np.abs(st_ref[rows]).max()
        assert d <= TOL["f32"], d
    assert force_err(a, acc_ref) <= 2 * TOL["f32"], force_err(a, acc_ref)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_field_variants_agree(torch, S, dtype):
    """Each pair of variants that runs one kernel under two register budgets
    (0 and 1 on the vector ALUs, 2 and 3 on the matrix cores in FP32) agrees
    bitwise, and every variant is deterministic; the matrix-core pair and the
    last two variants (degrees split over 2 or 4 waves) sum in other orders
    and agree with the vector pair to the force bar."""
    p = I.hernquist(20_000, 4242)
    plan = S.Plan(16, 10, dtype=dtype)
    x, y, z = (_dev(torch, p.pos[i], dtype) for i in range(3))
    m = _dev(torch, p.mass, dtype)
    c = plan.coeffs(x, y, z, m)
    nv = plan.num_field_variants
    assert nv == (6 if dtype == "f32" else 4)
    outs = []
    for v in list(range(nv)) + [nv - 1]:
        plan.field_variant = v
        outs.append(plan.forces(x, y, z, c, host=([("nfw", (232.98, 20.0))], 1.0),
                                centre=[20.0, 1.0, -2.0]))
    torch.cuda.synchronize()
    for i, j in [(0, 1), (nv, nv - 1)] + ([(2, 3)] if nv > 4 else []):
        for a, b in zip(outs[i], outs[j]):
            assert torch.equal(a, b), (i, j)
    g0 = np.stack([t.cpu().numpy() for t in outs[0]]).astype(np.float64)
    for k in ([2] if nv > 4 else []) + [nv - 2, nv - 1]:
        gk = np.stack([t.cpu().numpy() for t in outs[k]]).astype(np.float64)
        assert force_err(gk, g0) <= TOL[dtype], (k, force_err(gk, g0))
    plan.autotune(x, y, z, m)
    assert 0 <= plan.field_variant < nv


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 127, 129, 255, 257, 1000])
def test_field_variants_small_and_ragged_counts(torch, S, O, n, dtype):
    """Every lane of a wave joins the matrix-core chains (FP32 variants 2, 3)
    and every thread of the split-degree variants (the last two) reaches its
    barrier; lanes past the end evaluate the last particle and store
    nothing."""
    print(f"[ragged field] {dtype} n={n}", flush=True)
    p = I.plummer(max(n, 2), 900 + n)
    pos = _rounded(p.pos[:, :n], dtype)
    B = O.basis(10, 6)
    ref = O.coeffs(B, *_rounded(p.pos, dtype), _rounded(p.mass, dtype))
    Pref, gref = O.field(B, ref, *pos)
    plan = S.Plan(10, 6, dtype=dtype)
    td = torch.float32 if dtype == "f32" else torch.float64
    x, y, z = (_dev(torch, pos[i], dtype) for i in range(3))
    nv = plan.num_field_variants
    for fv in ((2, 3) if dtype == "f32" else ()) + (nv - 2, nv - 1):
        plan.field_variant = fv
        guard = torch.full((n + 64,), 7.0, dtype=td, device="cuda")
        ax = guard[:n]
        ay, az, pot = (torch.empty(n, dtype=td, device="cuda") for _ in range(3))
        plan.forces(x, y, z, torch.as_tensor(ref, device="cuda"), pot=True,
                    out=(ax, ay, az, pot))
        torch.cuda.synchronize()
        g = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()]).astype(np.float64)
        assert force_err(g, gref) <= TOL[dtype], (fv, force_err(g, gref))
        assert np.abs(pot.cpu().numpy() - Pref).max() / np.abs(Pref).max() <= TOL[dtype], fv
        assert (guard[n:].cpu().numpy() == 7.0).all(), fv


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_power_spectrum_matches_oracle(torch, S, O, dtype):
    p = I.plummer(20_000, 77)
    pos = _rounded(p.pos * np.array([[1.0], [0.8], [0.5]]), dtype)
    m = _rounded(p.mass, dtype)
    B = O.basis(10, 6)
    ref = O.coeffs(B, *pos, m)
    Eref = O.power(10, 6, ref)
    plan = S.Plan(10, 6, dtype=dtype)
    c = torch.as_tensor(_gpu_coeffs(torch, S, plan, pos, m, dtype), device="cuda")
    E = plan.power(c).cpu().numpy()
    # against the oracle: E_l = sum |a|^2 inherits twice the coefficient bar
    assert np.abs(E - Eref).max() / Eref.max() <= 2 * TOL[dtype]
    # the kernel's arithmetic, on the GPU's own coefficients
    own = O.power(10, 6, c.cpu().numpy())
    assert np.allclose(E, own, rtol=1e-13, atol=0)
    # a batch of two coefficient sets
    both = torch.stack([c, 2 * c])
    Eb = plan.power(both).cpu().numpy()
    assert np.allclose(Eb[0], own, rtol=1e-13) and np.allclose(Eb[1], 4 * own, rtol=1e-13)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("alpha", [1.0, 0.8])
def test_scaled_basis_with_plummer_host(torch, S, O, dtype, alpha):
    """b != 1 and G != 1 (Eq. psi_nlm with s = r/b; the normalisation scales
    as b/G), a host with a Plummer and a logarithmic component: coefficients,
    forces and three KDK steps against the oracle."""
    b, G = 1.7, 0.6
    print(f"[parity] scaled basis alpha={alpha} b={b} G={G} {dtype}", flush=True)
    p = I.plummer(6001, 55, a=1.5, G=G)
    pos = _rounded(p.pos, dtype)
    m = _rounded(p.mass, dtype)
    B = O.basis(10, 6, alpha=alpha, b=b, G=G)
    ref = O.coeffs(B, *pos, m)
    plan = S.Plan(10, 6, alpha=alpha, b=b, G=G, dtype=dtype)
    c = _gpu_coeffs(torch, S, plan, pos, m, dtype)
    assert coef_err(c, ref) <= TOL[dtype], coef_err(c, ref)
    assert (block_errs(c, ref, 10, 6, dtype) <= 1.0).all()
    comps = [("plummer", (40.0, 3.0)), ("log", (1.2, 0.5))]
    Ho = O.host([(O.HOST_PLUMMER, (40.0, 3.0)), (O.HOST_LOG, (1.2, 0.5))], G=G)
    centre = np.array([12.0, 5.0, -3.0])
    _, gscf = O.field(B, ref, *pos)
    _, g0, _ = O.host_eval(Ho, centre)
    gh = np.stack([O.host_eval(Ho, centre + pos[:, i])[1] for i in range(pos.shape[1])], axis=1)
    gref = gscf - gh + g0[:, None]
    x, y, z = (_dev(torch, pos[i], dtype) for i in range(3))
    for fv in range(plan.num_field_variants):
        plan.field_variant = fv
        ax, ay, az = plan.forces(x, y, z, torch.as_tensor(ref, device="cuda"), host=(comps, G),
                                 centre=centre)
        torch.cuda.synchronize()
        g = np.stack([ax.cpu().numpy(), ay.cpu().numpy(), az.cpu().numpy()]).astype(np.float64)
        assert force_err(g, gref) <= TOL[dtype], (fv, force_err(g, gref))
    cen0 = np.array([12.0, 5.0, -3.0, 0.4, 1.1, -0.2])
    st0 = _rounded(p.state(), dtype)
    st_ref, cen_ref, coef_ref, acc_ref = O.step(B, Ho, st0, m, cen0, 0.004, 3, want_acc=True)
    st = [_dev(torch, st0[i], dtype) for i in range(6)]
    coef = torch.empty(plan.T, dtype=torch.float64, device="cuda")
    cen, acc = plan.step(st, _dev(torch, m, dtype), 0.004, 3, host=(comps, G), centre=cen0,
                         coef_last=coef)
    torch.cuda.synchronize()
    out = np.stack([t.cpu().numpy() for t in st]).astype(np.float64)
    assert np.allclose(cen, cen_ref, rtol=0, atol=1e-12)
    for rows in (slice(0, 3), slice(3, 6)):
        d = np.abs(out[rows] - st_ref[rows]).max() / np.abs(st_ref[rows]).max()
        assert d <= TOL[dtype], d
    assert coef_err(coef.cpu().numpy(), coef_ref) <= TOL[dtype]


def test_single_precision_folds_over_long_unit_ranges(torch, S, O):
    """With one eighth of a resident round of units, each unit of the
    single-precision kernel covers about 25 stages at N = 2e5, so its sums
    pass through more than one two-sum fold into the (hi, lo) rows; the
    result matches the oracle and the one-round launch."""
    p = I.hernquist(200_000, 808)
    pos = _rounded(p.pos, "f32")
    m = _rounded(p.mass, "f32")
    B = O.basis(16, 10)
    ref = O.coeffs(B, *pos, m)
    plan = S.Plan(16, 10, dtype="f32")
    outs = []
    for div in (1, 8):
        plan.coef_units_div = div
        outs.append(_gpu_coeffs(torch, S, plan, pos, m, "f32"))
        assert coef_err(outs[-1], ref) <= TOL["f32"], (div, coef_err(outs[-1], ref))
        be = block_errs(outs[-1], ref, 16, 10, "f32")
        assert (be <= 1.0).all(), (div, be)
    assert coef_err(outs[1], outs[0]) <= TOL["f32"]
