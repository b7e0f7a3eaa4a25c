"""GPU checks of scf_step_batched (many clusters, one launch per kernel per
step, middle steps replayed from a HIP graph) against

  * the FP64 oracle's batched step (a loop of per-cluster steps), per step
    from identical states, to the plain-step bars;
  * the same kernels launched without the graph: bitwise identical, on every
    replay, with unrelated eager work and synchronisations in between;
  * the plain per-cluster scf_step on the same GPU.
"""
import math

import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-11}
HOST = I.CONFIG4_HOST


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


def _clusters(sizes, seed):
    """Plummer clusters of the given sizes on eccentric orbits in the composite
    host (the batched workload's recipe at reduced N)."""
    rng = np.random.default_rng(seed)
    parts, cens = [], []
    for i, n in enumerate(sizes):
        p = I.plummer(max(n, 1), seed + 10 + i)
        parts.append(p.state()[:, :n])
        r_apo = rng.uniform(15.0, 40.0)
        v = rng.uniform(0.5, 1.3)  # tangential: an eccentric bound orbit in this host
        th = rng.uniform(0, 2 * math.pi)
        cens.append(np.array([r_apo * math.cos(th), r_apo * math.sin(th), 0.3,
                              -v * math.sin(th), v * math.cos(th), 0.05]))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    st = np.concatenate(parts, axis=1) if sum(sizes) else np.zeros((6, 0))
    m = np.concatenate([np.full(n, 1.0 / max(n, 1)) for n in sizes]) if sum(sizes) else np.zeros(0)
    return off, st, m, np.array(cens)


def _ohost(O):
    kinds = {"hernquist": O.HOST_HERNQUIST, "mn": O.HOST_MN, "nfw": O.HOST_NFW}
    return O.host([(kinds[k], p) for k, p in HOST])


def _run(torch, S, plan, off, st0, m, cens, dtype, dt, nsteps, graph=False, coef=None):
    st = [_dev(torch, st0[i], dtype) for i in range(6)]
    md = _dev(torch, m, dtype)
    cen, acc = plan.step_batched(off, st, md, dt, nsteps, host=(HOST, 1.0), centres=cens,
                                 coef_last=coef, graph=graph)
    torch.cuda.synchronize()
    out = np.stack([t.cpu().numpy() for t in st]).astype(np.float64)
    a = np.stack([t.cpu().numpy() for t in acc]).astype(np.float64)
    return out, cen, a


# fv: the plan's field variant (the batched step runs variant 1's kernel for the
# matrix-core variants 2 and 3 of FP32 plans); cv: the coefficient variant (3 =
# the block kernel of FP64 plans)
@pytest.mark.parametrize("dtype,fv,cv", [("f32", 0, 0), ("f32", 2, 0), ("f32", 3, 0),
                                         ("f64", 0, 0), ("f64", 0, 3)])
def test_batched_matches_oracle(torch, S, O, dtype, fv, cv):
    sizes = [3000, 0, 11000, 6173, 1]
    print(f"[batched parity] sizes={sizes} {dtype} field variant {fv} coefficient variant {cv}",
          flush=True)
    off, st0, m, cens = _clusters(sizes, 4401)
    st0, m = _rounded(st0, dtype), _rounded(m, dtype)
    dt, nsteps = 0.005, 4
    B = O.basis(10, 6)
    st_ref, cen_ref, coef_ref = O.step_batched(B, _ohost(O), off, st0, m, cens, dt, nsteps)
    plan = S.Plan(10, 6, dtype=dtype)
    plan.field_variant = fv
    plan.variant = cv
    coef = torch.empty(len(sizes) * plan.T, dtype=torch.float64, device="cuda")
    out, cen, _ = _run(torch, S, plan, off, st0, m, cens, dtype, dt, nsteps, coef=coef)
    assert np.abs(cen - cen_ref).max() <= 1e-12
    tol = TOL[dtype]
    for c in range(len(sizes)):
        sl = slice(off[c], off[c + 1])
        if off[c + 1] == off[c]:
            continue
        for rows in (slice(0, 3), slice(3, 6)):
            ref = st_ref[rows, sl]
            d = np.abs(out[rows, sl] - ref).max() / np.abs(ref).max()
            assert d <= tol, (c, d)
    cg = coef.cpu().numpy().reshape(len(sizes), -1)
    for c in range(len(sizes)):
        if off[c + 1] == off[c]:
            assert np.all(cg[c] == 0.0)
            continue
        e = np.abs(cg[c] - coef_ref[c]).max() / np.abs(coef_ref[c]).max()
        assert e <= tol, (c, e)


@pytest.mark.parametrize("fv", [0, 3])
def test_batched_graph_replays_equal_eager(torch, S, fv):
    """Every graph replay equals the directly launched kernels bitwise,
    across several calls with other GPU work and host synchronisation in
    between; the graph is captured once for the repeated argument set."""
    sizes = [5000, 2500, 9000]
    off, st0, m, cens = _clusters(sizes, 4402)
    plan = S.Plan(10, 6, dtype="f32")
    plan.field_variant = fv
    md = _dev(torch, m, "f32")
    sg = [_dev(torch, st0[i], "f32") for i in range(6)]
    se = [_dev(torch, st0[i], "f32") for i in range(6)]
    cg, ce = cens.copy(), cens.copy()
    ag = ae = None
    for call in range(3):
        cg, ag = plan.step_batched(off, sg, md, 0.005, 4, host=(HOST, 1.0), centres=cg, acc=ag,
                                   graph=True)
        junk = torch.randn(1 << 20, device="cuda")
        junk = (junk * 2.0).sum()
        torch.cuda.synchronize()
        ce, ae = plan.step_batched(off, se, md, 0.005, 4, host=(HOST, 1.0), centres=ce, acc=ae,
                                   graph=False)
        torch.cuda.synchronize()
        for a, b in zip(sg + ag, se + ae):
            assert torch.equal(a, b), f"call {call}"
        assert np.array_equal(cg, ce)
    assert plan.graph_captures == 1


def test_batched_eight_step_graphs_across_centre_chunks(torch, S):
    """300 steps: runs of middle steps replay the eight-step graph, the others
    the one-step graph, and the centre table is re-uploaded after 256 steps;
    the result equals the directly launched kernels bitwise."""
    sizes = [3000, 1200]
    off, st0, m, cens = _clusters(sizes, 4403)
    plan = S.Plan(6, 4, dtype="f32")
    md = _dev(torch, m, "f32")
    sg = [_dev(torch, st0[i], "f32") for i in range(6)]
    se = [_dev(torch, st0[i], "f32") for i in range(6)]
    cg, ag = plan.step_batched(off, sg, md, 0.004, 300, host=(HOST, 1.0), centres=cens,
                               graph=True)
    ce, ae = plan.step_batched(off, se, md, 0.004, 300, host=(HOST, 1.0), centres=cens,
                               graph=False)
    torch.cuda.synchronize()
    for a, b in zip(sg + ag, se + ae):
        assert torch.equal(a, b)
    assert np.array_equal(cg, ce)
    assert plan.graph_captures == 1


@pytest.mark.parametrize("dtype,fv", [("f32", 0), ("f32", 3), ("f64", 0)])
def test_batched_equals_plain_per_cluster(torch, S, dtype, fv):
    sizes = [4000, 7000]
    off, st0, m, cens = _clusters(sizes, 4403)
    dt, nsteps = 0.005, 3
    plan = S.Plan(10, 6, dtype=dtype)
    plan.field_variant = fv
    out, cen, acc = _run(torch, S, plan, off, st0, m, cens, dtype, dt, nsteps)
    tol = 1e-6 if dtype == "f32" else 1e-13
    for c in range(len(sizes)):
        sl = slice(off[c], off[c + 1])
        st = [_dev(torch, st0[i, sl], dtype) for i in range(6)]
        cc, ac = plan.step(st, _dev(torch, m[sl], dtype), dt, nsteps, host=(HOST, 1.0),
                           centre=cens[c])
        torch.cuda.synchronize()
        o = np.stack([t.cpu().numpy() for t in st]).astype(np.float64)
        assert np.abs(cc - cen[c]).max() <= 1e-13
        assert np.abs(o - out[:, sl]).max() <= tol * np.abs(o).max()


def test_batched_split_call_and_edges(torch, S):
    sizes = [2000, 3000]
    off, st0, m, cens = _clusters(sizes, 4404)
    plan = S.Plan(10, 6, dtype="f32")
    md = _dev(torch, m, "f32")
    a = [_dev(torch, st0[i], "f32") for i in range(6)]
    cA, accA = plan.step_batched(off, a, md, 0.005, 5, host=(HOST, 1.0), centres=cens)
    b = [_dev(torch, st0[i], "f32") for i in range(6)]
    cB, accB = plan.step_batched(off, b, md, 0.005, 2, host=(HOST, 1.0), centres=cens)
    cB, accB = plan.step_batched(off, b, md, 0.005, 3, host=(HOST, 1.0), centres=cB, acc=accB)
    torch.cuda.synchronize()
    ref = np.stack([t.cpu().numpy() for t in a])
    got = np.stack([t.cpu().numpy() for t in b])
    assert np.abs(ref - got).max() <= 1e-6 * np.abs(ref).max()
    assert np.abs(cA - cB).max() <= 1e-12 * np.abs(cA).max()
    # nsteps = 0 only evaluates a(x0) (and leaves the state alone)
    c = [_dev(torch, st0[i], "f32") for i in range(6)]
    c0, acc0 = plan.step_batched(off, c, md, 0.005, 0, host=(HOST, 1.0), centres=cens)
    torch.cuda.synchronize()
    assert np.array_equal(c0, cens)
    assert np.array_equal(np.stack([t.cpu().numpy() for t in c]), st0.astype(np.float32))
    assert all(torch.isfinite(t).all() for t in acc0)
    # one cluster and an all-empty batch
    one = [_dev(torch, st0[i, :2000], "f32") for i in range(6)]
    plan.step_batched([0, 2000], one, md[:2000], 0.005, 2, host=(HOST, 1.0), centres=cens[:1])
    empty = [torch.empty(0, device="cuda") for _ in range(6)]
    ce, _ = plan.step_batched([0, 0, 0], empty, torch.empty(0, device="cuda"), 0.005, 3,
                              host=(HOST, 1.0), centres=cens)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(ce))
    with pytest.raises(S.ScfError):
        plan.step_batched([0, 3000, 2000], a, md, 0.005, 1, host=(HOST, 1.0), centres=cens)
    with pytest.raises(S.ScfError):
        plan.step_batched([1, 2000, 5000], a, md, 0.005, 1, host=(HOST, 1.0), centres=cens)
