"""scf_step_noalloc (static device scratch, no workspace argument) against
scf_step with a caller workspace: two calls in a row on one plan, the second
on fewer particles, each compared with scf_step on identical inputs.  Both run
the same kernels with the same launch geometry, so the results agree bitwise
(which is within every tolerance of the parity tests)."""
import numpy as np
import pytest

from paper_2602_13385_amd import inputs as I

pytestmark = pytest.mark.gpu


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


LOG_HOST = ([("log", (1.5, 1.0))], 1.0)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_step_matches_workspace_step(torch, S, dtype):
    td = torch.float32 if dtype == "f32" else torch.float64
    nd = np.float32 if dtype == "f32" else np.float64
    plan = S.Plan(10, 6, dtype=dtype)
    assert int(S.lib().scf_noalloc_scratch_bytes()) == 64 << 20
    for n, seed, nsteps in ((20_011, 41, 3), (3_001, 42, 2)):
        print(f"noalloc case dtype={dtype} n={n} seed={seed} nsteps={nsteps}", flush=True)
        p = I.plummer(n, seed)
        st0 = p.state().astype(nd)
        m = torch.as_tensor(p.mass.astype(nd), device="cuda")
        centre = np.array([20.0, 0.0, 0.0, 0.0, 1.498127, 0.0])
        outs = []
        for fn in (plan.step, plan.step_noalloc):
            st = [torch.as_tensor(np.ascontiguousarray(st0[i]), device="cuda") for i in range(6)]
            coef = torch.empty(S.ncoef(10, 6), dtype=torch.float64, device="cuda")
            cen, acc = fn(st, m, 0.005, nsteps, host=LOG_HOST, centre=centre, coef_last=coef)
            torch.cuda.synchronize()
            outs.append((np.stack([t.cpu().numpy() for t in st]),
                         np.stack([t.cpu().numpy() for t in acc]), cen, coef.cpu().numpy()))
        (s0, a0, c0, k0), (s1, a1, c1, k1) = outs
        assert np.isfinite(s1).all() and np.isfinite(k1).all()
        assert np.array_equal(s0, s1)
        assert np.array_equal(a0, a1)
        assert np.array_equal(c0, c1)
        assert np.array_equal(k0, k1)
        assert np.abs(k1).max() > 0
