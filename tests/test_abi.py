"""CPU checks of the C ABI: the library loads, exports every function that
include/scf.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    from paper_2602_13385_amd import scf
    if not os.path.exists(scf.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    scf.lib()
    return scf


def _declared():
    txt = open(os.path.join(ROOT, "include", "scf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(scf_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(S):
    names = _declared()
    assert "scf_step_adjoint" in names and "scf_coeffs" in names
    L = S.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(S.SIGNATURES), "binding and header disagree"


def test_ncoef_and_status_strings(S):
    L = S.lib()
    assert L.scf_ncoef(16, 10) == 17 * 121
    assert L.scf_ncoef(6, 4) == 175
    assert L.scf_ncoef(-1, 3) == 0
    for k, v in S.STATUS.items():
        assert L.scf_status_string(k).decode() == v


def _create(S, nmax, lmax, alpha=1.0, b=1.0, G=1.0, dtype=0, flags=0):
    h = C.c_void_p()
    basis = S.CBasis(nmax, lmax, alpha, b, G)
    st = S.lib().scf_plan_create(C.byref(h), C.byref(basis), dtype, flags)
    if st == 0:
        S.lib().scf_plan_destroy(h)
    return st


@pytest.mark.parametrize("args,status", [
    ((-1, 3), 1), ((4, -2), 1), ((6, 4, 1.0, 1.0, 1.0, 7), 1), ((6, 4, 1.0, 1.0, 1.0, 0, 3), 1),
    ((6, 4, 1.5), 2), ((6, 4, 0.0), 2), ((6, 4, 1.0, -1.0), 1), ((6, 4, 1.0, 1.0, 0.0), 1),
    ((40, 4), 2), ((6, 30), 2),
])
def test_plan_create_rejects_bad_arguments(S, args, status):
    assert _create(S, *args) == status
    assert len(S.lib().scf_last_error()) > 0


def test_null_pointers_rejected(S):
    L = S.lib()
    assert L.scf_plan_create(None, None, 0, 0) == 1
    assert L.scf_coeffs(None, 10, None, None, None, None, None, None, 0, None) == 1
    assert L.scf_workspace_size(None, 10, 1, None) == 1


def test_python_binding_has_no_cpu_fallback():
    src = open(os.path.join(ROOT, "paper_2602_13385_amd", "scf.py")).read()
    assert "oracle" not in src


def test_tidal_norm_matches_oracle(S, O):
    """scf_tidal_norm runs on the host (double precision, no device work)."""
    comps = [("hernquist", (1.11955, 1.0)), ("mn", (11.8372, 3.0, 0.28)), ("nfw", (124.107, 15.626))]
    H = O.host([(O.HOST_HERNQUIST, (1.11955, 1.0)), (O.HOST_MN, (11.8372, 3.0, 0.28)),
                (O.HOST_NFW, (124.107, 15.626))])
    for pos in ([20.0, 0.0, 0.0], [3.0, -4.0, 0.5], [0.2, 0.1, -8.0]):
        ref = O.tidal_norm(H, pos)
        assert S.tidal_norm((comps, 1.0), pos) == pytest.approx(ref, rel=1e-13)


def test_cadence_density_frame_calls_reject_a_null_plan(S):
    """The refresh-cadence, density and frame entry points validate their
    arguments before any device work."""
    L = S.lib()
    st = S.CCadenceState()
    cad = S.Cadence().c()
    out = (C.c_double * 5)()
    ab = (C.c_double * 2)(1.0, 1.0)
    sz = C.c_size_t()
    assert L.scf_cadence_workspace_size(None, 10, 1, C.byref(sz)) == 1
    assert L.scf_step_frozen(None, 10, *[None] * 9, 0, None, None, None, 0.01, 1, None, 0, None) == 1
    assert L.scf_select(None, 10, *[None] * 8, 0.999, None, None, C.byref(st), None, 0, None) == 1
    assert L.scf_coeffs_delta(None, 10, 1, None, None, None, None, None, None, 0, None) == 1
    assert L.scf_cadence_init(None, 10, *[None] * 7, 0.999, None, None, C.byref(st), None, 0,
                              None) == 1
    assert L.scf_evolve(None, 10, *[None] * 10, None, None, C.byref(cad), 1, None, None,
                        C.byref(st), None, None, 0, None) == 1
    assert L.scf_density(None, 10, None, None, None, None, None, None, 0, None) == 1
    assert L.scf_core(None, 10, *[None] * 9, C.cast(out, C.POINTER(C.c_double)), None, 0,
                      None) == 1
    assert L.scf_recentre(None, 10, None, None, None, None, C.cast(out, C.POINTER(C.c_double)),
                          1e-6, 10, None, None, 0, None) == 1
    assert L.scf_tune_basis(None, 10, None, None, None, None, 0.25,
                            C.cast(ab, C.POINTER(C.c_double)), None, None, 0, None) == 1
    assert L.scf_plan_set_basis(None, 0.5, 1.0) == 1
    assert L.scf_plan_get_basis(None, None) == 1
    for name in ("scf_select", "scf_evolve", "scf_tune_basis"):
        assert len(L.scf_last_error()) > 0, name


def test_bench_ceiling_rejects_bad_arguments(S):
    """The throughput microbenchmark checks kind (0..5), waves per SIMD (1..8)
    and iters before any device call."""
    L = S.lib()
    tf, ms = C.c_double(), C.c_double()
    dummy = C.c_void_p(256)  # never dereferenced: each call fails its argument check
    for kind, wv, it in ((6, 4, 10), (-1, 4, 10), (0, 0, 10), (0, 9, 10), (5, 4, 0)):
        assert L.scf_bench_ceiling(kind, wv, it, dummy, C.byref(tf), C.byref(ms)) == 1
    assert L.scf_bench_ceiling(0, 4, 10, None, C.byref(tf), C.byref(ms)) == 1
