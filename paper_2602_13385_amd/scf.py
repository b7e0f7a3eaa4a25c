"""Thin ctypes binding of libscf (include/scf.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of ``libscf.so``.  PyTorch provides device memory (tensors) and the current
stream.  If the library is missing this module raises ImportError-like
RuntimeError on first use; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscf.so")

F32, F64 = 0, 1
STEP_ACC_VALID = 1
STEP_NO_GRAPH = 2
STEP_GRAPH = 4
HOST_KINDS = {"log": 1, "hernquist": 2, "nfw": 3, "mn": 4, "plummer": 5}
MAX_HOST_COMP = 8

STATUS = {0: "SCF_OK", 1: "SCF_ERR_INVALID_ARG", 2: "SCF_ERR_UNSUPPORTED", 3: "SCF_ERR_WORKSPACE",
          4: "SCF_ERR_NONFINITE", 5: "SCF_ERR_HIP"}


class ScfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CBasis(C.Structure):
    _fields_ = [("nmax", C.c_int32), ("lmax", C.c_int32), ("alpha", C.c_double),
                ("b", C.c_double), ("G", C.c_double)]


class CHostComp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("p", C.c_double * 3)]


class CKernelTime(C.Structure):
    _fields_ = [("kind", C.c_int32), ("count", C.c_int32), ("total_ms", C.c_double)]


KERNEL_KINDS = 13


class CHost(C.Structure):
    _fields_ = [("ncomp", C.c_int32), ("pad", C.c_int32), ("G", C.c_double),
                ("comp", CHostComp * MAX_HOST_COMP)]


class CCadence(C.Structure):
    _fields_ = [("eta", C.c_double), ("dt_max", C.c_double), ("frac", C.c_double),
                ("c_dyn", C.c_double), ("refresh_every", C.c_int32), ("n_samples_tdyn", C.c_int32),
                ("ns_max", C.c_int32), ("recentre", C.c_int32), ("retune", C.c_int32),
                ("pad", C.c_int32), ("alpha_min", C.c_double)]


class CCadenceState(C.Structure):
    _fields_ = [("since", C.c_int32), ("pad", C.c_int32), ("nbound", C.c_int64), ("rx", C.c_double),
                ("rhm", C.c_double), ("mbound", C.c_double)]


class CIntervalLog(C.Structure):
    _fields_ = [("dt_int", C.c_double), ("nsub", C.c_int32), ("nsamples", C.c_int32),
                ("complete", C.c_int32), ("pad", C.c_int32), ("nbound", C.c_int64),
                ("nchanged", C.c_int64), ("rx", C.c_double), ("rhm", C.c_double),
                ("mbound", C.c_double), ("dx", C.c_double * 3), ("dv", C.c_double * 3),
                ("alpha", C.c_double), ("b", C.c_double)]


MAX_SAMPLES = 16


def paper_c_dyn():
    """c_dyn of the paper's t_dyn (scf_cadence_defaults)."""
    c = CCadence()
    lib().scf_cadence_defaults(C.byref(c))
    return c.c_dyn


@dataclass
class Cadence:
    """Parameters of the refresh cadence (include/scf.h, scf_cadence); c_dyn =
    None takes the library's value of the paper's t_dyn."""
    eta: float = 1.0 / 400.0
    dt_max: float = 0.005
    frac: float = 0.999
    refresh_every: int = 5
    n_samples_tdyn: int = 0
    c_dyn: float = None
    ns_max: int = 8
    recentre: bool = False
    retune: bool = False
    alpha_min: float = 0.25

    def c(self):
        c_dyn = paper_c_dyn() if self.c_dyn is None else self.c_dyn
        return CCadence(float(self.eta), float(self.dt_max), float(self.frac), float(c_dyn),
                        int(self.refresh_every), int(self.n_samples_tdyn), int(self.ns_max),
                        1 if self.recentre else 0, 1 if self.retune else 0, 0,
                        float(self.alpha_min))


def _state_dict(st):
    return {"since": st.since, "nbound": st.nbound, "rx": st.rx, "rhm": st.rhm, "mbound": st.mbound}


_lib = None

# exported functions: name -> (restype, argtypes)
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
SIGNATURES = {
    "scf_ncoef": (C.c_int64, [C.c_int32, C.c_int32]),
    "scf_plan_create": (C.c_int, [C.POINTER(_vp), C.POINTER(CBasis), C.c_int32, C.c_uint32]),
    "scf_plan_destroy": (None, [_vp]),
    "scf_workspace_size": (C.c_int, [_vp, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "scf_coeffs": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "scf_forces": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, C.POINTER(CHost), _dp, _vp, _vp,
                             _vp, _vp, _vp, C.c_size_t, _vp]),
    "scf_step": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                           C.c_uint32, C.POINTER(CHost), _dp, C.c_double, C.c_int32, _vp, _vp,
                           C.c_size_t, _vp]),
    "scf_plan_weights_size": (C.c_int64, [_vp]),
    "scf_step_keep_weights": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                        _vp, _vp, C.c_uint32, C.POINTER(CHost), _dp, C.c_double,
                                        C.c_int32, _vp, _vp, _vp, C.c_size_t, _vp]),
    "scf_noalloc_scratch_bytes": (C.c_size_t, []),
    "scf_step_noalloc": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, C.c_uint32, C.POINTER(CHost), _dp, C.c_double, C.c_int32,
                                   _vp, _vp]),
    "scf_step_batched": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int64), _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _vp, _vp, _vp, C.c_uint32, C.POINTER(CHost), _dp,
                                   C.c_double, C.c_int32, _vp, _vp, C.c_size_t, _vp]),
    "scf_step_adjoint": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   C.POINTER(CHost), _dp, C.c_double, C.c_int32, C.POINTER(_vp),
                                   _dp, _dp, _vp, _vp, C.c_size_t, _vp]),
    "scf_adjoint_workspace_size": (C.c_int, [_vp, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "scf_plan_num_variants": (C.c_int32, [_vp]),
    "scf_plan_variant": (C.c_int32, [_vp]),
    "scf_plan_graph_captures": (C.c_int32, [_vp]),
    "scf_plan_set_variant": (C.c_int, [_vp, C.c_int32]),
    "scf_plan_coef_units_div": (C.c_int32, [_vp]),
    "scf_plan_set_coef_units_div": (C.c_int, [_vp, C.c_int32]),
    "scf_plan_describe": (C.c_char_p, [_vp]),
    "scf_autotune": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp, _dp]),
    "scf_plan_num_field_variants": (C.c_int32, [_vp]),
    "scf_plan_field_variant": (C.c_int32, [_vp]),
    "scf_plan_set_field_variant": (C.c_int, [_vp, C.c_int32]),
    "scf_autotune_field": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                     C.c_size_t, _vp, _dp]),
    "scf_power_spectrum": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp]),
    "scf_tidal_norm": (C.c_int, [C.POINTER(CHost), _dp, _dp]),
    "scf_cadence_defaults": (None, [C.c_void_p]),
    "scf_cadence_workspace_size": (C.c_int, [_vp, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "scf_step_frozen": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                  C.c_uint32, _vp, C.POINTER(CHost), _dp, C.c_double, C.c_int32,
                                  _vp, C.c_size_t, _vp]),
    "scf_select": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_double,
                             _vp, _vp, C.POINTER(CCadenceState), _vp, C.c_size_t, _vp]),
    "scf_coeffs_delta": (C.c_int, [_vp, C.c_int64, C.c_int32, C.POINTER(_vp), _vp, _vp, _vp,
                                   C.POINTER(C.c_int64), _vp, C.c_size_t, _vp]),
    "scf_cadence_init": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_double,
                                   _vp, _vp, C.POINTER(CCadenceState), _vp, C.c_size_t, _vp]),
    "scf_evolve": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                             C.POINTER(CHost), _dp, C.POINTER(CCadence), C.c_int32, _vp, _vp,
                             C.POINTER(CCadenceState), C.POINTER(CIntervalLog), _vp, C.c_size_t,
                             _vp]),
    "scf_density": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp]),
    "scf_core": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _dp, _vp,
                           C.c_size_t, _vp]),
    "scf_recentre": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, _dp, C.c_double, C.c_int32,
                               C.POINTER(C.c_int32), _vp, C.c_size_t, _vp]),
    "scf_tune_basis": (C.c_int, [_vp, C.c_int64, _vp, _vp, _vp, _vp, C.c_double, _dp, _dp, _vp,
                                 C.c_size_t, _vp]),
    "scf_plan_set_basis": (C.c_int, [_vp, C.c_double, C.c_double]),
    "scf_plan_get_basis": (C.c_int, [_vp, C.POINTER(CBasis)]),
    "scf_profile_enable": (C.c_int, [_vp, C.c_int32]),
    "scf_profile_read": (C.c_int, [_vp, C.c_void_p]),
    "scf_kernel_name": (C.c_char_p, [C.c_int32]),
    "scf_bench_ceiling": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _vp, _dp, _dp]),
    "scf_status_string": (C.c_char_p, [C.c_int]),
    "scf_last_error": (C.c_char_p, []),
}


def lib():
    """Load libscf.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libscf.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise ScfError(status, lib().scf_last_error().decode())


def bench_ceiling(kind, waves_per_simd, iters=20000):
    """scf_bench_ceiling: (TFLOP/s, ms) of a throughput microbenchmark
    (kind 0/1: FP32 FMA chains, 2/3/4: FP32 MFMA 4x4x1 / 16x16x4 / 32x32x2,
    5: kinds 0 and 2 together in every wave)."""
    torch = _torch()
    scratch = torch.empty(8 * 4096, dtype=torch.float32, device="cuda")
    tf = C.c_double()
    ms = C.c_double()
    torch.cuda.synchronize()
    _check(lib().scf_bench_ceiling(int(kind), int(waves_per_simd), int(iters), _ptr(scratch),
                                   C.byref(tf), C.byref(ms)))
    return tf.value, ms.value


def ncoef(nmax, lmax):
    return int(lib().scf_ncoef(nmax, lmax))


def make_host(components, G=1.0):
    """components: list of (kind, params) with kind a name or integer."""
    h = CHost()
    if components is None:
        return h
    if len(components) > MAX_HOST_COMP:
        raise ValueError("too many host components")
    h.ncomp = len(components)
    h.G = float(G)
    for i, (kind, params) in enumerate(components):
        h.comp[i].kind = HOST_KINDS[kind] if isinstance(kind, str) else int(kind)
        pp = list(params) + [0.0] * (3 - len(params))
        for k in range(3):
            h.comp[i].p[k] = float(pp[k])
    return h


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def tidal_norm(host, pos):
    """Frobenius norm of the host's tidal tensor at pos (3,), host = (components, G)."""
    h = make_host(host[0], host[1])
    p = (C.c_double * 3)(*[float(v) for v in pos[:3]])
    out = C.c_double(0.0)
    _check(lib().scf_tidal_norm(C.byref(h), C.cast(p, _dp), C.byref(out)))
    return out.value


class Plan:
    """An SCF plan: basis tables and kernels for one (basis, dtype)."""

    def __init__(self, nmax, lmax, alpha=1.0, b=1.0, G=1.0, dtype="f32"):
        self.nmax, self.lmax = int(nmax), int(lmax)
        self.alpha, self.b, self.G = float(alpha), float(b), float(G)
        self.dtype = F32 if dtype in ("f32", "float32", F32) else F64
        self.basis = CBasis(self.nmax, self.lmax, self.alpha, self.b, self.G)
        self._h = C.c_void_p()
        _check(lib().scf_plan_create(C.byref(self._h), C.byref(self.basis), self.dtype, 0))
        self.T = ncoef(self.nmax, self.lmax)
        self._ws = None

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float32 if self.dtype == F32 else torch.float64

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _lib is not None:
            _lib.scf_plan_destroy(h)
            self._h = None

    @property
    def num_variants(self):
        return int(lib().scf_plan_num_variants(self._h))

    @property
    def variant(self):
        return int(lib().scf_plan_variant(self._h))

    @variant.setter
    def variant(self, v):
        _check(lib().scf_plan_set_variant(self._h, int(v)))

    def describe(self):
        return lib().scf_plan_describe(self._h).decode()

    @property
    def coef_units_div(self):
        return int(lib().scf_plan_coef_units_div(self._h))

    @coef_units_div.setter
    def coef_units_div(self, d):
        _check(lib().scf_plan_set_coef_units_div(self._h, int(d)))

    @property
    def field_variant(self):
        return int(lib().scf_plan_field_variant(self._h))

    @field_variant.setter
    def field_variant(self, v):
        _check(lib().scf_plan_set_field_variant(self._h, int(v)))

    @property
    def num_field_variants(self):
        return int(lib().scf_plan_num_field_variants(self._h))

    def autotune(self, x, y, z, m, field=True):
        """Time the coefficient-kernel variants (and, with field=True, the
        field-kernel variants) on these particles; keep the fastest.
        Returns (coefficient variant, its ms)."""
        torch = _torch()
        self._check_arrays(x, y, z, m)
        ws = self.workspace(x.numel(), device=x.device)
        best = C.c_double(0.0)
        _check(lib().scf_autotune(self._h, x.numel(), _ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(ws),
                                  ws.numel(), _stream(), C.byref(best)))
        if field:
            a = [torch.empty_like(x) for _ in range(3)]
            fbest = C.c_double(0.0)
            _check(lib().scf_autotune_field(self._h, x.numel(), _ptr(x), _ptr(y), _ptr(z), _ptr(m),
                                            *[_ptr(t) for t in a], _ptr(ws), ws.numel(), _stream(),
                                            C.byref(fbest)))
        return self.variant, best.value

    def profile(self, enable=True):
        """Turn per-kernel HIP-event timing on or off."""
        _check(lib().scf_profile_enable(self._h, 1 if enable else 0))

    def kernel_times(self):
        """{kernel name: (launches, total ms)} since the last call."""
        arr = (CKernelTime * KERNEL_KINDS)()
        _check(lib().scf_profile_read(self._h, C.cast(arr, C.c_void_p)))
        return {lib().scf_kernel_name(k).decode(): (arr[k].count, arr[k].total_ms)
                for k in range(KERNEL_KINDS) if arr[k].count}

    def workspace(self, n, nclusters=1, device=None):
        torch = _torch()
        need = C.c_size_t()
        _check(lib().scf_workspace_size(self._h, int(n), int(nclusters), C.byref(need)))
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = torch.empty(max(need.value, 256), dtype=torch.uint8,
                                   device=device or torch.device("cuda"))
        return self._ws

    def _check_arrays(self, *ts):
        for t in ts:
            if t is None:
                continue
            if t.dtype != self.torch_dtype or not t.is_cuda or not t.is_contiguous():
                raise TypeError(f"expected contiguous {self.torch_dtype} CUDA tensors")

    def coeffs(self, x, y, z, m, out=None):
        torch = _torch()
        self._check_arrays(x, y, z, m)
        n = x.numel()
        if out is None:
            out = torch.empty(self.T, dtype=torch.float64, device=x.device)
        ws = self.workspace(n, device=x.device)
        _check(lib().scf_coeffs(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(out),
                                _ptr(ws), ws.numel(), _stream()))
        return out

    def forces(self, x, y, z, coef, host=None, centre=None, pot=False, out=None):
        """Accelerations (and the potential with pot=True) at x, y, z; out =
        (ax, ay, az[, pot]) names caller-owned output tensors."""
        torch = _torch()
        self._check_arrays(x, y, z)
        n = x.numel()
        if out is not None:
            ax, ay, az = out[:3]
            p = out[3] if pot else None
            self._check_arrays(x, ax, ay, az, *([p] if pot else []))
        else:
            ax, ay, az = (torch.empty_like(x) for _ in range(3))
            p = torch.empty_like(x) if pot else None
        h = make_host(host[0], host[1]) if host is not None else None
        cen = (C.c_double * 3)(*[float(v) for v in centre[:3]]) if centre is not None else None
        ws = self.workspace(n, device=x.device)
        _check(lib().scf_forces(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(coef),
                                C.byref(h) if h is not None else None,
                                C.cast(cen, _dp) if cen is not None else None, _ptr(ax),
                                _ptr(ay), _ptr(az), _ptr(p), _ptr(ws), ws.numel(), _stream()))
        return (ax, ay, az, p) if pot else (ax, ay, az)

    @property
    def weights_size(self):
        """Elements of one force-weight row (see step's w_hist)."""
        return int(lib().scf_plan_weights_size(self._h))

    def step(self, st, m, dt, nsteps, host=None, centre=None, acc=None, coef_last=None,
             w_hist=None):
        """Advance st = [x, y, z, vx, vy, vz] in place.  acc = [ax, ay, az]
        (in/out; pass the previous call's to skip the start-up evaluation).
        w_hist (a contiguous device tensor of the plan's real type with at least
        (nsteps + 1) * weights_size elements) keeps the force weights of every
        kick for step_adjoint (scf_step_keep_weights).  Returns (centre (6,)
        numpy, acc)."""
        torch = _torch()
        self._check_arrays(*st, m)
        n = st[0].numel()
        acc_valid = acc is not None
        if acc is None:
            acc = [torch.empty_like(st[0]) for _ in range(3)]
        cen = (C.c_double * 6)(*[float(v) for v in (centre if centre is not None else np.zeros(6))])
        h = make_host(host[0], host[1]) if host is not None else None
        ws = self.workspace(n, device=st[0].device)
        common = (STEP_ACC_VALID if acc_valid else 0, C.byref(h) if h is not None else None,
                  C.cast(cen, _dp), float(dt), int(nsteps), _ptr(coef_last))
        if w_hist is None:
            _check(lib().scf_step(self._h, n, *[_ptr(t) for t in st], _ptr(m),
                                  *[_ptr(t) for t in acc], *common, _ptr(ws), ws.numel(),
                                  _stream()))
        else:
            self._check_weights(w_hist, nsteps, st[0])
            _check(lib().scf_step_keep_weights(self._h, n, *[_ptr(t) for t in st], _ptr(m),
                                               *[_ptr(t) for t in acc], *common, _ptr(w_hist),
                                               _ptr(ws), ws.numel(), _stream()))
        return np.array(cen[:]), acc

    def _check_weights(self, w_hist, nsteps, like):
        if (w_hist.dtype != like.dtype or not w_hist.is_cuda or not w_hist.is_contiguous()
                or w_hist.numel() < (int(nsteps) + 1) * self.weights_size):
            raise TypeError("w_hist must be a contiguous CUDA tensor of the plan's real type "
                            "with (nsteps + 1) * weights_size elements")

    def step_noalloc(self, st, m, dt, nsteps, host=None, centre=None, acc=None, coef_last=None):
        """step() through scf_step_noalloc: the library's static device scratch
        replaces the workspace, so nothing is allocated for it."""
        torch = _torch()
        self._check_arrays(*st, m)
        n = st[0].numel()
        acc_valid = acc is not None
        if acc is None:
            acc = [torch.empty_like(st[0]) for _ in range(3)]
        cen = (C.c_double * 6)(*[float(v) for v in (centre if centre is not None else np.zeros(6))])
        h = make_host(host[0], host[1]) if host is not None else None
        _check(lib().scf_step_noalloc(self._h, n, *[_ptr(t) for t in st], _ptr(m),
                                      *[_ptr(t) for t in acc], STEP_ACC_VALID if acc_valid else 0,
                                      C.byref(h) if h is not None else None, C.cast(cen, _dp),
                                      float(dt), int(nsteps), _ptr(coef_last), _stream()))
        return np.array(cen[:]), acc

    def adjoint_workspace(self, n, nsteps, device=None):
        torch = _torch()
        need = C.c_size_t()
        _check(lib().scf_adjoint_workspace_size(self._h, int(n), int(nsteps), C.byref(need)))
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = torch.empty(max(need.value, 256), dtype=torch.uint8,
                                   device=device or torch.device("cuda"))
        return self._ws

    def step_adjoint(self, st0, m, dt, nsteps, lam, lam_centre, host=None, centre0=None,
                     w_hist=None):
        """Reverse mode of step() over nsteps steps starting from the synchronised
        state st0 = [x, y, z, vx, vy, vz] (not modified).  lam: 6 device tensors
        holding dL/d(final state), overwritten with dL/d(initial state).
        lam_centre: (6,) dL/d(final R, V).  w_hist: the force weights that
        step(st0, ..., w_hist=) kept for this segment (then the recompute skips
        the coefficient passes), or None.  Returns (dL/d(initial R, V) (6,),
        dL/d(host parameters) (ncomp, 3))."""
        self._check_arrays(*st0, m, *lam)
        if w_hist is not None:
            self._check_weights(w_hist, nsteps, st0[0])
        n = st0[0].numel()
        h = make_host(host[0], host[1]) if host is not None else None
        ncomp = h.ncomp if h is not None else 0
        cen = (C.c_double * 6)(*[float(v) for v in (centre0 if centre0 is not None else np.zeros(6))])
        lc = (C.c_double * 6)(*[float(v) for v in lam_centre])
        gh = (C.c_double * max(3 * ncomp, 1))()
        lp = (C.c_void_p * 6)(*[t.data_ptr() for t in lam])
        ws = self.adjoint_workspace(n, nsteps, device=st0[0].device)
        _check(lib().scf_step_adjoint(self._h, n, *[_ptr(t) for t in st0], _ptr(m),
                                      C.byref(h) if h is not None else None, C.cast(cen, _dp),
                                      float(dt), int(nsteps), C.cast(lp, C.POINTER(C.c_void_p)),
                                      C.cast(lc, _dp), C.cast(gh, _dp), _ptr(w_hist), _ptr(ws),
                                      ws.numel(), _stream()))
        return np.array(lc[:]), np.array(gh[:3 * ncomp]).reshape(ncomp, 3)

    def power(self, coef):
        """E_l = sum_{n,m} |a_nlm|^2 of one coefficient vector (or of a batch,
        shape (nclusters, ncoef)); returns a device tensor (..., lmax + 1)."""
        torch = _torch()
        c = coef.reshape(-1, self.T)
        if c.dtype != torch.float64 or not c.is_cuda or not c.is_contiguous():
            raise TypeError("expected a contiguous float64 CUDA tensor")
        out = torch.empty(c.shape[0], self.lmax + 1, dtype=torch.float64, device=c.device)
        _check(lib().scf_power_spectrum(self._h, c.shape[0], _ptr(c), _ptr(out), _stream()))
        return out.reshape(*coef.shape[:-1], self.lmax + 1)

    @property
    def graph_captures(self):
        return int(lib().scf_plan_graph_captures(self._h))

    def step_batched(self, offsets, st, m, dt, nsteps, host=None, centres=None, acc=None,
                     coef_last=None, graph=False):
        """Advance nclusters clusters concatenated in st = [x, y, z, vx, vy, vz]
        (cluster c owns [offsets[c], offsets[c+1])) in place.  centres: (nclusters, 6).
        graph=True replays the middle steps from HIP graphs (bitwise the same
        results; direct launches are faster on the MI355X).
        Returns (centres (nclusters, 6) numpy, acc)."""
        torch = _torch()
        self._check_arrays(*st, m)
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        ncl = len(off) - 1
        n = int(off[-1])
        if st[0].numel() < n:
            raise ValueError("particle arrays shorter than offsets[-1]")
        acc_valid = acc is not None
        if acc is None:
            acc = [torch.empty_like(st[0]) for _ in range(3)]
        cen = np.zeros((ncl, 6)) if centres is None else np.array(centres, dtype=np.float64)
        cen = np.ascontiguousarray(cen.reshape(ncl, 6))
        h = make_host(host[0], host[1]) if host is not None else None
        ws = self.workspace(n, nclusters=ncl, device=st[0].device)
        flags = (STEP_ACC_VALID if acc_valid else 0) | (STEP_GRAPH if graph else 0)
        _check(lib().scf_step_batched(self._h, ncl, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                      *[_ptr(t) for t in st], _ptr(m), *[_ptr(t) for t in acc],
                                      flags, C.byref(h) if h is not None else None,
                                      cen.ctypes.data_as(_dp), float(dt), int(nsteps),
                                      _ptr(coef_last), _ptr(ws), ws.numel(), _stream()))
        return cen, acc

    # ---- refresh cadence (Sec. 2.2) -----------------------------------------
    def cadence_workspace(self, n, ns_max=1, device=None):
        torch = _torch()
        need = C.c_size_t()
        _check(lib().scf_cadence_workspace_size(self._h, int(n), int(ns_max), C.byref(need)))
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = torch.empty(max(need.value, 256), dtype=torch.uint8,
                                   device=device or torch.device("cuda"))
        return self._ws

    def step_frozen(self, st, coef, dt, nsteps, host=None, centre=None, acc=None):
        """Advance st = [x, y, z, vx, vy, vz] in place in the frozen potential
        of coef (+ the host's differential field).  Returns (centre, acc)."""
        torch = _torch()
        self._check_arrays(*st)
        n = st[0].numel()
        acc_valid = acc is not None
        if acc is None:
            acc = [torch.empty_like(st[0]) for _ in range(3)]
        cen = (C.c_double * 6)(*[float(v) for v in (centre if centre is not None else np.zeros(6))])
        h = make_host(host[0], host[1]) if host is not None else None
        ws = self.workspace(n, device=st[0].device)
        _check(lib().scf_step_frozen(self._h, n, *[_ptr(t) for t in st], *[_ptr(t) for t in acc],
                                     STEP_ACC_VALID if acc_valid else 0, _ptr(coef),
                                     C.byref(h) if h is not None else None, C.cast(cen, _dp),
                                     float(dt), int(nsteps), _ptr(ws), ws.numel(), _stream()))
        return np.array(cen[:]), acc

    def select(self, st, m, coef, frac=0.999, bound=False):
        """Selection in the potential of coef: returns (w, bound flags or None,
        {nbound, rx, rhm, mbound})."""
        torch = _torch()
        self._check_arrays(*st, m)
        n = st[0].numel()
        w = torch.empty_like(m)
        b = torch.empty(n, dtype=torch.uint8, device=m.device) if bound else None
        out = CCadenceState()
        ws = self.cadence_workspace(n, 1, device=m.device)
        _check(lib().scf_select(self._h, n, *[_ptr(t) for t in st], _ptr(m), _ptr(coef),
                                float(frac), _ptr(w), _ptr(b), C.byref(out), _ptr(ws), ws.numel(),
                                _stream()))
        d = _state_dict(out)
        del d["since"]
        return w, b, d

    def escaped(self, st, m):
        """Escapers of st in the potential of the particles' own coefficients
        (|v|^2/2 + psi_SCF >= 0, cluster frame): the complement of
        scf_select's bound flags, as a device bool tensor."""
        coef = self.coeffs(st[0], st[1], st[2], m)
        _, b, _ = self.select([t.contiguous() for t in st], m, coef, 1.0, bound=True)
        return b == 0

    def coeffs_delta(self, snaps, w_old, w_new, coef):
        """coef += mean over snapshots [(x, y, z), ...] of the coefficients of
        the particles whose weight changed, weights w_new - w_old (in place).
        Returns the number of changed particles."""
        flat = [t for xyz in snaps for t in xyz]
        self._check_arrays(*flat, w_old, w_new)
        n = w_old.numel()
        arr = (C.c_void_p * len(flat))(*[t.data_ptr() for t in flat])
        nch = C.c_int64()
        ws = self.cadence_workspace(n, len(snaps), device=w_old.device)
        _check(lib().scf_coeffs_delta(self._h, n, len(snaps), C.cast(arr, C.POINTER(C.c_void_p)),
                                      _ptr(w_old), _ptr(w_new), _ptr(coef), C.byref(nch), _ptr(ws),
                                      ws.numel(), _stream()))
        return int(nch.value)

    def cadence_init(self, st, m, frac=0.999):
        """Start of a cadence: returns (coef, w, state dict)."""
        torch = _torch()
        self._check_arrays(*st, m)
        n = st[0].numel()
        coef = torch.empty(self.T, dtype=torch.float64, device=m.device)
        w = torch.empty_like(m)
        cs = CCadenceState()
        ws = self.cadence_workspace(n, 1, device=m.device)
        _check(lib().scf_cadence_init(self._h, n, *[_ptr(t) for t in st], _ptr(m), float(frac),
                                      _ptr(coef), _ptr(w), C.byref(cs), _ptr(ws), ws.numel(),
                                      _stream()))
        return coef, w, _state_dict(cs)

    def evolve(self, st, m, nint, cadence, host, centre, coef, w, state, acc=None):
        """nint intervals of the cadence; st, coef and w are updated in place.
        Returns (centre (6,), state dict, log list of dicts)."""
        torch = _torch()
        self._check_arrays(*st, m, w)
        n = st[0].numel()
        if acc is None:
            acc = [torch.empty_like(st[0]) for _ in range(3)]
        cen = (C.c_double * 6)(*[float(v) for v in centre])
        h = make_host(host[0], host[1])
        cs = CCadenceState(int(state["since"]), 0, int(state["nbound"]), float(state["rx"]),
                           float(state["rhm"]), float(state["mbound"]))
        logs = (CIntervalLog * max(int(nint), 1))()
        cad = cadence.c()
        ws = self.cadence_workspace(n, cadence.ns_max, device=m.device)
        _check(lib().scf_evolve(self._h, n, *[_ptr(t) for t in st], _ptr(m),
                                *[_ptr(t) for t in acc], C.byref(h), C.cast(cen, _dp),
                                C.byref(cad), int(nint), _ptr(coef), _ptr(w), C.byref(cs),
                                C.cast(logs, C.POINTER(CIntervalLog)), _ptr(ws), ws.numel(),
                                _stream()))
        log = [{"dt_int": e.dt_int, "nsub": e.nsub, "nsamples": e.nsamples,
                "kind": "complete" if e.complete else "intermediate", "nbound": e.nbound,
                "nchanged": e.nchanged, "rx": e.rx, "rhm": e.rhm, "mbound": e.mbound,
                "dx": np.array(e.dx[:]), "dv": np.array(e.dv[:]), "alpha": e.alpha, "b": e.b}
               for e in logs[:int(nint)]]
        self._sync_basis()
        return np.array(cen[:]), _state_dict(cs), log

    def density(self, x, y, z, coef):
        """rho_SCF (Eq. total_dens) at the points (device tensor)."""
        torch = _torch()
        self._check_arrays(x, y, z)
        n = x.numel()
        rho = torch.empty_like(x)
        ws = self.cadence_workspace(n, 1, device=x.device)
        _check(lib().scf_density(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(coef), _ptr(rho),
                                 _ptr(ws), ws.numel(), _stream()))
        return rho

    def core(self, st, m, w, coef):
        """Core radius and velocity (Sec. 2.1) over the particles with w > 0:
        returns (r_core, v_core (3,), core mass)."""
        self._check_arrays(*st, m, w)
        n = m.numel()
        out = (C.c_double * 5)()
        ws = self.cadence_workspace(n, 1, device=m.device)
        _check(lib().scf_core(self._h, n, *[_ptr(t) for t in st], _ptr(m), _ptr(w), _ptr(coef),
                              C.cast(out, _dp), _ptr(ws), ws.numel(), _stream()))
        return out[0], np.array(out[1:4]), out[4]

    def recentre(self, x, y, z, w, centre=(0.0, 0.0, 0.0), tol=1e-6, maxit=100):
        """Frame centre (Sec. 2.1): the a_000 maximum of the particles with
        w > 0, searched from centre.  Returns (centre (3,), steps)."""
        self._check_arrays(x, y, z, w)
        n = x.numel()
        c = (C.c_double * 3)(*[float(v) for v in centre])
        steps = C.c_int32()
        ws = self.cadence_workspace(n, 1, device=x.device)
        _check(lib().scf_recentre(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(w), C.cast(c, _dp),
                                  float(tol), int(maxit), C.byref(steps), _ptr(ws), ws.numel(),
                                  _stream()))
        return np.array(c[:]), int(steps.value)

    def _sync_basis(self):
        b = CBasis()
        _check(lib().scf_plan_get_basis(self._h, C.byref(b)))
        self.basis = b
        self.alpha, self.b = float(b.alpha), float(b.b)

    def set_basis(self, alpha, b):
        """Replace the plan's alpha and b (tables recomputed)."""
        _check(lib().scf_plan_set_basis(self._h, float(alpha), float(b)))
        self._sync_basis()

    def tune_basis(self, x, y, z, w, alpha_min=0.25, start=None):
        """(alpha, b) maximising a_000 of the particles with w > 0 about the
        origin, and that maximum; the plan is not changed."""
        self._check_arrays(x, y, z, w)
        n = x.numel()
        ab = (C.c_double * 2)(*(start if start is not None else (self.alpha, self.b)))
        val = C.c_double()
        ws = self.cadence_workspace(n, 1, device=x.device)
        _check(lib().scf_tune_basis(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(w),
                                    float(alpha_min), C.cast(ab, _dp), C.byref(val), _ptr(ws),
                                    ws.numel(), _stream()))
        return float(ab[0]), float(ab[1]), float(val.value)
