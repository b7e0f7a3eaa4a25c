"""ctypes wrapper of the FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library; the two agree only through the documented coefficient
layout and the paper's definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "scf_oracle.c")

HOST_LOG, HOST_HERNQUIST, HOST_NFW, HOST_MN, HOST_PLUMMER = 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no hand intrinsics)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Basis(C.Structure):
    _fields_ = [("nmax", C.c_int32), ("lmax", C.c_int32), ("alpha", C.c_double),
                ("b", C.c_double), ("G", C.c_double)]


class Comp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("p", C.c_double * 3)]


class Host(C.Structure):
    _fields_ = [("ncomp", C.c_int32), ("pad", C.c_int32), ("G", C.c_double), ("comp", Comp * 8)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_num_threads.restype = C.c_int32
        L.orc_num_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_ncoef.restype = C.c_int64
        L.orc_ncoef.argtypes = [C.c_int32, C.c_int32]
        L.orc_gegenbauer.restype = C.c_double
        L.orc_gegenbauer.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_radial_raw.argtypes = [C.c_double, C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.orc_energy_inner.restype = C.c_double
        L.orc_energy_inner.argtypes = [C.POINTER(Basis), C.c_int32, C.c_int32, C.c_int32]
        L.orc_norms.argtypes = [C.POINTER(Basis), dp]
        L.orc_radial.argtypes = [C.POINTER(Basis), C.c_int32, C.c_double, dp, dp]
        L.orc_ylm.argtypes = [C.c_int32, C.c_double, C.c_double, dp, dp]
        L.orc_coeffs.restype = C.c_int
        L.orc_coeffs.argtypes = [C.POINTER(Basis), C.c_int64, dp, dp, dp, dp, dp]
        L.orc_field.restype = C.c_int
        L.orc_field.argtypes = [C.POINTER(Basis), dp, C.c_int64, dp, dp, dp, dp, dp, dp, dp]
        L.orc_host_eval.argtypes = [C.POINTER(Host), dp, dp, dp, dp]
        L.orc_host_dgrad_dparam.argtypes = [C.POINTER(Host), dp, dp]
        L.orc_power.argtypes = [C.c_int32, C.c_int32, dp, dp]
        L.orc_tidal_norm.restype = C.c_double
        L.orc_tidal_norm.argtypes = [C.POINTER(Host), dp]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.POINTER(Basis), C.POINTER(Host), C.c_int64, dp, dp, dp, dp, dp,
                               dp, dp, dp, C.c_double, C.c_int32, dp, dp]
        L.orc_step_frozen.restype = C.c_int
        L.orc_step_frozen.argtypes = [C.POINTER(Basis), C.POINTER(Host), C.c_int64, dp, dp, dp,
                                      dp, dp, dp, dp, dp, C.c_double, C.c_int32]
        L.orc_orbit.restype = C.c_int
        L.orc_orbit.argtypes = [C.POINTER(Host), dp, C.c_double, C.c_int32, dp]
        L.orc_step_batched.restype = C.c_int
        L.orc_step_batched.argtypes = [C.POINTER(Basis), C.POINTER(Host), C.c_int32,
                                       C.POINTER(C.c_int64), dp, dp, dp, dp, dp, dp, dp, dp,
                                       C.c_double, C.c_int32, dp]
        L.orc_step_adjoint.restype = C.c_int
        L.orc_step_adjoint.argtypes = [C.POINTER(Basis), C.POINTER(Host), C.c_int64, dp, dp, dp,
                                       dp, dp, dp, dp, dp, C.c_double, C.c_int32, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def basis(nmax, lmax, alpha=1.0, b=1.0, G=1.0):
    return Basis(int(nmax), int(lmax), float(alpha), float(b), float(G))


def host(components, G=1.0):
    """components: list of (kind, (p0, p1, p2))."""
    h = Host()
    h.ncomp = len(components)
    h.G = float(G)
    for i, (kind, params) in enumerate(components):
        h.comp[i].kind = int(kind)
        pp = list(params) + [0.0] * (3 - len(params))
        for k in range(3):
            h.comp[i].p[k] = float(pp[k])
    return h


def set_threads(n):
    lib().orc_set_threads(int(n))


def num_threads():
    return int(lib().orc_num_threads())


def ncoef(nmax, lmax):
    return int(lib().orc_ncoef(nmax, lmax))


def gegenbauer(n, lam, x):
    return lib().orc_gegenbauer(int(n), float(lam), float(x))


def radial_raw(alpha, l, nmax, s):
    f = np.zeros(nmax + 1)
    df = np.zeros(nmax + 1)
    lib().orc_radial_raw(float(alpha), int(l), int(nmax), float(s), _p(f), _p(df))
    return f, df


def energy_inner(B, l, n1, n2):
    return lib().orc_energy_inner(C.byref(B), int(l), int(n1), int(n2))


def norms(B):
    N = np.zeros((B.nmax + 1) * (B.lmax + 1))
    lib().orc_norms(C.byref(B), _p(N))
    return N.reshape(B.nmax + 1, B.lmax + 1)


def radial(B, l, r):
    U = np.zeros(B.nmax + 1)
    dU = np.zeros(B.nmax + 1)
    lib().orc_radial(C.byref(B), int(l), float(r), _p(U), _p(dU))
    return U, dU


def ylm(lmax, theta, phi):
    k = (lmax + 1) * (lmax + 2) // 2
    re = np.zeros(k)
    im = np.zeros(k)
    lib().orc_ylm(int(lmax), float(theta), float(phi), _p(re), _p(im))
    return re + 1j * im


def coeffs(B, x, y, z, m):
    x, y, z, m = map(_f64, (x, y, z, m))
    out = np.zeros(ncoef(B.nmax, B.lmax))
    rc = lib().orc_coeffs(C.byref(B), len(x), _p(x), _p(y), _p(z), _p(m), _p(out))
    assert rc == 0
    return out


def field(B, coef, x, y, z, pot=True, acc=True):
    x, y, z, coef = map(_f64, (x, y, z, coef))
    n = len(x)
    P = np.zeros(n) if pot else None
    gx = np.zeros(n) if acc else None
    gy = np.zeros(n) if acc else None
    gz = np.zeros(n) if acc else None
    rc = lib().orc_field(C.byref(B), _p(coef), n, _p(x), _p(y), _p(z), _p(P), _p(gx), _p(gy),
                         _p(gz))
    assert rc == 0
    return P, (np.stack([gx, gy, gz]) if acc else None)


def density_scale(B):
    """K_nl = [n(n + 2 lambda_l) + p_l (p_l + 1)] / alpha^2, p_l = alpha (2l+1),
    lambda_l = p_l + 1/2, per stored coefficient: the radial Laplacian of
    s^l (1 + s^(1/alpha))^(-p) C_n^lambda(xi) is -K_nl s^(1/alpha - 2)
    (1 + s^(1/alpha))^(-2) times that same function (from the Gegenbauer
    differential equation)."""
    L2 = (B.lmax + 1) ** 2
    K = np.zeros(ncoef(B.nmax, B.lmax))
    for n in range(B.nmax + 1):
        for l in range(B.lmax + 1):
            p = B.alpha * (2 * l + 1)
            lam = p + 0.5
            K[n * L2 + l * l: n * L2 + (l + 1) ** 2] = (n * (n + 2 * lam) + p * (p + 1)) / B.alpha ** 2
    return K


def density(B, coef, x, y, z):
    """rho_SCF = sum a_nlm D_n^l Y_l^m (Eq. total_dens), with the density basis
    D = nabla^2 U / (4 pi G): rho = -s^(1/alpha-2) (1 + s^(1/alpha))^(-2)
    / (4 pi G b^2) times the potential of the coefficients K_nl a_nlm."""
    x, y, z = map(_f64, (x, y, z))
    pot, _ = field(B, np.asarray(coef, dtype=np.float64) * density_scale(B), x, y, z, acc=False)
    s = np.sqrt(x * x + y * y + z * z) / B.b
    t = s ** (1.0 / B.alpha)
    return -(s ** (1.0 / B.alpha - 2.0)) / (1.0 + t) ** 2 / (4.0 * np.pi * B.G * B.b ** 2) * pot


def core(B, coef, state, m, w):
    """Frame velocity of Sec. 2.1 over the particles with w > 0:
    r_core = sqrt(sum rho^2 r^2 / sum rho^2) with rho = rho_SCF at each, and
    the mass-weighted mean velocity of those with r <= r_core.
    Returns (r_core, v_core (3,), core mass)."""
    st = np.asarray(state, dtype=np.float64)
    sel = np.asarray(w) > 0
    rho = density(B, coef, st[0], st[1], st[2])
    r2 = (st[:3] ** 2).sum(0)
    q = rho[sel] ** 2
    rc2 = (q * r2[sel]).sum() / q.sum()
    inc = sel & (r2 <= rc2)
    mm = np.asarray(m, dtype=np.float64)[inc]
    v = (st[3:, inc] * mm).sum(1) / mm.sum()
    return float(np.sqrt(rc2)), v, float(mm.sum())


def host_eval(H, pos):
    pos = _f64(pos)
    pot = np.zeros(1)
    g = np.zeros(3)
    hs = np.zeros(9)
    lib().orc_host_eval(C.byref(H), _p(pos), _p(pot), _p(g), _p(hs))
    return pot[0], g, hs.reshape(3, 3)


def host_dgrad_dparam(H, pos):
    pos = _f64(pos)
    out = np.zeros(H.ncomp * 9)
    lib().orc_host_dgrad_dparam(C.byref(H), _p(pos), _p(out))
    return out.reshape(H.ncomp, 3, 3)


def power(nmax, lmax, coef):
    """E_l = sum_{n,m} |a_nlm|^2, l = 0..lmax."""
    coef = _f64(coef)
    El = np.zeros(lmax + 1)
    lib().orc_power(int(nmax), int(lmax), _p(coef), _p(El))
    return El


def tidal_norm(H, pos):
    return float(lib().orc_tidal_norm(C.byref(H), _p(_f64(np.asarray(pos, dtype=np.float64)))))


def step(B, H, state, m, centre, dt, nsteps, want_acc=False):
    """state: (6, n) array x,y,z,vx,vy,vz (copied); centre: (6,) R,V (copied)."""
    st = np.array(state, dtype=np.float64, copy=True)
    cen = _f64(np.array(centre, dtype=np.float64, copy=True))
    m = _f64(m)
    n = st.shape[1]
    coef = np.zeros(ncoef(B.nmax, B.lmax))
    acc = np.zeros(3 * n) if want_acc else None
    rows = [np.ascontiguousarray(st[i]) for i in range(6)]
    rc = lib().orc_step(C.byref(B), C.byref(H) if H is not None else None, n,
                        *[_p(r) for r in rows], _p(m), _p(cen), float(dt), int(nsteps),
                        _p(coef), _p(acc))
    assert rc == 0
    out = np.stack(rows)
    if want_acc:
        return out, cen, coef, acc.reshape(3, n)
    return out, cen, coef


def step_frozen(B, H, state, coef, centre, dt, nsteps):
    """KDK steps in the frozen potential of coef (+ host differential field);
    returns (state (6, n), centre (6,))."""
    st = np.array(state, dtype=np.float64, copy=True)
    rows = [np.ascontiguousarray(st[i]) for i in range(6)]
    cen = _f64(np.array(centre, dtype=np.float64, copy=True))
    rc = lib().orc_step_frozen(C.byref(B), C.byref(H) if H is not None else None, st.shape[1],
                               *[_p(r) for r in rows], _p(_f64(coef)), _p(cen), float(dt),
                               int(nsteps))
    assert rc == 0
    return np.stack(rows), cen


def orbit(H, centre, dt, nsteps):
    """Centre orbit in the host alone; returns the (nsteps+1, 6) trajectory."""
    cen = _f64(np.array(centre, dtype=np.float64, copy=True))
    traj = np.zeros((nsteps + 1) * 6)
    rc = lib().orc_orbit(C.byref(H) if H is not None else None, _p(cen), float(dt), int(nsteps),
                         _p(traj))
    assert rc == 0
    return traj.reshape(nsteps + 1, 6)


def step_batched(B, H, offsets, state, m, centres, dt, nsteps):
    st = np.array(state, dtype=np.float64, copy=True)
    rows = [np.ascontiguousarray(st[i]) for i in range(6)]
    cen = _f64(np.array(centres, dtype=np.float64, copy=True)).reshape(-1)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    ncl = len(off) - 1
    coef = np.zeros(ncl * ncoef(B.nmax, B.lmax))
    rc = lib().orc_step_batched(C.byref(B), C.byref(H) if H is not None else None, ncl,
                                off.ctypes.data_as(C.POINTER(C.c_int64)), *[_p(r) for r in rows],
                                _p(_f64(m)), _p(cen), float(dt), int(nsteps), _p(coef))
    assert rc == 0
    return np.stack(rows), cen.reshape(ncl, 6), coef.reshape(ncl, -1)


def step_adjoint(B, H, state0, m, centre0, dt, nsteps, lam, lam_centre):
    """Returns (lam0 (6,n), lam_centre0 (6,), grad_host (ncomp,3))."""
    st = np.array(state0, dtype=np.float64, copy=True)
    rows = [np.ascontiguousarray(st[i]) for i in range(6)]
    lam = _f64(np.array(lam, dtype=np.float64, copy=True)).reshape(-1)
    lc = _f64(np.array(lam_centre, dtype=np.float64, copy=True))
    nc = H.ncomp if H is not None else 0
    gh = np.zeros(max(nc, 1) * 3)
    rc = lib().orc_step_adjoint(C.byref(B), C.byref(H) if H is not None else None, st.shape[1],
                                *[_p(r) for r in rows], _p(_f64(m)), _p(_f64(centre0)),
                                float(dt), int(nsteps), _p(lam), _p(lc), _p(gh))
    assert rc == 0
    return lam.reshape(6, -1), lc, gh[: nc * 3].reshape(nc, 3) if nc else gh[:0].reshape(0, 3)
