"""ctypes wrapper of the plain FP64 CPU oracle (oracle/sph_oracle.cpp).

TEST INFRASTRUCTURE: only the tests, the smoke check and the bench's CPU
baseline use this module.  The GPU library never imports or links it, and it
never imports the GPU package.

Every function takes a `Params` from `sph_workloads` and numpy arrays in SoA
layout: d-vector fields have shape (dim, n) float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.cpp")
_LIB = os.path.join(_HERE, "libsph_oracle.so")

_d = ctypes.c_double
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_P = ctypes.c_void_p


class OrcParams(ctypes.Structure):
    _fields_ = [("dim", _i32), ("kernel", _i32), ("cell_div", _i32), ("brute", _i32),
                ("periodic", _i32 * 3), ("cell_order", _i32),
                ("h", _d), ("rho0", _d), ("c0", _d), ("nu", _d), ("eta", _d), ("dt", _d),
                ("g", _d * 3), ("lo", _d * 3), ("hi", _d * 3)]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no contraction, so sums are the plain ones)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_kernel_w.restype = _d
        L.orc_kernel_w.argtypes = [_P, _d]
        L.orc_kernel_dwdr.restype = _d
        L.orc_kernel_dwdr.argtypes = [_P, _d]
        L.orc_kernel_d2wdr2.restype = _d
        L.orc_kernel_d2wdr2.argtypes = [_P, _d]
        L.orc_grid.argtypes = [_P, _P, _P]
        L.orc_nkeys.restype = _i64
        L.orc_nkeys.argtypes = [_P]
        L.orc_cell_keys.argtypes = [_P, _i64, _P, _P]
        L.orc_bin_sort.argtypes = [_P, _i64, _P, _P, _P, _P, _P]
        L.orc_neighbors.restype = _i64
        L.orc_neighbors.argtypes = [_P, _i64, _P, _P, _P, _i64]
        L.orc_density.argtypes = [_P, _i64, _P, _P, _P]
        L.orc_eos.argtypes = [_P, _i64, _P, _P]
        L.orc_eos.restype = None
        L.orc_momentum.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _P, _P]
        L.orc_evaluate.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _P, _P]
        L.orc_diag.argtypes = [_P, _i64, _P, _P, _P]
        L.orc_diag.restype = None
        L.orc_step.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _i64, ctypes.c_int, _P]
        L.orc_eval_subset.argtypes = [_P, _i64, _P, _P, _P, _P, _i64, _P, _P, _P, _P]
        L.orc_rhs_adjoint.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_adjoint_ke.argtypes = [_P, _i64, _P, _P, _P, _P, _i64, _P, _P, _P]
        L.orc_rollout_ke.argtypes = [_P, _i64, _P, _P, _P, _P, _i64, _P]
        L.orc_step_continuity.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _i64, _P, _P, _P]
        L.orc_step_continuity_pc.argtypes = [_P, _i64, _P, _P, _P, _P, _P, _i64, _i32, _P, _P,
                                             _P]
        L.orc_continuity.argtypes = [_P, _i64, _P, _P, _P, _P, _P]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads(1)  # one thread unless asked otherwise
        _lib = L
    return _lib


def set_threads(k: int) -> int:
    """Run the per-destination loops on k OpenMP threads (results are bitwise
    the same for every k); returns the number in effect."""
    return int(lib().orc_set_threads(int(k)))


def params(p, brute: bool = False) -> OrcParams:
    o = OrcParams()
    o.dim = p.dim
    o.kernel = p.kernel
    o.cell_div = p.cell_div
    o.cell_order = int(getattr(p, "cell_order", 0))
    o.brute = 1 if brute else 0
    for k in range(3):
        o.periodic[k] = int(p.periodic[k])
        o.g[k] = float(p.g[k])
        o.lo[k] = float(p.lo[k])
        o.hi[k] = float(p.hi[k])
    o.h, o.rho0, o.c0, o.nu, o.eta, o.dt = p.h, p.rho0, p.c0, p.nu, p.eta, p.dt
    return o


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(_P)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle: invalid grid (periodic axis shorter than the stencil, "
                         "or more than 2^31 cells)")


def kernel_w(p, r):
    o = params(p)
    return np.array([lib().orc_kernel_w(ctypes.byref(o), float(v)) for v in np.ravel(r)])


def kernel_dwdr(p, r):
    o = params(p)
    return np.array([lib().orc_kernel_dwdr(ctypes.byref(o), float(v)) for v in np.ravel(r)])


def kernel_d2wdr2(p, r):
    o = params(p)
    return np.array([lib().orc_kernel_d2wdr2(ctypes.byref(o), float(v)) for v in np.ravel(r)])


def grid(p):
    o = params(p)
    nc = np.zeros(3, np.int64)
    cs = np.zeros(3, np.float64)
    _check(lib().orc_grid(ctypes.byref(o), _ptr(nc), _ptr(cs)))
    return nc, cs


def cell_keys(p, x):
    x = _c(x, np.float64)
    n = x.shape[1]
    keys = np.zeros(n, np.uint32)
    _check(lib().orc_cell_keys(ctypes.byref(params(p)), n, _ptr(x), _ptr(keys)))
    return keys


def bin_sort(p, x):
    """(keys_sorted, perm, cell_start, cell_end) of a stable sort by cell key."""
    x = _c(x, np.float64)
    n = x.shape[1]
    ncells = int(lib().orc_nkeys(ctypes.byref(params(p))))
    _check(0 if ncells > 0 else -1)
    keys = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.int64)
    cs = np.zeros(ncells, np.uint32)
    ce = np.zeros(ncells, np.uint32)
    _check(lib().orc_bin_sort(ctypes.byref(params(p)), n, _ptr(x), _ptr(keys), _ptr(perm),
                              _ptr(cs), _ptr(ce)))
    return keys, perm, cs, ce


def neighbors(p, x, brute=False):
    """CSR (offsets, idx) of the neighbour sets, rows ascending."""
    x = _c(x, np.float64)
    n = x.shape[1]
    off = np.zeros(n + 1, np.int64)
    o = params(p, brute)
    total = lib().orc_neighbors(ctypes.byref(o), n, _ptr(x), _ptr(off), None, 0)
    if total < 0:
        _check(-1)
    idx = np.zeros(max(total, 1), np.int64)
    lib().orc_neighbors(ctypes.byref(o), n, _ptr(x), _ptr(off), _ptr(idx), total)
    return off, idx[:total]


def density(p, x, m, brute=False):
    x = _c(x, np.float64)
    m = _c(m, np.float64)
    rho = np.zeros(x.shape[1])
    _check(lib().orc_density(ctypes.byref(params(p, brute)), x.shape[1], _ptr(x), _ptr(m),
                             _ptr(rho)))
    return rho


def eos(p, rho):
    rho = _c(rho, np.float64)
    out = np.zeros_like(rho)
    lib().orc_eos(ctypes.byref(params(p)), rho.shape[0], _ptr(rho), _ptr(out))
    return out


def momentum(p, x, v, m, ptype, rho, pr, brute=False):
    x, v = _c(x, np.float64), _c(v, np.float64)
    m, rho, pr = _c(m, np.float64), _c(rho, np.float64), _c(pr, np.float64)
    ptype = _c(ptype, np.uint8)
    a = np.zeros_like(x)
    _check(lib().orc_momentum(ctypes.byref(params(p, brute)), x.shape[1], _ptr(x), _ptr(v),
                              _ptr(m), _ptr(ptype), _ptr(rho), _ptr(pr), _ptr(a)))
    return a


def evaluate(p, x, v, m, ptype, brute=False):
    """(rho, p, a) at positions x and velocities v."""
    x, v, m = _c(x, np.float64), _c(v, np.float64), _c(m, np.float64)
    ptype = _c(ptype, np.uint8)
    n = x.shape[1]
    rho, pr, a = np.zeros(n), np.zeros(n), np.zeros_like(x)
    _check(lib().orc_evaluate(ctypes.byref(params(p, brute)), n, _ptr(x), _ptr(v), _ptr(m),
                              _ptr(ptype), _ptr(rho), _ptr(pr), _ptr(a)))
    return rho, pr, a


def diag(p, u, m):
    u, m = _c(u, np.float64), _c(m, np.float64)
    out = np.zeros(4)
    lib().orc_diag(ctypes.byref(params(p)), m.shape[0], _ptr(u), _ptr(m), _ptr(out))
    return out[:1 + p.dim]


def step(p, x, u, m, ptype, nsteps, a=None, prime=True, want_diag=False, brute=False):
    """Run nsteps predictor-corrector steps.  Returns dict of x, u, a, rho, p
    (and diag: (nsteps, 1+dim) if requested).  Inputs are not modified."""
    x, u, m = _c(x, np.float64).copy(), _c(u, np.float64).copy(), _c(m, np.float64)
    ptype = _c(ptype, np.uint8)
    n = x.shape[1]
    a = np.zeros_like(x) if a is None else _c(a, np.float64).copy()
    rho, pr = np.zeros(n), np.zeros(n)
    dg = np.zeros((max(nsteps, 1), 1 + p.dim)) if want_diag else None
    _check(lib().orc_step(ctypes.byref(params(p, brute)), n, _ptr(x), _ptr(u), _ptr(a), _ptr(m),
                          _ptr(ptype), _ptr(rho), _ptr(pr), nsteps, 1 if prime else 0,
                          _ptr(dg) if dg is not None else None))
    out = dict(x=x, u=u, a=a, rho=rho, p=pr)
    if want_diag:
        out["diag"] = dg[:nsteps]
    return out


def step_continuity(p, x, u, rho, m, ptype, nsteps):
    """nsteps of the paper's worked example (continuity density, EOS, momentum,
    Euler stage).  Returns dict of x, u, rho after the steps and p, a, arho of
    the last step's evaluation.  Inputs are not modified."""
    x, u, rho = (_c(t, np.float64).copy() for t in (x, u, rho))
    m, ptype = _c(m, np.float64), _c(ptype, np.uint8)
    n = x.shape[1]
    pr, a, arho = np.zeros(n), np.zeros_like(x), np.zeros(n)
    _check(lib().orc_step_continuity(ctypes.byref(params(p)), n, _ptr(x), _ptr(u), _ptr(rho),
                                     _ptr(m), _ptr(ptype), nsteps, _ptr(pr), _ptr(a),
                                     _ptr(arho)))
    return dict(x=x, u=u, rho=rho, p=pr, a=a, arho=arho)


def step_continuity_pc(p, x, u, rho, m, ptype, nsteps, a=None, arho=None, prime=True):
    """nsteps of the continuity scheme under the predictor-corrector
    integration (rho kicked like u).  Returns dict of x, u, rho after the steps
    and p, a, arho of the last evaluation.  Inputs are not modified."""
    x, u, rho = (_c(t, np.float64).copy() for t in (x, u, rho))
    m, ptype = _c(m, np.float64), _c(ptype, np.uint8)
    n = x.shape[1]
    a = np.zeros_like(x) if a is None else _c(a, np.float64).copy()
    arho = np.zeros(n) if arho is None else _c(arho, np.float64).copy()
    pr = np.zeros(n)
    _check(lib().orc_step_continuity_pc(ctypes.byref(params(p)), n, _ptr(x), _ptr(u), _ptr(rho),
                                        _ptr(m), _ptr(ptype), nsteps, 1 if prime else 0,
                                        _ptr(pr), _ptr(a), _ptr(arho)))
    return dict(x=x, u=u, rho=rho, p=pr, a=a, arho=arho)


def continuity(p, x, v, m, ptype):
    """d rho/dt of the continuity equation at (x, v)."""
    x, v, m = _c(x, np.float64), _c(v, np.float64), _c(m, np.float64)
    ptype = _c(ptype, np.uint8)
    arho = np.zeros(x.shape[1])
    _check(lib().orc_continuity(ctypes.byref(params(p)), x.shape[1], _ptr(x), _ptr(v), _ptr(m),
                                _ptr(ptype), _ptr(arho)))
    return arho


def eval_subset(p, x, v, m, ptype, sub):
    x, v, m = _c(x, np.float64), _c(v, np.float64), _c(m, np.float64)
    ptype = _c(ptype, np.uint8)
    sub = _c(sub, np.int64)
    k = sub.shape[0]
    rho, pr, a = np.zeros(k), np.zeros(k), np.zeros((p.dim, k))
    _check(lib().orc_eval_subset(ctypes.byref(params(p)), x.shape[1], _ptr(x), _ptr(v), _ptr(m),
                                 _ptr(ptype), k, _ptr(sub), _ptr(rho), _ptr(pr), _ptr(a)))
    return rho, pr, a


def rhs_adjoint(p, x, v, m, ptype, lam):
    """((dA/dx)^T lam, (dA/dv)^T lam, (dA/dnu)^T lam) at (x, v)."""
    x, v, m, lam = (_c(t, np.float64) for t in (x, v, m, lam))
    ptype = _c(ptype, np.uint8)
    lx, lv = np.zeros_like(x), np.zeros_like(x)
    lnu = np.zeros(1)
    _check(lib().orc_rhs_adjoint(ctypes.byref(params(p)), x.shape[1], _ptr(x), _ptr(v), _ptr(m),
                                 _ptr(ptype), _ptr(lam), _ptr(lx), _ptr(lv), _ptr(lnu)))
    return lx, lv, float(lnu[0])


def adjoint_ke(p, x0, u0, m, ptype, nsteps):
    """(grad_u0, grad_nu, KE) of KE(u^N) after nsteps from (x0, u0)."""
    x0, u0, m = _c(x0, np.float64), _c(u0, np.float64), _c(m, np.float64)
    ptype = _c(ptype, np.uint8)
    gu = np.zeros_like(u0)
    gnu = np.zeros(1)
    ke = np.zeros(1)
    _check(lib().orc_adjoint_ke(ctypes.byref(params(p)), x0.shape[1], _ptr(x0), _ptr(u0),
                                _ptr(m), _ptr(ptype), nsteps, _ptr(gu), _ptr(gnu), _ptr(ke)))
    return gu, float(gnu[0]), float(ke[0])


def rollout_ke(p, x0, u0, m, ptype, nsteps):
    x0, u0, m = _c(x0, np.float64), _c(u0, np.float64), _c(m, np.float64)
    ptype = _c(ptype, np.uint8)
    ke = np.zeros(1)
    _check(lib().orc_rollout_ke(ctypes.byref(params(p)), x0.shape[1], _ptr(x0), _ptr(u0),
                                _ptr(m), _ptr(ptype), nsteps, _ptr(ke)))
    return float(ke[0])
