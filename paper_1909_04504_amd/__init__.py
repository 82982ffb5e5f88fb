"""Python binding of the MI355X WCSPH library (include/sph.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of libsph_mi355x.so.  torch provides device memory and the current stream.
There is no CPU fallback: if the library cannot be loaded, import fails.

The entry points keep the C names without the prefix: bin_sort, neighbors,
density, eos, momentum, step, step_backward, accel_backward, check.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

from . import build as _build

SPH_OK, SPH_EINVAL, SPH_EWORKSPACE, SPH_ECAPACITY = 0, -1, -2, -3
SPH_EDOMAIN, SPH_ENONFINITE, SPH_EDEVICE = -4, -5, -6
FP64, FP32_MIXED = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20  # SPH_NOALLOC_SCRATCH_BYTES of sph.h
SUMMATION, CONTINUITY = 0, 1  # sph_params.scheme
PREDICTOR_CORRECTOR, EULER = 0, 1  # sph_params.integrator

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_P = ctypes.c_void_p


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sph error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("dim", _i32), ("kernel", _i32), ("precision", _i32), ("cell_div", _i32),
                ("periodic", _i32 * 3), ("nbr_cap", _i32),
                ("h", _d), ("rho0", _d), ("c0", _d), ("nu", _d), ("eta", _d), ("dt", _d),
                ("g", _d * 3), ("lo", _d * 3), ("hi", _d * 3),
                ("scheme", _i32), ("integrator", _i32), ("pair_tiles", _i32),
                ("cell_order", _i32)]


class Particles(ctypes.Structure):
    _fields_ = [("n", _i64), ("x", _P * 3), ("u", _P * 3), ("a", _P * 3), ("rho", _P),
                ("p", _P), ("m", _P), ("type", _P), ("id", _P), ("arho", _P)]


EXPORTED = ("sph_grid", "sph_workspace_bytes", "sph_bin_sort", "sph_neighbors", "sph_density",
            "sph_eos", "sph_momentum", "sph_step", "sph_step_backward", "sph_accel_backward",
            "sph_check", "sph_last_error", "sph_read_interactions", "sph_timer_enable",
            "sph_timer_read", "sph_step_noalloc", "sph_ke_seed")

_lib = None


def lib():
    """The loaded library; built first only if no built library exists."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.sph_last_error.restype = ctypes.c_char_p
        L.sph_last_error.argtypes = []
        L.sph_grid.argtypes = [_P, _P, _P]
        L.sph_workspace_bytes.restype = ctypes.c_size_t
        L.sph_workspace_bytes.argtypes = [_P, _i64, _i64]
        L.sph_bin_sort.argtypes = [_P, _P, _P, ctypes.c_size_t, _P, _P, _P]
        L.sph_neighbors.argtypes = [_P, _P, _P, _P, _i64, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.sph_density.argtypes = [_P, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.sph_eos.argtypes = [_P, _P, _P]
        L.sph_momentum.argtypes = [_P, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.sph_step.argtypes = [_P, _P, _i64, ctypes.c_int, _P, ctypes.c_size_t, _P, _P]
        L.sph_step_noalloc.argtypes = [_P, _P, _i64, ctypes.c_int, _P, _P]
        L.sph_ke_seed.argtypes = [_P, _P, ctypes.c_double, _P, _P]
        L.sph_step_backward.argtypes = [_P, _P, _i64, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.sph_accel_backward.argtypes = [_P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
        L.sph_check.argtypes = [_P, ctypes.c_size_t, _P]
        L.sph_read_interactions.argtypes = [_P, ctypes.c_size_t, _P, ctypes.c_int, _P]
        L.sph_timer_enable.argtypes = [ctypes.c_int]
        L.sph_timer_read.argtypes = [ctypes.c_int, _P, _P, _P, ctypes.c_int]
        _lib = L
    return _lib


def _rc(code: int):
    if code != SPH_OK:
        raise SphError(code, lib().sph_last_error().decode())


def make_params(p, precision: int = FP64, nbr_cap: int = 0, pair_tiles: int = 0) -> Params:
    """C parameter struct from a sph_workloads.Params-like object.  nbr_cap:
    neighbour-list capacity per particle (0 default, < 0 cell walks only);
    pair_tiles: LDS-staged tiles of the 3D mixed-precision passes (0 where
    they apply, < 0 never, k > 0 at most k staged particles per tile)."""
    c = Params()
    c.dim, c.kernel, c.precision, c.cell_div = p.dim, p.kernel, precision, p.cell_div
    for k in range(3):
        c.periodic[k] = int(p.periodic[k])
        c.g[k], c.lo[k], c.hi[k] = float(p.g[k]), float(p.lo[k]), float(p.hi[k])
    c.nbr_cap = int(nbr_cap)
    c.pair_tiles = int(pair_tiles)
    c.scheme = int(getattr(p, "scheme", 0))
    c.cell_order = int(getattr(p, "cell_order", 0))
    c.integrator = int(getattr(p, "integrator", 0))
    c.h, c.rho0, c.c0, c.nu, c.eta, c.dt = p.h, p.rho0, p.c0, p.nu, p.eta, p.dt
    return c


def pair_dtype(precision: int) -> torch.dtype:
    return torch.float64 if precision == FP64 else torch.float32


def _dev(v, dtype, device) -> torch.Tensor:
    """A contiguous device tensor copy of a numpy array or tensor."""
    if torch.is_tensor(v):
        return v.detach().to(device=device, dtype=dtype).contiguous().clone()
    return torch.as_tensor(np.ascontiguousarray(v)).to(device=device, dtype=dtype)


class DeviceParticles:
    """Device arrays of one particle set (SoA; vectors as (dim, n) tensors)."""

    def __init__(self, x, u, m, ptype, pid, precision: int = FP64, a=None, device="cuda",
                 rho=None, scheme: int = SUMMATION):
        T = pair_dtype(precision)
        # rho is FP64 under the continuity scheme (an integrated state)
        TR = torch.float64 if scheme == CONTINUITY else T
        self.precision = precision
        self.x = _dev(x, torch.float64, device)
        self.u = _dev(u, torch.float64, device)
        self.dim, self.n = self.x.shape
        self.a = (torch.zeros((self.dim, self.n), dtype=T, device=device) if a is None else
                  _dev(a, T, device))
        # rho is an output of the summation scheme and a state (input) of the
        # continuity scheme
        self.rho = (torch.zeros(self.n, dtype=TR, device=device) if rho is None else
                    _dev(rho, TR, device))
        self.p = torch.zeros(self.n, dtype=T, device=device)
        # drho/dt: the continuity scheme's rate (FP64), absent otherwise
        self.arho = (torch.zeros(self.n, dtype=torch.float64, device=device)
                     if scheme == CONTINUITY else None)
        self.m = _dev(m, torch.float64, device)
        self.type = _dev(ptype, torch.uint8, device)
        self.id = _dev(pid, torch.int32, device)

    @classmethod
    def from_state(cls, s, precision: int = FP64, device="cuda", scheme: int = SUMMATION):
        return cls(s.x, s.u, s.m, s.ptype, s.pid, precision, device=device,
                   rho=getattr(s, "rho", None), scheme=scheme)

    def struct(self, prm: Optional[Params] = None) -> Particles:
        """The C view of these arrays; with prm, first checks that their
        element types are the ones prm implies (a mismatch would make the
        library read past the ends of the arrays)."""
        if prm is not None:
            T = pair_dtype(prm.precision)
            TR = torch.float64 if prm.scheme == CONTINUITY else T
            if (prm.dim != self.dim or self.a.dtype != T or self.p.dtype != T
                    or self.rho.dtype != TR
                    or (prm.scheme == CONTINUITY and (self.arho is None or
                                                     self.arho.dtype != torch.float64))):
                raise ValueError(
                    f"particle arrays (dim {self.dim}, a {self.a.dtype}, rho "
                    f"{self.rho.dtype}) do not match the parameters (dim {prm.dim}, "
                    f"precision {prm.precision}, scheme {prm.scheme})")
        c = Particles()
        c.n = self.n
        for k in range(self.dim):
            c.x[k] = self.x[k].data_ptr()
            c.u[k] = self.u[k].data_ptr()
            c.a[k] = self.a[k].data_ptr()
        c.rho, c.p = self.rho.data_ptr(), self.p.data_ptr()
        c.m, c.type, c.id = self.m.data_ptr(), self.type.data_ptr(), self.id.data_ptr()
        c.arho = self.arho.data_ptr() if self.arho is not None else None
        return c

    def numpy(self) -> dict:
        out = {k: getattr(self, k).cpu().numpy() for k in
               ("x", "u", "a", "rho", "p", "m", "type", "id")}
        if self.arho is not None:
            out["arho"] = self.arho.cpu().numpy()
        return out

    def clone(self) -> "DeviceParticles":
        o = object.__new__(DeviceParticles)
        o.__dict__.update({k: (v.clone() if torch.is_tensor(v) else v)
                           for k, v in self.__dict__.items()})
        return o


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def grid(prm: Params):
    nc = (ctypes.c_int64 * 3)()
    ncells = ctypes.c_int64()
    _rc(lib().sph_grid(ctypes.byref(prm), nc, ctypes.byref(ncells)))
    return tuple(nc), ncells.value


def workspace_bytes(prm: Params, n: int, adjoint_k: int = 0) -> int:
    b = lib().sph_workspace_bytes(ctypes.byref(prm), n, adjoint_k)
    if b == 0:
        raise SphError(SPH_EINVAL, lib().sph_last_error().decode())
    return b


def workspace(prm: Params, n: int, adjoint_k: int = 0, device="cuda") -> torch.Tensor:
    """A zero-filled workspace tensor (torch allocations are 256-byte aligned)."""
    return torch.zeros(workspace_bytes(prm, n, adjoint_k), dtype=torch.uint8, device=device)


def cell_arrays(prm: Params, device="cuda"):
    _, ncells = grid(prm)
    return (torch.zeros(ncells, dtype=torch.int32, device=device),
            torch.zeros(ncells, dtype=torch.int32, device=device))


def bin_sort(prm: Params, dp: DeviceParticles, ws: torch.Tensor, cell_start, cell_end,
             stream=None):
    s = dp.struct(prm)
    _rc(lib().sph_bin_sort(ctypes.byref(prm), ctypes.byref(s), ws.data_ptr(), ws.numel(),
                           cell_start.data_ptr(), cell_end.data_ptr(), _stream(stream)))


def neighbors(prm: Params, dp: DeviceParticles, cell_start, cell_end, capacity: int, offsets,
              nbr: Optional[torch.Tensor], ws: torch.Tensor, stream=None) -> int:
    """Fills offsets (int64, n+1) and nbr (int32, capacity); returns the total.
    Raises SphError(SPH_ECAPACITY) with .total set if capacity is too small."""
    s = dp.struct(prm)
    total = ctypes.c_int64()
    rc = lib().sph_neighbors(ctypes.byref(prm), ctypes.byref(s), cell_start.data_ptr(),
                             cell_end.data_ptr(), capacity, offsets.data_ptr(),
                             nbr.data_ptr() if nbr is not None else None, ctypes.byref(total),
                             ws.data_ptr(), ws.numel(), _stream(stream))
    if rc == SPH_ECAPACITY:
        e = SphError(rc, lib().sph_last_error().decode())
        e.total = total.value
        raise e
    _rc(rc)
    return total.value


def density(prm, dp, cell_start, cell_end, ws, stream=None):
    s = dp.struct(prm)
    _rc(lib().sph_density(ctypes.byref(prm), ctypes.byref(s), cell_start.data_ptr(),
                          cell_end.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))


def eos(prm, dp, stream=None):
    s = dp.struct(prm)
    _rc(lib().sph_eos(ctypes.byref(prm), ctypes.byref(s), _stream(stream)))


def momentum(prm, dp, cell_start, cell_end, ws, stream=None):
    s = dp.struct(prm)
    _rc(lib().sph_momentum(ctypes.byref(prm), ctypes.byref(s), cell_start.data_ptr(),
                           cell_end.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))


def step(prm, dp, nsteps: int, ws, prime: bool = True, diag: Optional[torch.Tensor] = None,
         stream=None):
    s = dp.struct(prm)
    _rc(lib().sph_step(ctypes.byref(prm), ctypes.byref(s), nsteps, 1 if prime else 0,
                       ws.data_ptr(), ws.numel(), diag.data_ptr() if diag is not None else None,
                       _stream(stream)))


def step_noalloc(prm, dp, nsteps: int, prime: bool = True, diag: Optional[torch.Tensor] = None,
                 stream=None):
    """sph_step_noalloc: sph_step on the library's static device scratch."""
    s = dp.struct(prm)
    _rc(lib().sph_step_noalloc(ctypes.byref(prm), ctypes.byref(s), nsteps, 1 if prime else 0,
                               diag.data_ptr() if diag is not None else None, _stream(stream)))


def ke_seed(prm, dp, scale: float, lam, stream=None):
    """sph_ke_seed: lam = adjoint of scale * KE at dp's state."""
    s = dp.struct(prm)
    _rc(lib().sph_ke_seed(ctypes.byref(prm), ctypes.byref(s), float(scale), lam.data_ptr(),
                          _stream(stream)))


def step_backward(prm, ckpt: DeviceParticles, k: int, lam_in, lam_out, dJ_dnu, ws, stream=None):
    s = ckpt.struct(prm)
    _rc(lib().sph_step_backward(ctypes.byref(prm), ctypes.byref(s), k, lam_in.data_ptr(),
                                lam_out.data_ptr(), dJ_dnu.data_ptr(), ws.data_ptr(), ws.numel(),
                                _stream(stream)))


def accel_backward(prm, st: DeviceParticles, lam_a, lam_x, lam_u, dJ_dnu, ws, stream=None):
    s = st.struct(prm)
    _rc(lib().sph_accel_backward(ctypes.byref(prm), ctypes.byref(s), lam_a.data_ptr(),
                                 lam_x.data_ptr(), lam_u.data_ptr(), dJ_dnu.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream(stream)))


def check(ws, stream=None):
    _rc(lib().sph_check(ws.data_ptr(), ws.numel(), _stream(stream)))


def read_interactions(ws, reset: bool = True, stream=None) -> int:
    """Total interactions sum_i |N(i)| accumulated by density evaluations."""
    t = ctypes.c_int64()
    _rc(lib().sph_read_interactions(ws.data_ptr(), ws.numel(), ctypes.byref(t),
                                    1 if reset else 0, _stream(stream)))
    return t.value


def timer_enable(on: bool = True):
    _rc(lib().sph_timer_enable(1 if on else 0))


def timer_read(reset: bool = True) -> dict:
    """{kernel name: (total ms, launches)} of the launches timed so far."""
    k = 32
    names = (ctypes.c_char_p * k)()
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    n = lib().sph_timer_read(k, names, ms, cnt, 1 if reset else 0)
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(n, k)) if cnt[i] > 0}
