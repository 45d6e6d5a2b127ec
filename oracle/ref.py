"""ctypes wrapper around the FP64 C oracle (oracle/mx_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg.  Arrays are numpy float64 shaped (ny, nx)
in 2D or (nz, ny, nx) in 3D (x contiguous); they are updated in place.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mx_oracle.c")
LIB = os.path.join(HERE, "libmxoracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over grid rows)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nx", C.c_long), ("ny", C.c_long), ("nz", C.c_long),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("blocks", C.c_int), ("sweeps", C.c_int), ("tol", C.c_double),
                ("check_every", C.c_int), ("filter_passes", C.c_int), ("lumped", C.c_int),
                ("four_pi", C.c_double), ("solver", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int * 2), ("resid", C.c_double * 2), ("rhs", C.c_double * 2),
                ("nonconverged", C.c_int * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P3 = C.POINTER(C.c_double) * 3
        L.ora_step.argtypes = [C.POINTER(_Cfg), P3, P3, C.c_void_p, C.c_double, C.c_void_p, C.POINTER(_Stats)]
        L.ora_step.restype = C.c_int
        L.ora_faraday.argtypes = [C.POINTER(_Cfg), P3, P3]
        L.ora_filter.argtypes = [C.POINTER(_Cfg), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ora_rhs.argtypes = [C.POINTER(_Cfg), P3, C.c_void_p, C.c_double, P3]
        L.ora_apply_A.argtypes = [C.POINTER(_Cfg), P3, P3, C.c_int]
        L.ora_solve.argtypes = [C.POINTER(_Cfg), P3, P3, C.c_void_p, C.POINTER(_Stats)]
        L.ora_adjoint_step.argtypes = [C.POINTER(_Cfg), P3, P3, C.c_void_p, C.c_double, C.c_void_p]
        L.ora_num_threads.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int]
        PD = C.POINTER(C.c_double)
        L.ora_pic_push_deposit.argtypes = [C.POINTER(_Cfg), P3, P3, C.c_long, C.c_double, C.c_double, C.c_double,
                                           PD, PD, PD, PD, PD, P3]
        L.ora_pic_push_deposit.restype = C.c_int
        L.ora_pic_deposit_charge.argtypes = [C.POINTER(_Cfg), C.c_long, C.c_double, C.c_double, PD, PD, PD]
        _lib = L
    return _lib


@dataclass
class Config:
    ndim: int
    shape: tuple            # (ny, nx) or (nz, ny, nx)
    dt: float
    d: Sequence[float] = (1.0, 1.0, 1.0)
    blocks: int = 3
    sweeps: int = 20
    tol: float = 0.0
    check_every: int = 1
    filter_passes: int = 0
    lumped: bool = False
    four_pi: float = 4.0 * math.pi
    solver: int = 0                 # 0: Alg 1; 1: Chebyshev semi-iteration

    def c(self) -> _Cfg:
        if self.solver != 0 and self.ndim == 3 and not (self.d[0] == self.d[1] == self.d[2]):
            raise ValueError("the 3D Chebyshev solve is defined for cubic cells only")
        if self.ndim == 2:
            ny, nx = self.shape
            nz = 1
        else:
            nz, ny, nx = self.shape
        d = list(self.d) + [1.0] * (3 - len(self.d))
        return _Cfg(self.ndim, nx, ny, nz, d[0], d[1], d[2], self.dt, self.blocks, self.sweeps,
                    self.tol, self.check_every, self.filter_passes, int(self.lumped), self.four_pi,
                    int(self.solver))


def _p3(arrs):
    for a in arrs:
        assert a.dtype == np.float64 and a.flags.c_contiguous
    return (C.POINTER(C.c_double) * 3)(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs])


def _opt_p3(arrs):
    if arrs is None:
        return None
    return C.cast(C.pointer(_p3(arrs)), C.c_void_p)


@dataclass
class StepStats:
    sweeps: tuple
    resid: tuple
    rhs: tuple
    nonconverged: tuple


def step(cfg: Config, E: List[np.ndarray], B: List[np.ndarray], J0: Optional[List[np.ndarray]] = None,
         env: float = 0.0, replay: Optional[Sequence[int]] = None) -> StepStats:
    L = lib()
    c = cfg.c()
    st = _Stats()
    rep = None
    if replay is not None:
        rep_arr = (C.c_int * 2)(*replay)
        rep = C.cast(rep_arr, C.c_void_p)
    J = _opt_p3(J0) if J0 is not None else None
    rc = L.ora_step(C.byref(c), _p3(E), _p3(B), J, env, rep, C.byref(st))
    if rc != 0:
        raise FloatingPointError("oracle step produced a non-finite value")
    return StepStats(tuple(st.sweeps), tuple(st.resid), tuple(st.rhs), tuple(st.nonconverged))


def run(cfg: Config, E, B, nsteps: int, J0=None, env=None, replay=None) -> List[StepStats]:
    """nsteps steps; env[n] scales J0 at step n; replay[n] = per-block counts."""
    out = []
    for n in range(nsteps):
        out.append(step(cfg, E, B, J0, 0.0 if env is None else float(env[n]),
                        None if replay is None else replay[n]))
    return out


def faraday(cfg: Config, E, B):
    lib().ora_faraday(C.byref(cfg.c()), _p3(E), _p3(B))


def filt(cfg: Config, src: np.ndarray) -> np.ndarray:
    dst = np.empty_like(src)
    lib().ora_filter(C.byref(cfg.c()), src.ctypes.data_as(C.POINTER(C.c_double)),
                     dst.ctypes.data_as(C.POINTER(C.c_double)))
    return dst


def rhs(cfg: Config, B, Jf=None, src_scale: float = 1.0):
    out = [np.zeros_like(B[0]) for _ in range(3)]
    lib().ora_rhs(C.byref(cfg.c()), _p3(B), _opt_p3(Jf), src_scale, _p3(out))
    return out


def apply_A(cfg: Config, x, mask: int = 7):
    y = [np.zeros_like(x[0]) for _ in range(3)]
    lib().ora_apply_A(C.byref(cfg.c()), _p3(x), _p3(y), mask)
    return y


def solve(cfg: Config, b, replay=None):
    x = [np.zeros_like(b[0]) for _ in range(3)]
    st = _Stats()
    rep = None
    if replay is not None:
        rep_arr = (C.c_int * 2)(*replay)
        rep = C.cast(rep_arr, C.c_void_p)
    lib().ora_solve(C.byref(cfg.c()), _p3(b), _p3(x), rep, C.byref(st))
    return x, StepStats(tuple(st.sweeps), tuple(st.resid), tuple(st.rhs), tuple(st.nonconverged))


def adjoint_step(cfg: Config, Ebar, Bbar, J0bar, env: float, sweeps: Sequence[int]):
    rep_arr = (C.c_int * 2)(*sweeps)
    lib().ora_adjoint_step(C.byref(cfg.c()), _p3(Ebar), _p3(Bbar), _opt_p3(J0bar), env,
                           C.cast(rep_arr, C.c_void_p))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (OpenMP)."""
    lib().ora_set_num_threads(int(n))


def _pd(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def pic_push_deposit(cfg: Config, E, B, q: float, m: float, w: float, x, y, ux, uy, uz, J) -> None:
    """One relativistic Boris push of a 2D species (positions x, y at n,
    momenta u = gamma v at n - 1/2, updated in place) in E^n and
    B^n = B^{n-1/2} - (dt/2) curl E^n, with its charge-conserving current
    J^{n+1/2} added into J (three arrays placed like E)."""
    bad = lib().ora_pic_push_deposit(C.byref(cfg.c()), _p3(E), _p3(B), len(x), q, m, w, _pd(x), _pd(y), _pd(ux),
                                     _pd(uy), _pd(uz), _p3(J))
    if bad:
        raise ValueError("a particle moved a cell or more in one step")


def pic_deposit_charge(cfg: Config, q: float, w: float, x, y, rho) -> None:
    """rho at the nodes += the species' charge density (linear shapes)."""
    lib().ora_pic_deposit_charge(C.byref(cfg.c()), len(x), q, w, _pd(x), _pd(y), _pd(rho))
