"""FP64 CPU oracle of the coupled two-domain CNS right-hand side and the MPRK
step (ctypes wrapper around ``mprk_oracle.c`` (2D) and ``mprk_oracle3d.c``
(3D)).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  The product path (the
HIP library and its binding) never imports this package, and this package
never imports the product path.

Arrays are float64, C-contiguous, shaped ``[4, nz, nx]`` with the components
(rho, rho u, rho w, rho E), x fastest and row 0 at the bottom; in 3D
``[5, nz, ny, nx]`` with (rho, rho u, rho v, rho w, rho E).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mprk_oracle.c")
_SRC3 = os.path.join(_HERE, "mprk_oracle3d.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Strict IEEE: no contraction into fused multiply-adds, no fast-math.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                            for f in (_SRC, _SRC3))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, _SRC3, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("nz_lower", ctypes.c_int32),
        ("nz_upper", ctypes.c_int32),
        ("fast_is_lower", ctypes.c_int32),
        ("n_buffer", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dz_lower", ctypes.c_double),
        ("dz_upper", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_lower", ctypes.c_double),
        ("mu_upper", ctypes.c_double),
        ("gravity", ctypes.c_double),
    ]


@dataclass
class Problem:
    """Geometry and physics of two vertically stacked domains."""

    nx: int
    nz_lower: int
    nz_upper: int
    dx: float
    dz_lower: float
    dz_upper: float
    fast_is_lower: bool = True
    n_buffer: int = 4
    gamma: float = 1.4
    prandtl: float = 0.72
    mu_lower: float = 1e-3
    mu_upper: float = 1e-3
    gravity: float = 0.0

    def _c(self) -> _Cfg:
        return _Cfg(self.nx, self.nz_lower, self.nz_upper, int(bool(self.fast_is_lower)),
                    self.n_buffer, 0, self.dx, self.dz_lower, self.dz_upper, self.gamma,
                    self.prandtl, self.mu_lower, self.mu_upper, self.gravity)

    def shape(self, lower: bool):
        return (4, self.nz_lower if lower else self.nz_upper, self.nx)


class _Cfg3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz_lower", ctypes.c_int32),
        ("nz_upper", ctypes.c_int32),
        ("fast_is_lower", ctypes.c_int32),
        ("n_buffer", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dy", ctypes.c_double),
        ("dz_lower", ctypes.c_double),
        ("dz_upper", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_lower", ctypes.c_double),
        ("mu_upper", ctypes.c_double),
        ("gravity", ctypes.c_double),
    ]


@dataclass
class Problem3:
    """Geometry and physics of two vertically stacked 3D domains (x, y
    periodic)."""

    nx: int
    ny: int
    nz_lower: int
    nz_upper: int
    dx: float
    dy: float
    dz_lower: float
    dz_upper: float
    fast_is_lower: bool = True
    n_buffer: int = 4
    gamma: float = 1.4
    prandtl: float = 0.72
    mu_lower: float = 1e-3
    mu_upper: float = 1e-3
    gravity: float = 0.0

    def _c(self) -> _Cfg3:
        return _Cfg3(self.nx, self.ny, self.nz_lower, self.nz_upper, int(bool(self.fast_is_lower)),
                     self.n_buffer, self.dx, self.dy, self.dz_lower, self.dz_upper, self.gamma,
                     self.prandtl, self.mu_lower, self.mu_upper, self.gravity)

    def shape(self, lower: bool):
        return (5, self.nz_lower if lower else self.nz_upper, self.ny, self.nx)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Cfg)
        lib.orc_rhs.argtypes = [P, _D, _D, _D, _D]
        lib.orc_rhs_rows.argtypes = [P, _D, _D, _D, _D] + [ctypes.c_int] * 4
        lib.orc_interface.argtypes = [P, _D, _D, _D]
        lib.orc_llf.argtypes = [_D, _D, ctypes.c_int, ctypes.c_double, _D]
        lib.orc_tableau.argtypes = [ctypes.c_int, ctypes.c_int] + [_D] * 9
        lib.orc_mprk_step.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _D]
        lib.orc_mprk_run.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int64, _D, _D]
        lib.orc_sr_step.argtypes = [P, ctypes.c_int, ctypes.c_double, _D, _D]
        lib.orc_sr_run.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_int64, _D, _D]
        lib.orc_totals.argtypes = [P, _D, _D, _D]
        lib.orc_wave_measures.argtypes = [P, _D, _D, _D, _D, _D]
        lib.orc_dt_rule.argtypes = [P, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_dt_rule.restype = ctypes.c_double
        P3 = ctypes.POINTER(_Cfg3)
        lib.orc3_rhs.argtypes = [P3, _D, _D, _D, _D]
        lib.orc3_interface.argtypes = [P3, _D, _D, _D]
        lib.orc3_llf.argtypes = [_D, _D, ctypes.c_int, ctypes.c_double, _D]
        lib.orc3_mprk_step.argtypes = [P3, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _D]
        lib.orc3_mprk_run.argtypes = [P3, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int64, _D, _D]
        lib.orc3_totals.argtypes = [P3, _D, _D, _D]
        lib.orc3_wave_measures.argtypes = [P3, _D, _D, _D, _D, _D]
        lib.orc3_dt_rule.argtypes = [P3, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc3_dt_rule.restype = ctypes.c_double
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _check(pb: Problem, qlo: np.ndarray, qup: np.ndarray):
    if qlo.shape != pb.shape(True) or qup.shape != pb.shape(False):
        raise ValueError("state shapes %s/%s do not match the problem" % (qlo.shape, qup.shape))


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def rhs(pb: Problem, qlo, qup, rows_lower=None, rows_upper=None):
    """Coupled RHS dq/dt of both domains.  Optional row ranges (lo, hi)
    restrict the evaluation; other rows of the result are zero."""
    qlo = np.ascontiguousarray(qlo, dtype=np.float64)
    qup = np.ascontiguousarray(qup, dtype=np.float64)
    _check(pb, qlo, qup)
    rlo = np.zeros_like(qlo)
    rup = np.zeros_like(qup)
    c = pb._c()
    if rows_lower is None and rows_upper is None:
        _load().orc_rhs(ctypes.byref(c), _ptr(qlo), _ptr(qup), _ptr(rlo), _ptr(rup))
    else:
        l0, l1 = rows_lower if rows_lower is not None else (0, 0)
        u0, u1 = rows_upper if rows_upper is not None else (0, 0)
        _load().orc_rhs_rows(ctypes.byref(c), _ptr(qlo), _ptr(qup), _ptr(rlo), _ptr(rup),
                             l0, l1, u0, u1)
    return rlo, rup


def interface(pb: Problem, qlo, qup) -> np.ndarray:
    """Per column: (sigma_xz, Pi_z, u_w1, u_w2, T_w1, T_w2)."""
    qlo = np.ascontiguousarray(qlo, dtype=np.float64)
    qup = np.ascontiguousarray(qup, dtype=np.float64)
    out = np.zeros((pb.nx, 6))
    c = pb._c()
    _load().orc_interface(ctypes.byref(c), _ptr(qlo), _ptr(qup), _ptr(out))
    return out


def llf(qL, qR, direction: int, gamma: float = 1.4) -> np.ndarray:
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    F = np.zeros(4)
    _load().orc_llf(_ptr(qL), _ptr(qR), int(direction), float(gamma), _ptr(F))
    return F


def tableau(base: int, m: int) -> dict:
    """Expanded MPRK tableaux {F,B,S: (a, b, c)} with ms stages."""
    s = {2: 2, 3: 3}[base]
    ms = m * s
    arrs = [np.zeros((ms, ms)) if i % 3 == 0 else np.zeros(ms) for i in range(9)]
    rc = _load().orc_tableau(int(base), int(m), *[_ptr(a) for a in arrs])
    if rc != s:
        raise ValueError("bad base/m")
    return {"F": tuple(arrs[0:3]), "B": tuple(arrs[3:6]), "S": tuple(arrs[6:9]), "s": s}


def mprk_step(pb: Problem, base: int, m: int, dt: float, qlo: np.ndarray, qup: np.ndarray):
    """One MPRK step (Algorithm 1, Butcher form), in place."""
    _check(pb, qlo, qup)
    c = pb._c()
    rc = _load().orc_mprk_step(ctypes.byref(c), base, m, dt, _ptr(qlo), _ptr(qup))
    if rc:
        raise ValueError("orc_mprk_step failed")


def mprk_run(pb: Problem, base: int, m: int, dt: float, nsteps: int, qlo, qup):
    _check(pb, qlo, qup)
    c = pb._c()
    rc = _load().orc_mprk_run(ctypes.byref(c), base, m, dt, int(nsteps), _ptr(qlo), _ptr(qup))
    if rc:
        raise ValueError("orc_mprk_run failed")


def sr_step(pb: Problem, base: int, dt: float, qlo, qup):
    """One single-rate base-method step on the coupled state, in place."""
    _check(pb, qlo, qup)
    c = pb._c()
    if _load().orc_sr_step(ctypes.byref(c), base, dt, _ptr(qlo), _ptr(qup)):
        raise ValueError("orc_sr_step failed")


def sr_run(pb: Problem, base: int, dt: float, nsteps: int, qlo, qup):
    _check(pb, qlo, qup)
    c = pb._c()
    if _load().orc_sr_run(ctypes.byref(c), base, dt, int(nsteps), _ptr(qlo), _ptr(qup)):
        raise ValueError("orc_sr_run failed")


def totals(pb: Problem, qlo, qup) -> np.ndarray:
    """[2, 4]: sum of q |K| per domain (lower, upper) and component."""
    out = np.zeros(8)
    c = pb._c()
    _load().orc_totals(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                       _ptr(np.ascontiguousarray(qup)), _ptr(out))
    return out.reshape(2, 4)


def wave_measures(pb: Problem, qlo, qup):
    """(lam[2], cour[2], vis[2], bad) per domain (lower, upper): max over
    cells of the directional sum of (|u_d|+a)/d_d; max over cells and
    directions of (|u_d|+a)/d_d (times dt: the paper's Courant number); max
    diffusion coefficient times sum 1/d_d^2; bad = 1 on a non-physical state."""
    lam = np.zeros(2)
    cour = np.zeros(2)
    vis = np.zeros(2)
    c = pb._c()
    bad = _load().orc_wave_measures(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                                    _ptr(np.ascontiguousarray(qup)), _ptr(lam), _ptr(cour),
                                    _ptr(vis))
    return lam, cour, vis, int(bad)


def dt_rule(pb: Problem, qlo, qup, m: int, cr: float = 0.5, dn: float = 0.25) -> float:
    c = pb._c()
    return float(_load().orc_dt_rule(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                                     _ptr(np.ascontiguousarray(qup)), int(m), cr, dn))


# ---- 3D ---------------------------------------------------------------------
def rhs3(pb: Problem3, qlo, qup):
    """Coupled 3D RHS of both domains (all planes)."""
    qlo = np.ascontiguousarray(qlo, dtype=np.float64)
    qup = np.ascontiguousarray(qup, dtype=np.float64)
    _check(pb, qlo, qup)
    rlo = np.zeros_like(qlo)
    rup = np.zeros_like(qup)
    c = pb._c()
    _load().orc3_rhs(ctypes.byref(c), _ptr(qlo), _ptr(qup), _ptr(rlo), _ptr(rup))
    return rlo, rup


def interface3(pb: Problem3, qlo, qup) -> np.ndarray:
    """Per column [ny, nx, 8]: sigma_xz, sigma_yz, Pi_z, u_w1, v_w1, T_w1,
    u_w2, v_w2."""
    out = np.zeros((pb.ny, pb.nx, 8))
    c = pb._c()
    _load().orc3_interface(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                           _ptr(np.ascontiguousarray(qup)), _ptr(out))
    return out


def llf3(qL, qR, direction: int, gamma: float = 1.4) -> np.ndarray:
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    F = np.zeros(5)
    _load().orc3_llf(_ptr(qL), _ptr(qR), int(direction), float(gamma), _ptr(F))
    return F


def mprk_run3(pb: Problem3, base: int, m: int, dt: float, nsteps: int, qlo, qup):
    """nsteps MPRK steps in 3D, in place."""
    _check(pb, qlo, qup)
    c = pb._c()
    rc = _load().orc3_mprk_run(ctypes.byref(c), base, m, dt, int(nsteps), _ptr(qlo), _ptr(qup))
    if rc:
        raise ValueError("orc3_mprk_run failed")


def totals3(pb: Problem3, qlo, qup) -> np.ndarray:
    """[2, 5]: sum of q |K| per domain and component."""
    out = np.zeros(10)
    c = pb._c()
    _load().orc3_totals(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                        _ptr(np.ascontiguousarray(qup)), _ptr(out))
    return out.reshape(2, 5)


def wave_measures3(pb: Problem3, qlo, qup):
    lam = np.zeros(2)
    cour = np.zeros(2)
    vis = np.zeros(2)
    c = pb._c()
    bad = _load().orc3_wave_measures(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                                     _ptr(np.ascontiguousarray(qup)), _ptr(lam), _ptr(cour),
                                     _ptr(vis))
    return lam, cour, vis, int(bad)


def dt_rule3(pb: Problem3, qlo, qup, m: int, cr: float = 0.5, dn: float = 0.25) -> float:
    c = pb._c()
    return float(_load().orc3_dt_rule(ctypes.byref(c), _ptr(np.ascontiguousarray(qlo)),
                                      _ptr(np.ascontiguousarray(qup)), int(m), cr, dn))
