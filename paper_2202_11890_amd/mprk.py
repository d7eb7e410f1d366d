"""Python binding of the MPRK C ABI (``include/mprk.h``).

Argument marshalling only: every step of the computation runs in the HIP
library ``libmprk.so`` built next to this file.  PyTorch supplies device
memory and the HIP stream.  There is no fallback: if the library is missing
or fails to load, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

ABI_VERSION = 2
OK, EINVAL, EBUFFER, EWORKSPACE, EHIP, ENONFINITE, EUNSUPPORTED, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
EXEC_LAUNCH, EXEC_PERSISTENT, EXEC_GRAPH = 0, 1, 2
TILE_32X16, TILE_16X32, TILE_64X8, TILE_32X8, TILE_SHAPES = 0, 1, 2, 3, 4
TILE_NAMES = ("32x16", "16x32", "64x8", "32x8")
REGION_F, REGION_B, REGION_S, REGION_ALL = 1, 2, 4, 7

_HERE = os.path.dirname(os.path.abspath(__file__))
# Always the in-tree build next to this file.
LIB_PATH = os.path.join(_HERE, "libmprk.so")


class mprk_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz_lower", ctypes.c_int32),
        ("nz_upper", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dy", ctypes.c_double),
        ("dz_lower", ctypes.c_double),
        ("dz_upper", ctypes.c_double),
        ("fast_is_lower", ctypes.c_int32),
        ("n_buffer", ctypes.c_int32),
        ("base_rk", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_lower", ctypes.c_double),
        ("mu_upper", ctypes.c_double),
        ("gravity", ctypes.c_double),
        ("flux_bits", ctypes.c_int32),
        ("strict_buffer", ctypes.c_int32),
    ]


class mprk_stats(ctypes.Structure):
    _fields_ = [
        ("totals_lower", ctypes.c_double * 5),
        ("totals_upper", ctypes.c_double * 5),
        ("lambda_lower", ctypes.c_double),
        ("lambda_upper", ctypes.c_double),
        ("courant_lower", ctypes.c_double),
        ("courant_upper", ctypes.c_double),
        ("visc_lower", ctypes.c_double),
        ("visc_upper", ctypes.c_double),
        ("steps_done", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {
            "totals_lower": list(self.totals_lower),
            "totals_upper": list(self.totals_upper),
            "lambda_lower": self.lambda_lower,
            "lambda_upper": self.lambda_upper,
            "courant_lower": self.courant_lower,
            "courant_upper": self.courant_upper,
            "visc_lower": self.visc_lower,
            "visc_upper": self.visc_upper,
            "steps_done": self.steps_done,
            "status": self.status,
        }


class mprk_member(ctypes.Structure):
    _fields_ = [
        ("cfg", mprk_config),
        ("q_lower", ctypes.c_void_p),
        ("q_upper", ctypes.c_void_p),
        ("dt", ctypes.c_double),
    ]


EXPORTS = ("mprk_validate", "mprk_workspace_bytes", "mprk_create", "mprk_set_stream", "mprk_rhs",
           "mprk_step", "mprk_run", "mprk_diagnostics", "mprk_diagnostics_static", "mprk_stable_dt",
           "mprk_set_exec",
           "mprk_set_wait_limit", "mprk_set_tile",
           "mprk_profile_enable", "mprk_profile_take", "mprk_destroy", "mprk_strerror",
           "mprk_batch_validate", "mprk_batch_workspace_bytes", "mprk_batch_create",
           "mprk_batch_set_exec", "mprk_batch_set_tile", "mprk_batch_set_wait_limit", "mprk_batch_set_dt",
           "mprk_batch_set_adaptive", "mprk_batch_get_dt",
           "mprk_batch_tune", "mprk_batch_run", "mprk_batch_diagnostics", "mprk_batch_destroy")

_lib = None


class MprkError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (where, strerror(code), code))


def load(path: str = LIB_PATH):
    """Load libmprk.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    C = ctypes.POINTER(mprk_config)
    S = ctypes.POINTER(mprk_stats)
    V = ctypes.c_void_p
    lib.mprk_validate.argtypes = [C, ctypes.c_char_p, ctypes.c_size_t]
    lib.mprk_workspace_bytes.argtypes = [C]
    lib.mprk_workspace_bytes.restype = ctypes.c_size_t
    lib.mprk_create.argtypes = [C, V, V, V, ctypes.c_size_t, V, ctypes.POINTER(V)]
    lib.mprk_set_stream.argtypes = [V, V]
    lib.mprk_rhs.argtypes = [V, V, V, V, V, ctypes.c_int]
    lib.mprk_step.argtypes = [V, ctypes.c_double]
    lib.mprk_run.argtypes = [V, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, S]
    lib.mprk_diagnostics.argtypes = [V, S]
    lib.mprk_diagnostics_static.argtypes = [C, V, V, V, S]
    lib.mprk_stable_dt.argtypes = [C, S, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_double)]
    lib.mprk_set_exec.argtypes = [V, ctypes.c_int]
    lib.mprk_set_wait_limit.argtypes = [V, ctypes.c_double]
    lib.mprk_set_tile.argtypes = [V, ctypes.c_int]
    M = ctypes.POINTER(mprk_member)
    lib.mprk_batch_validate.argtypes = [M, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]
    lib.mprk_batch_workspace_bytes.argtypes = [M, ctypes.c_int32]
    lib.mprk_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.mprk_batch_create.argtypes = [M, ctypes.c_int32, V, ctypes.c_size_t, V, ctypes.POINTER(V)]
    lib.mprk_batch_set_exec.argtypes = [V, ctypes.c_int]
    lib.mprk_batch_set_tile.argtypes = [V, ctypes.c_int]
    lib.mprk_batch_set_wait_limit.argtypes = [V, ctypes.c_double]
    lib.mprk_batch_set_dt.argtypes = [V, ctypes.c_int32, ctypes.c_double]
    lib.mprk_batch_set_adaptive.argtypes = [V, ctypes.c_double, ctypes.c_double]
    lib.mprk_batch_get_dt.argtypes = [V, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.mprk_batch_tune.argtypes = [V, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.mprk_batch_run.argtypes = [V, ctypes.c_int64, ctypes.c_int64, S]
    lib.mprk_batch_diagnostics.argtypes = [V, S]
    lib.mprk_batch_destroy.argtypes = [V]
    lib.mprk_profile_enable.argtypes = [V, ctypes.c_int]
    lib.mprk_profile_take.argtypes = [V, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.mprk_destroy.argtypes = [V]
    lib.mprk_strerror.argtypes = [ctypes.c_int]
    lib.mprk_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().mprk_strerror(int(code)).decode()
    except RuntimeError:
        return "status %d" % code


# ---- same-named thin wrappers ---------------------------------------------
def mprk_validate(cfg: mprk_config):
    buf = ctypes.create_string_buffer(256)
    rc = load().mprk_validate(ctypes.byref(cfg), buf, 256)
    return rc, buf.value.decode()


def mprk_workspace_bytes(cfg: mprk_config) -> int:
    return int(load().mprk_workspace_bytes(ctypes.byref(cfg)))


def mprk_create(cfg, q_lower_ptr, q_upper_ptr, ws_ptr, ws_bytes, stream_ptr):
    out = ctypes.c_void_p()
    rc = load().mprk_create(ctypes.byref(cfg), q_lower_ptr, q_upper_ptr, ws_ptr, ws_bytes,
                            stream_ptr, ctypes.byref(out))
    return rc, out.value


def mprk_rhs(ctx, ql, qu, rl, ru, mask):
    return load().mprk_rhs(ctx, ql, qu, rl, ru, int(mask))


def mprk_step(ctx, dt):
    return load().mprk_step(ctx, float(dt))


def mprk_run(ctx, dt, nsteps, check_every):
    st = mprk_stats()
    rc = load().mprk_run(ctx, float(dt), int(nsteps), int(check_every), ctypes.byref(st))
    return rc, st


def mprk_diagnostics(ctx):
    st = mprk_stats()
    rc = load().mprk_diagnostics(ctx, ctypes.byref(st))
    return rc, st


def mprk_diagnostics_static(cfg, q_lower_ptr, q_upper_ptr, stream_ptr):
    """Allocation-free diagnostics of a state pair (no context, no workspace)."""
    st = mprk_stats()
    rc = load().mprk_diagnostics_static(ctypes.byref(cfg), q_lower_ptr, q_upper_ptr, stream_ptr,
                                        ctypes.byref(st))
    return rc, st


def mprk_stable_dt(cfg, st, cr, dn):
    dt = ctypes.c_double()
    rc = load().mprk_stable_dt(ctypes.byref(cfg), ctypes.byref(st), float(cr), float(dn),
                               ctypes.byref(dt))
    return rc, dt.value


def mprk_set_exec(ctx, mode):
    return load().mprk_set_exec(ctx, int(mode))


def mprk_set_wait_limit(ctx, seconds):
    return load().mprk_set_wait_limit(ctx, float(seconds))


def mprk_set_tile(ctx, shape):
    return load().mprk_set_tile(ctx, int(shape))


def mprk_profile_enable(ctx, on):
    return load().mprk_profile_enable(ctx, int(bool(on)))


def mprk_profile_take(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    rc = load().mprk_profile_take(ctx, ctypes.byref(ms), ctypes.byref(n))
    return rc, ms.value, n.value


def mprk_destroy(ctx):
    return load().mprk_destroy(ctx)


def _members(members):
    arr = (mprk_member * len(members))()
    for i, m in enumerate(members):
        arr[i] = m
    return arr


def mprk_batch_validate(members):
    buf = ctypes.create_string_buffer(256)
    rc = load().mprk_batch_validate(_members(members), len(members), buf, 256)
    return rc, buf.value.decode()


def mprk_batch_workspace_bytes(members) -> int:
    return int(load().mprk_batch_workspace_bytes(_members(members), len(members)))


def mprk_batch_create(members, ws_ptr, ws_bytes, stream_ptr):
    out = ctypes.c_void_p()
    rc = load().mprk_batch_create(_members(members), len(members), ws_ptr, ws_bytes, stream_ptr,
                                  ctypes.byref(out))
    return rc, out.value


def mprk_batch_set_exec(b, mode):
    return load().mprk_batch_set_exec(b, int(mode))


def mprk_batch_set_tile(b, shape):
    return load().mprk_batch_set_tile(b, int(shape))


def mprk_batch_set_wait_limit(b, seconds):
    return load().mprk_batch_set_wait_limit(b, float(seconds))


def mprk_batch_set_dt(b, member, dt):
    return load().mprk_batch_set_dt(b, int(member), float(dt))


def mprk_batch_set_adaptive(b, cr, dn):
    return load().mprk_batch_set_adaptive(b, float(cr), float(dn))


def mprk_batch_get_dt(b, member):
    dt = ctypes.c_double()
    rc = load().mprk_batch_get_dt(b, int(member), ctypes.byref(dt))
    return rc, dt.value


def mprk_batch_tune(b, reps):
    ms = (ctypes.c_double * TILE_SHAPES)()
    best = ctypes.c_int32()
    rc = load().mprk_batch_tune(b, int(reps), ms, ctypes.byref(best))
    return rc, list(ms), best.value


def mprk_batch_run(b, n, nsteps, check_every):
    st = (mprk_stats * n)()
    rc = load().mprk_batch_run(b, int(nsteps), int(check_every), st)
    return rc, list(st)


def mprk_batch_diagnostics(b, n):
    st = (mprk_stats * n)()
    rc = load().mprk_batch_diagnostics(b, st)
    return rc, list(st)


def mprk_batch_destroy(b):
    return load().mprk_batch_destroy(b)


# ---- convenience ----------------------------------------------------------
def config(nx, nz_lower, nz_upper, dx, dz_lower, dz_upper, *, fast_is_lower=True, n_buffer=4,
           base_rk=2, m=2, gamma=1.4, prandtl=0.72, mu_lower=1e-3, mu_upper=1e-3, gravity=0.0,
           flux_bits=64, strict_buffer=0, dim=2, ny=1, dy=0.0) -> mprk_config:
    return mprk_config(ABI_VERSION, dim, nx, ny, nz_lower, nz_upper, dx, dy, dz_lower, dz_upper,
                       int(bool(fast_is_lower)), n_buffer, base_rk, m, gamma, prandtl, mu_lower,
                       mu_upper, gravity, flux_bits, strict_buffer)


def config3_of_workload(w, **over) -> mprk_config:
    """Configuration of a 3D workload (inputs.Workload3)."""
    kw = dict(fast_is_lower=w.fast_is_lower, n_buffer=w.n_buffer, base_rk=w.base, m=w.m,
              gamma=w.gamma, prandtl=w.prandtl, mu_lower=w.mu_lower, mu_upper=w.mu_upper,
              gravity=w.gravity, dim=3, ny=w.ny, dy=w.dy)
    kw.update(over)
    return config(w.nx, w.nz_lower, w.nz_upper, w.dx, w.dz_lower, w.dz_upper, **kw)


def config_of_workload(w, **over) -> mprk_config:
    kw = dict(fast_is_lower=w.fast_is_lower, n_buffer=w.n_buffer, base_rk=w.base, m=w.m,
              gamma=w.gamma, prandtl=w.prandtl, mu_lower=w.mu_lower, mu_upper=w.mu_upper,
              gravity=w.gravity)
    kw.update(over)
    return config(w.nx, w.nz_lower, w.nz_upper, w.dx, w.dz_lower, w.dz_upper, **kw)


def _check(rc, where):
    if rc != OK:
        raise MprkError(rc, where)


class Solver:
    """Owns the workspace tensor and the context; the state tensors belong to
    the caller and are updated in place."""

    def __init__(self, cfg: mprk_config, q_lower, q_upper, stream=None, exec_mode=None, tile=None):
        import torch

        for t in (q_lower, q_upper):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("state must be contiguous float64 device tensors")
        if cfg.dim == 3:
            want = (5, cfg.nz_lower, cfg.ny, cfg.nx), (5, cfg.nz_upper, cfg.ny, cfg.nx)
        else:
            want = (4, cfg.nz_lower, cfg.nx), (4, cfg.nz_upper, cfg.nx)
        if tuple(q_lower.shape) != want[0] or tuple(q_upper.shape) != want[1]:
            raise ValueError("state shapes do not match the configuration")
        rc, msg = mprk_validate(cfg)
        _check(rc, "mprk_validate: " + msg)
        self.cfg = cfg
        self.q_lower, self.q_upper = q_lower, q_upper
        nbytes = mprk_workspace_bytes(cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=q_lower.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self._ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(q_lower.device)
        rc, self.ctx = mprk_create(cfg, q_lower.data_ptr(), q_upper.data_ptr(), self._ws_ptr,
                                   nbytes, self.stream.cuda_stream)
        _check(rc, "mprk_create")
        if exec_mode is not None:
            self.set_exec(exec_mode)
        if tile is not None:
            self.set_tile(tile)

    def rhs(self, q_lower, q_upper, r_lower, r_upper, mask=REGION_ALL):
        _check(mprk_rhs(self.ctx, q_lower.data_ptr(), q_upper.data_ptr(), r_lower.data_ptr(),
                        r_upper.data_ptr(), mask), "mprk_rhs")

    def step(self, dt):
        _check(mprk_step(self.ctx, dt), "mprk_step")

    def run(self, dt, nsteps, check_every=0) -> dict:
        rc, st = mprk_run(self.ctx, dt, nsteps, check_every)
        _check(rc, "mprk_run")
        return st.as_dict()

    def diagnostics(self, check=True) -> dict:
        rc, st = mprk_diagnostics(self.ctx)
        if check:
            _check(rc, "mprk_diagnostics")
        return st.as_dict()

    def stable_dt(self, cr=0.5, dn=0.25) -> float:
        rc, st = mprk_diagnostics(self.ctx)
        _check(rc, "mprk_diagnostics")
        rc, dt = mprk_stable_dt(self.cfg, st, cr, dn)
        _check(rc, "mprk_stable_dt")
        return dt

    def set_exec(self, mode: int):
        _check(mprk_set_exec(self.ctx, mode), "mprk_set_exec")

    def set_wait_limit(self, seconds: float):
        _check(mprk_set_wait_limit(self.ctx, seconds), "mprk_set_wait_limit")

    def set_tile(self, shape: int):
        _check(mprk_set_tile(self.ctx, shape), "mprk_set_tile")

    def profile(self, on: bool):
        _check(mprk_profile_enable(self.ctx, on), "mprk_profile_enable")

    def profile_take(self):
        """(summed stage-kernel milliseconds, launches) since the last take."""
        rc, ms, n = mprk_profile_take(self.ctx)
        _check(rc, "mprk_profile_take")
        return ms, n

    def close(self):
        if getattr(self, "ctx", None):
            mprk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_state(t, cfg):
    import torch

    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("state must be contiguous float64 device tensors")


class Batch:
    """A batch of independent members advanced together (``mprk_batch_*``).

    ``members`` is a sequence of (config, q_lower, q_upper, dt); the state
    tensors belong to the caller and are updated in place; the workspace
    tensor belongs to this object."""

    def __init__(self, members, stream=None, exec_mode=None, tile=None):
        import torch

        if not members:
            raise ValueError("empty batch")
        recs = []
        self._keep = []
        for cfg, ql, qu, dt in members:
            _check_state(ql, cfg)
            _check_state(qu, cfg)
            if tuple(ql.shape) != (4, cfg.nz_lower, cfg.nx) or \
                    tuple(qu.shape) != (4, cfg.nz_upper, cfg.nx):
                raise ValueError("state shapes do not match the configuration")
            recs.append(mprk_member(cfg, ql.data_ptr(), qu.data_ptr(), float(dt)))
            self._keep.append((ql, qu))
        rc, msg = mprk_batch_validate(recs)
        _check(rc, "mprk_batch_validate: " + msg)
        self.n = len(recs)
        self.members = recs
        nbytes = mprk_batch_workspace_bytes(recs)
        dev = members[0][1].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        rc, self.b = mprk_batch_create(recs, self.workspace.data_ptr() + off, nbytes,
                                       self.stream.cuda_stream)
        _check(rc, "mprk_batch_create")
        self.workspace_bytes = nbytes
        if exec_mode is not None:
            self.set_exec(exec_mode)
        if tile is not None:
            self.set_tile(tile)

    def set_exec(self, mode: int):
        _check(mprk_batch_set_exec(self.b, mode), "mprk_batch_set_exec")

    def set_tile(self, shape: int):
        _check(mprk_batch_set_tile(self.b, shape), "mprk_batch_set_tile")

    def set_wait_limit(self, seconds: float):
        _check(mprk_batch_set_wait_limit(self.b, seconds), "mprk_batch_set_wait_limit")

    def set_dt(self, member: int, dt: float):
        _check(mprk_batch_set_dt(self.b, member, dt), "mprk_batch_set_dt")
        self.members[member].dt = float(dt)

    def set_adaptive(self, cr: float, dn: float = 0.25):
        _check(mprk_batch_set_adaptive(self.b, cr, dn), "mprk_batch_set_adaptive")

    def dts(self) -> list:
        out = []
        for i in range(self.n):
            rc, dt = mprk_batch_get_dt(self.b, i)
            _check(rc, "mprk_batch_get_dt")
            out.append(dt)
        return out

    def stable_dts(self, cr=0.5, dn=0.25) -> list:
        """Step of each member from its current state (the rule of mprk_stable_dt)."""
        rc, st = mprk_batch_diagnostics(self.b, self.n)
        _check(rc, "mprk_batch_diagnostics")
        out = []
        for m, s in zip(self.members, st):
            rc, dt = mprk_stable_dt(m.cfg, s, cr, dn)
            _check(rc, "mprk_stable_dt")
            out.append(dt)
        return out

    def tune(self, reps: int = 3):
        """(milliseconds per slow step for each tile shape, chosen shape)."""
        rc, ms, best = mprk_batch_tune(self.b, reps)
        _check(rc, "mprk_batch_tune")
        return ms, best

    def run(self, nsteps: int, check_every: int = 0) -> list:
        rc, st = mprk_batch_run(self.b, self.n, nsteps, check_every)
        _check(rc, "mprk_batch_run")
        return [x.as_dict() for x in st]

    def run_status(self, nsteps: int, check_every: int = 0):
        """Like run, but returns (status code, per-member stats) instead of
        raising when a member's state is bad."""
        rc, st = mprk_batch_run(self.b, self.n, nsteps, check_every)
        return rc, [x.as_dict() for x in st]

    def diagnostics(self, check=True) -> list:
        rc, st = mprk_batch_diagnostics(self.b, self.n)
        if check:
            _check(rc, "mprk_batch_diagnostics")
        return [x.as_dict() for x in st]

    def close(self):
        if getattr(self, "b", None):
            mprk_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
