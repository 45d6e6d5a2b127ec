"""ctypes binding of the C ABI in include/mx.h (argument marshalling only).

Every step of the field update runs in the HIP library ``libmx.so``; this
module only converts torch tensors to device pointers and Python values to
the C structs.  It raises if the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import sys
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmx.so")

MX_OK, MX_EINVAL, MX_ECFL, MX_EWORKSPACE, MX_EDEVICE, MX_ENONFINITE, MX_ESTATE = 0, -1, -2, -3, -4, -5, -6
MX_F32, MX_F64 = 0, 1
MX_TE, MX_TM, MX_ALL = 1, 2, 3
FORM_STANDARD, FORM_DELTA = 0, 1
VARIANT_AUTO, VARIANT_TILE, VARIANT_STREAM, VARIANT_STREAM_BLOCK, VARIANT_STREAM_FUSED = 0, 1, 2, 3, 4
SOLVER_ALG1, SOLVER_CHEBYSHEV = 0, 1
WARN_NOCONV_GUARANTEE = 1

EXPORTS = ["mx_profile_enable", "mx_profile_read", "mx_last_error", "mx_config_default", "mx_validate", "mx_workspace_size", "mx_init",
           "mx_bind_fields", "mx_set_current", "mx_step", "mx_get_step", "mx_set_step",
           "mx_get_sweeps_per_pass", "mx_get_block_sweeps_per_pass", "mx_destroy", "mx_adjoint", "mx_sources_assemble",
           "mx_sources_project", "mx_batch_workspace_size", "mx_batch_init", "mx_batch_bind",
           "mx_batch_step", "mx_batch_get_plan", "mx_batch_get_schedule", "mx_batch_destroy",
           "mx_step_static", "mx_pic_push", "mx_pic_charge"]
STATIC_SCRATCH_BYTES = 64 << 20   # MX_STATIC_SCRATCH_BYTES


class MxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mx error {code}: {msg}")
        self.code = code


class CConfig(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int64 * 3), ("d", C.c_double * 3), ("dt", C.c_double),
                ("dtype", C.c_int), ("blocks", C.c_int), ("sweeps", C.c_int), ("tol", C.c_double),
                ("filter_passes", C.c_int), ("lumped", C.c_int), ("four_pi", C.c_double),
                ("form", C.c_int), ("sweeps_per_pass", C.c_int), ("variant", C.c_int),
                ("solver", C.c_int)]


class CProfile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 7), ("ms", C.c_double * 7), ("bytes", C.c_double * 7)]


PROF_CATEGORIES = ("front", "sweep", "other", "adjoint", "sweep_last", "particles", "front_sweep")


class CStats(C.Structure):
    _fields_ = [("sweeps", C.c_int * 2), ("resid", C.c_double * 2), ("rhs", C.c_double * 2),
                ("nonconverged", C.c_int * 2)]


_lib = None


def lib():
    """Load libmx.so (built by paper_1907_13088_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_1907_13088_amd.build)")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libmx bind to that one, so the process holds a single
        # runtime (tensors allocated by torch are then known to libmx)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        P = C.POINTER
        L.mx_last_error.restype = C.c_char_p
        L.mx_config_default.argtypes = [P(CConfig)]
        L.mx_validate.argtypes = [P(CConfig), P(C.c_int)]
        L.mx_workspace_size.argtypes = [P(CConfig), P(C.c_size_t)]
        L.mx_init.argtypes = [P(CConfig), vp, vp, C.c_size_t, P(vp)]
        L.mx_bind_fields.argtypes = [vp, P(vp), P(vp)]
        L.mx_set_current.argtypes = [vp, P(vp)]
        L.mx_step.argtypes = [vp, C.c_int, P(C.c_double), P(C.c_int), P(CStats)]
        L.mx_get_step.argtypes = [vp, P(C.c_int64)]
        L.mx_set_step.argtypes = [vp, C.c_int64]
        L.mx_get_sweeps_per_pass.argtypes = [vp, P(C.c_int)]
        L.mx_get_block_sweeps_per_pass.argtypes = [vp, P(C.c_int)]
        L.mx_destroy.argtypes = [vp]
        L.mx_profile_enable.argtypes = [vp, C.c_int]
        L.mx_profile_read.argtypes = [vp, P(CProfile)]
        L.mx_adjoint.argtypes = [vp, C.c_int, P(C.c_double), P(C.c_int), P(vp), P(vp), P(vp)]
        L.mx_sources_assemble.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, P(vp)]
        L.mx_sources_project.argtypes = [vp, C.c_int, C.c_int, vp, vp, P(vp), vp]
        L.mx_step_static.argtypes = [P(CConfig), vp, P(vp), P(vp), P(vp), C.c_int, P(C.c_double), P(C.c_int),
                                     P(CStats)]
        L.mx_pic_push.argtypes = [vp, C.c_int64, C.c_double, C.c_double, C.c_double, P(vp), P(vp), P(vp), C.c_int]
        L.mx_pic_charge.argtypes = [vp, C.c_int64, C.c_double, C.c_double, P(vp), vp, C.c_int]
        if hasattr(L, "mx_batch_init"):
            L.mx_batch_workspace_size.argtypes = [P(CConfig), C.c_int, P(C.c_size_t)]
            L.mx_batch_init.argtypes = [P(CConfig), C.c_int, vp, vp, C.c_size_t, P(vp)]
            L.mx_batch_bind.argtypes = [vp, C.c_int, P(vp), P(vp)]
            L.mx_batch_step.argtypes = [vp, C.c_int, C.c_int]
            L.mx_batch_get_plan.argtypes = [vp, P(C.c_int), P(C.c_int), P(C.c_int)]
            L.mx_batch_get_schedule.argtypes = [vp, C.c_int, P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int)]
            L.mx_batch_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != MX_OK:
        raise MxError(rc, lib().mx_last_error().decode())


def make_config(ndim: int, n: Sequence[int], dt: float, d: Sequence[float] = (1.0, 1.0, 1.0),
                dtype: str = "f32", blocks: int = MX_ALL, sweeps: int = 20, tol: float = 0.0,
                filter_passes: int = 0, lumped: bool = False, four_pi: float = 4.0 * math.pi,
                form: int = FORM_STANDARD, sweeps_per_pass: int = 0, variant: int = 0,
                solver: int = 0) -> CConfig:
    """n and d are in axis order (x, y[, z])."""
    c = CConfig()
    lib().mx_config_default(C.byref(c))
    c.ndim = ndim
    nn = list(n) + [1] * (3 - len(n))
    dd = list(d) + [1.0] * (3 - len(d))
    for a in range(3):
        c.n[a] = int(nn[a])
        c.d[a] = float(dd[a])
    c.dt = float(dt)
    c.dtype = MX_F64 if dtype in ("f64", "float64", "double") else MX_F32
    c.blocks = int(blocks)
    c.sweeps = int(sweeps)
    c.tol = float(tol)
    c.filter_passes = int(filter_passes)
    c.lumped = int(bool(lumped))
    c.four_pi = float(four_pi)
    c.form = int(form)
    c.sweeps_per_pass = int(sweeps_per_pass)
    c.variant = int(variant)
    c.solver = int(solver)
    return c


def validate(cfg: CConfig) -> int:
    w = C.c_int(0)
    _check(lib().mx_validate(C.byref(cfg), C.byref(w)))
    return w.value


def workspace_size(cfg: CConfig) -> int:
    b = C.c_size_t(0)
    _check(lib().mx_workspace_size(C.byref(cfg), C.byref(b)))
    return b.value


def _device(device):
    import torch
    d = torch.device(device if device is not None else "cuda")
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _ptrs(ts) -> "C.Array":
    return (C.c_void_p * 3)(*[C.c_void_p(t.data_ptr()) for t in ts])


@dataclass
class Stats:
    sweeps: tuple
    resid: tuple
    rhs: tuple
    nonconverged: tuple


def _step_args(nsteps, env, replay, stats):
    envp = None
    if env is not None:
        assert len(env) >= nsteps
        envp = (C.c_double * max(nsteps, 1))(*[float(x) for x in env[:nsteps]])
    rp = None
    if replay is not None:
        flat = []
        for s in range(nsteps):
            flat += [int(replay[s][0]), int(replay[s][1])]
        rp = (C.c_int * max(2 * nsteps, 1))(*flat)
    st = (CStats * max(nsteps, 1))() if stats else None
    return envp, rp, st


def _stats_list(st, nsteps):
    return [Stats(tuple(x.sweeps), tuple(x.resid), tuple(x.rhs), tuple(x.nonconverged)) for x in st[:nsteps]]


def step_static(cfg: CConfig, E: Sequence, B: Sequence, J0: Optional[Sequence] = None, nsteps: int = 1,
                env: Optional[Sequence[float]] = None, replay: Optional[Sequence[Sequence[int]]] = None,
                stats: bool = False, stream=None) -> Optional[List["Stats"]]:
    """mx_step_static: nsteps steps of (E, B) in place on the library's static
    device scratch (no allocation; configs up to STATIC_SCRATCH_BYTES of
    workspace), on the current device and the given (default: current) stream."""
    import torch
    validate(cfg)
    td = torch.float64 if cfg.dtype == MX_F64 else torch.float32
    for t in list(E) + list(B) + (list(J0) if J0 is not None else []):
        if t.dtype != td or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"fields must be contiguous {td} CUDA tensors")
    s = stream if stream is not None else torch.cuda.current_stream()
    envp, rp, st = _step_args(nsteps, env, replay, stats)
    _check(lib().mx_step_static(C.byref(cfg), C.c_void_p(s.cuda_stream), _ptrs(E), _ptrs(B),
                                _ptrs(J0) if J0 is not None else None, nsteps, envp, rp, st))
    return _stats_list(st, nsteps) if stats else None


class Grid:
    """One periodic grid and its bound state (torch tensors on the GPU)."""

    def __init__(self, cfg: CConfig, device=None, stream=None):
        import torch
        self.cfg = cfg
        self.torch_dtype = torch.float64 if cfg.dtype == MX_F64 else torch.float32
        self.device = _device(device)
        validate(cfg)
        nbytes = workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().mx_init(C.byref(cfg), C.c_void_p(self.stream.cuda_stream),
                             C.c_void_p(self.workspace.data_ptr()), nbytes, C.byref(h)))
        self.h = h
        self.E = self.B = self.J0 = None

    @property
    def shape(self):
        c = self.cfg
        return (int(c.n[1]), int(c.n[0])) if c.ndim == 2 else (int(c.n[2]), int(c.n[1]), int(c.n[0]))

    def _check_field(self, t):
        if (t.dtype != self.torch_dtype or t.device != self.device or not t.is_contiguous()
                or tuple(t.shape) != self.shape):
            raise ValueError(f"field must be a contiguous {self.torch_dtype} tensor of shape {self.shape} "
                             f"on {self.device}")

    def bind(self, E: Sequence, B: Sequence):
        for t in list(E) + list(B):
            self._check_field(t)
        self.E, self.B = list(E), list(B)
        _check(lib().mx_bind_fields(self.h, _ptrs(self.E), _ptrs(self.B)))

    def set_current(self, J0: Optional[Sequence]):
        if J0 is None:
            self.J0 = None
            _check(lib().mx_set_current(self.h, None))
            return
        for t in J0:
            self._check_field(t)
        self.J0 = list(J0)
        _check(lib().mx_set_current(self.h, _ptrs(self.J0)))

    def step(self, nsteps: int, env: Optional[Sequence[float]] = None,
             replay: Optional[Sequence[Sequence[int]]] = None, stats: bool = False) -> Optional[List[Stats]]:
        envp, rp, st = _step_args(nsteps, env, replay, stats)
        _check(lib().mx_step(self.h, nsteps, envp, rp, st))
        return _stats_list(st, nsteps) if stats else None

    def adjoint(self, nsteps: int, env: Optional[Sequence[float]], sweeps: Sequence[Sequence[int]],
                Ebar: Sequence, Bbar: Sequence, dJ0: Optional[Sequence] = None):
        for t in list(Ebar) + list(Bbar) + (list(dJ0) if dJ0 is not None else []):
            self._check_field(t)
        envp = (C.c_double * max(nsteps, 1))(*([float(x) for x in env[:nsteps]] if env is not None else [0.0] * max(nsteps, 1)))
        flat = []
        for s in range(nsteps):
            flat += [int(sweeps[s][0]), int(sweeps[s][1])]
        sp = (C.c_int * max(2 * nsteps, 1))(*(flat or [0]))
        _check(lib().mx_adjoint(self.h, nsteps, envp, sp, _ptrs(Ebar), _ptrs(Bbar),
                                _ptrs(dJ0) if dJ0 is not None else None))

    def sources_assemble(self, origins, shapes, amps, J0: Sequence):
        nsrc, W = int(shapes.shape[0]), int(shapes.shape[-1])
        _check(lib().mx_sources_assemble(self.h, nsrc, W, C.c_void_p(origins.data_ptr()),
                                         C.c_void_p(shapes.data_ptr()), C.c_void_p(amps.data_ptr()),
                                         _ptrs(J0)))

    def sources_project(self, origins, shapes, G: Sequence, grad):
        nsrc, W = int(shapes.shape[0]), int(shapes.shape[-1])
        _check(lib().mx_sources_project(self.h, nsrc, W, C.c_void_p(origins.data_ptr()),
                                        C.c_void_p(shapes.data_ptr()), _ptrs(G), C.c_void_p(grad.data_ptr())))

    def pic_push(self, q: float, m: float, w: float, pos: Sequence, u: Sequence, J: Sequence,
                 accumulate: bool = False):
        """One Boris push of a species (pos = (x, y), u = gamma v, device
        vectors in the grid dtype, updated in place) in the bound fields; its
        current J^{n+1/2} overwrites J (or is added with accumulate=True)."""
        np_ = int(pos[0].numel())
        for t in list(pos) + list(u):
            if t.dtype != self.torch_dtype or not t.is_contiguous() or t.numel() != np_:
                raise ValueError("particle arrays must be contiguous vectors of one length in the grid dtype")
        for t in J:
            self._check_field(t)
        _check(lib().mx_pic_push(self.h, np_, float(q), float(m), float(w), _ptrs(pos), _ptrs(u), _ptrs(J),
                                 int(bool(accumulate))))

    def pic_charge(self, q: float, w: float, pos: Sequence, rho, accumulate: bool = False):
        """Charge density of a species at the nodes (overwrites rho, or adds)."""
        self._check_field(rho)
        _check(lib().mx_pic_charge(self.h, int(pos[0].numel()), float(q), float(w), _ptrs(pos),
                                   C.c_void_p(rho.data_ptr()), int(bool(accumulate))))

    def profile_enable(self, on: bool = True):
        """True: reset the per-kernel timers and record; False: pause."""
        _check(lib().mx_profile_enable(self.h, int(bool(on))))

    def profile_resume(self):
        """Record again without resetting (sample some steps of a run)."""
        _check(lib().mx_profile_enable(self.h, 2))

    def profile_read(self) -> dict:
        p = CProfile()
        _check(lib().mx_profile_read(self.h, C.byref(p)))
        return {name: {"launches": int(p.launches[i]), "ms": float(p.ms[i]), "bytes": float(p.bytes[i])}
                for i, name in enumerate(PROF_CATEGORIES)}

    @property
    def step_count(self) -> int:
        n = C.c_int64()
        _check(lib().mx_get_step(self.h, C.byref(n)))
        return n.value

    @step_count.setter
    def step_count(self, n: int):
        _check(lib().mx_set_step(self.h, int(n)))

    @property
    def sweeps_per_pass(self) -> int:
        k = C.c_int()
        _check(lib().mx_get_sweeps_per_pass(self.h, C.byref(k)))
        return k.value

    @property
    def block_sweeps_per_pass(self) -> tuple:
        """(TE, TM) sweeps per pass (3D: first entry)."""
        k = (C.c_int * 2)()
        _check(lib().mx_get_block_sweeps_per_pass(self.h, k))
        return (k[0], k[1])

    def close(self):
        if getattr(self, "h", None):
            lib().mx_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone: leave
        # the handle to the process exit instead of calling into it (the
        # check is bound at definition: module globals such as sys may
        # already be cleared when this runs)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent 2D grids stepped together (mx_batch_*)."""

    def __init__(self, cfgs: Sequence[CConfig], device=None, stream=None):
        import torch
        self.cfgs = list(cfgs)
        arr = (CConfig * len(cfgs))(*cfgs)
        self._arr = arr
        self.device = _device(device)
        b = C.c_size_t(0)
        _check(lib().mx_batch_workspace_size(arr, len(cfgs), C.byref(b)))
        self.workspace = torch.empty(max(b.value, 256), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().mx_batch_init(arr, len(cfgs), C.c_void_p(self.stream.cuda_stream),
                                   C.c_void_p(self.workspace.data_ptr()), b.value, C.byref(h)))
        self.h = h
        self.fields = [None] * len(cfgs)

    def bind(self, g: int, E, B):
        self.fields[g] = (list(E), list(B))
        _check(lib().mx_batch_bind(self.h, g, _ptrs(E), _ptrs(B)))

    def step(self, nsteps: int, persistent: bool = False):
        _check(lib().mx_batch_step(self.h, nsteps, int(bool(persistent))))

    def plan(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(lib().mx_batch_get_plan(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {"sweeps_per_pass": a.value, "tiles": b.value, "persistent_blocks": c.value}

    def schedule(self, persistent):
        """The tuned shape of one schedule: deepest pass, chunk rows of the
        sweep and of the front work items, work items of one step."""
        a, b, f, c = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _check(lib().mx_batch_get_schedule(self.h, int(bool(persistent)), C.byref(a), C.byref(b), C.byref(f),
                                           C.byref(c)))
        return {"sweeps_per_pass": a.value, "chunk_rows": b.value, "front_rows": f.value, "items_per_step": c.value}

    def close(self):
        if getattr(self, "h", None):
            lib().mx_batch_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone: leave
        # the handle to the process exit instead of calling into it (the
        # check is bound at definition: module globals such as sys may
        # already be cleared when this runs)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
