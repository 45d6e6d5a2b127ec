"""Helpers for the GPU parity tests: run a workload through the HIP library
(via the C-ABI binding) and through the FP64 oracle on the same inputs."""
import math
import sys
import time

import numpy as np

from oracle import ref
from paper_1907_13088_amd import mx


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def torch_fields(arrs, dtype):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    return [torch.tensor(a, dtype=td, device="cuda").contiguous() for a in arrs]


def to_np(ts):
    return [t.detach().cpu().double().numpy() for t in ts]


def gpu_config(w, dtype=None, spp=0, form=mx.FORM_STANDARD, sweeps=None, tol=None, blocks=None,
               lumped=False, variant=0, solver=0):
    n = w.shape[::-1]
    return mx.make_config(w.ndim, n, w.dt, w.d, dtype or w.dtype, blocks if blocks is not None else w.blocks,
                          w.sweeps if sweeps is None else sweeps, w.tol if tol is None else tol,
                          w.filter_passes, lumped=lumped, form=form, sweeps_per_pass=spp, variant=variant,
                          solver=solver)


def run_gpu(w, nsteps, dtype=None, spp=0, form=mx.FORM_STANDARD, replay=None, sweeps=None, tol=None,
            blocks=None, lumped=False, E=None, B=None, variant=0, solver=0):
    import torch
    dt_ = dtype or w.dtype
    cfg = gpu_config(w, dt_, spp, form, sweeps, tol, blocks, lumped, variant, solver)
    g = mx.Grid(cfg)
    Et = torch_fields(w.E if E is None else E, dt_)
    Bt = torch_fields(w.B if B is None else B, dt_)
    g.bind(Et, Bt)
    if w.J0 is not None:
        Jt = torch_fields(w.J0, dt_)
        g.set_current(Jt)
    env = None if w.env is None else list(w.env[:nsteps])
    st = g.step(nsteps, env=env, replay=replay, stats=True)
    torch.cuda.synchronize()
    out = (to_np(Et), to_np(Bt), st, g.sweeps_per_pass)
    g.close()
    return out


def oracle_config(w, sweeps=None, tol=None, check_every=1, blocks=None, lumped=False, solver=0):
    return ref.Config(ndim=w.ndim, shape=w.shape, dt=w.dt, d=w.d,
                      blocks=w.blocks if blocks is None else blocks,
                      sweeps=w.sweeps if sweeps is None else sweeps, tol=w.tol if tol is None else tol,
                      check_every=check_every, filter_passes=w.filter_passes, lumped=lumped, solver=solver)


def run_oracle(w, nsteps, sweeps=None, tol=None, check_every=1, replay=None, blocks=None, lumped=False,
               solver=0):
    cfg = oracle_config(w, sweeps, tol, check_every, blocks, lumped, solver)
    E = [a.copy() for a in w.E]
    B = [a.copy() for a in w.B]
    t0 = time.time()
    st = ref.run(cfg, E, B, nsteps, w.J0, None if w.env is None else w.env, replay)
    log(f"oracle {w.name} {w.shape} x {nsteps} steps: {time.time() - t0:.1f}s")
    return E, B, st


def rel_err(got, want):
    """Normwise relative error of the state: max |got - want| of each
    component over the max norm of the whole compared state (a component that
    only carries small noise is measured against the field scale, not its own)."""
    scale = max(float(np.abs(w_).max()) for w_ in want)
    if scale == 0.0:
        scale = 1.0
    return [float(np.abs(g_ - w_).max() / scale) for g_, w_ in zip(got, want)]
