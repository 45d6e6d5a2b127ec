"""The allocation-free entry point mx_step_static (through the C-ABI) against
mx_init + mx_step on the same inputs: the same kernels run on the library's
static scratch instead of a caller workspace, so the states agree bitwise.
Two calls in a row, the second with a smaller grid (the scratch keeps the
first call's contents), in a fixed-count and in a tolerance configuration;
a config whose workspace exceeds the static scratch is refused on the host."""
import numpy as np
import pytest

from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import gpu_config, log, torch_fields

pytestmark = pytest.mark.gpu


def _via_grid(w, cfg, nsteps):
    import torch
    g = mx.Grid(cfg)
    E, B = torch_fields(w.E, w.dtype), torch_fields(w.B, w.dtype)
    g.bind(E, B)
    if w.J0 is not None:
        g.set_current(torch_fields(w.J0, w.dtype))
    st = g.step(nsteps, env=None if w.env is None else list(w.env[:nsteps]), stats=True)
    torch.cuda.synchronize()
    g.close()
    return E + B, st


def _via_static(w, cfg, nsteps):
    import torch
    E, B = torch_fields(w.E, w.dtype), torch_fields(w.B, w.dtype)
    J = torch_fields(w.J0, w.dtype) if w.J0 is not None else None
    st = mx.step_static(cfg, E, B, J, nsteps, env=None if w.env is None else list(w.env[:nsteps]), stats=True)
    torch.cuda.synchronize()
    return E + B, st


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_static_step_equals_workspace_step_two_calls(dtype):
    import torch
    big = I.modes_2d((200, 136), nmodes=48, npulses=8, filter_passes=3, m=20, steps=5, seed=4101, dtype=dtype)
    small = I.modes_2d((72, 40), nmodes=12, npulses=3, filter_passes=1, m=20, steps=7, seed=4102, dtype=dtype)
    for w, nsteps in ((big, 5), (small, 7)):
        cfg = gpu_config(w)
        want, _ = _via_grid(w, cfg, nsteps)
        got, _ = _via_static(w, cfg, nsteps)
        for a, b in zip(got, want):
            assert torch.equal(a, b)
        log(f"static step {w.shape} {dtype} x {nsteps}: bitwise equal to mx_step")


def test_static_step_tolerance_two_calls():
    import torch
    te = I.planewave_te_2d(n=128, steps=6)                  # FP64, tol 1e-12
    small = I.modes_2d((64, 48), nmodes=10, npulses=2, filter_passes=2, m=150, steps=4, seed=4103, dtype="f64")
    for w, nsteps, tol in ((te, 6, None), (small, 4, 1e-10)):
        cfg = gpu_config(w, tol=tol)
        want, stw = _via_grid(w, cfg, nsteps)
        got, stg = _via_static(w, cfg, nsteps)
        assert [s.sweeps for s in stg] == [s.sweeps for s in stw]
        assert all(s.sweeps[0] > 0 for s in stg)
        for a, b in zip(got, want):
            assert torch.equal(a, b)
        log(f"static tolerance step {w.shape} x {nsteps}: counts {[s.sweeps for s in stg]}, bitwise equal")


def test_static_step_refuses_configs_beyond_the_scratch():
    import torch
    cfg = mx.make_config(2, (4096, 4096), 0.3, (1.0, 1.0), "f32", mx.MX_ALL, 20, 0.0, 0)
    assert mx.workspace_size(cfg) > mx.STATIC_SCRATCH_BYTES
    E = [torch.zeros((4096, 4096), dtype=torch.float32, device="cuda") for _ in range(3)]
    B = [torch.zeros_like(E[0]) for _ in range(3)]
    with pytest.raises(mx.MxError) as ei:
        mx.step_static(cfg, E, B, None, 1)
    assert ei.value.code == mx.MX_EWORKSPACE and "static scratch" in str(ei.value)
    cheb = mx.make_config(2, (64, 64), 0.3, (1.0, 1.0), "f64", mx.MX_ALL, 5, 0.0, 0, solver=mx.SOLVER_CHEBYSHEV)
    E = [torch.zeros((64, 64), dtype=torch.float64, device="cuda") for _ in range(3)]
    B = [torch.zeros_like(E[0]) for _ in range(3)]
    with pytest.raises(mx.MxError) as ei:
        mx.step_static(cheb, E, B, None, 1)
    assert ei.value.code == mx.MX_EINVAL
