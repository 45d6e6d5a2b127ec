"""The full-size workloads held to their stated accuracy over their whole
run length (through the C-ABI).

* 4096^2 TE+TM, FP32, current with 3 filter passes, m = 20, 1000 steps: the
  FP32 state stays within 1e-5 (normwise) of the FP64 GPU state on the same
  inputs; the FP64 path is itself pinned to the oracle to 1e-12 per step in
  the parity tests.  The frequencies of two probed lattice modes, fitted
  from their Fourier amplitudes over the last steps, agree between the two
  precisions and with the eigenvalues of the finite-m step matrix T(k).
* 512^3, FP32, tolerance 1e-7 (delta form), 200 steps: every step converges
  and the FP32 state stays within 1e-5 of an FP64 run replaying its counts.
(The 2048^2 adjoint over its 500 steps is held to the oracle's gradients in
test_gpu_adjoint.py.)
"""
import math

import numpy as np
import pytest

from oracle import spectral as S
from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _omega_fit(series, dt):
    """Angular frequency of a series a_n = c+ e^{-i w n dt} + c- e^{i w n dt}
    from a_{n+1} + a_{n-1} = 2 cos(w dt) a_n, least squares."""
    a = np.asarray(series)
    c = (np.vdot(a[1:-1], a[2:] + a[:-2]) / (2.0 * np.vdot(a[1:-1], a[1:-1]))).real
    return math.acos(max(-1.0, min(1.0, c))) / dt


def _project(F, k, offset):
    """(2/N) sum F exp(-i k.(x + offset)) of a 2D device tensor, in FP64."""
    import torch
    ny, nx = F.shape
    ex = torch.exp(-1j * k[0] * (torch.arange(nx, dtype=torch.float64, device=F.device) + offset[0]))
    ey = torch.exp(-1j * k[1] * (torch.arange(ny, dtype=torch.float64, device=F.device) + offset[1]))
    return complex(2.0 * (ey @ (F.double().to(torch.complex128) @ ex)) / F.numel())


@pytest.mark.timeout(900)
def test_modes_2d_4096_fp32_within_1e5_of_fp64_after_1000_steps():
    import torch
    w = I.modes_2d()    # 4096^2, 256 modes, 64 pulses, p = 3, m = 20, 1000 steps, FP32 inputs
    n = w.shape[0]
    nsteps, tail = w.steps, 8
    env = [float(x) for x in w.env]
    probes = sorted([md for md in w.meta["modes"] if math.hypot(*S.lattice_k(md["n"], (n, n))) > 1.0],
                    key=lambda md: -abs(md["amp"]))[:2]
    state, series = {}, {}
    for dtype in ("f32", "f64"):
        td = torch.float32 if dtype == "f32" else torch.float64
        log(f"4096^2 x {nsteps} steps, {dtype}")
        g = mx.Grid(mx.make_config(2, (n, n), w.dt, (1.0, 1.0), dtype, mx.MX_ALL, w.sweeps, 0.0, w.filter_passes))
        E = [torch.tensor(a, dtype=td, device="cuda") for a in w.E]
        B = [torch.tensor(a, dtype=td, device="cuda") for a in w.B]
        J = [torch.tensor(a, dtype=td, device="cuda") for a in w.J0]
        g.bind(E, B)
        g.set_current(J)
        g.step(nsteps - tail, env[:nsteps - tail])
        ser = [[] for _ in probes]
        for s in range(nsteps - tail, nsteps + 1):
            for i, md in enumerate(probes):
                k = S.lattice_k(md["n"], (n, n))
                F, off = (B[2], I.B_OFFSETS[2][2]) if md["pol"] == "TE" else (E[2], I.E_OFFSETS[2][2])
                ser[i].append(_project(F, k, off))
            if s < nsteps:
                g.step(1, env[s:s + 1])
        torch.cuda.synchronize()
        state[dtype] = [t.double() for t in E + B]
        series[dtype] = ser
        del g, E, B, J
        torch.cuda.empty_cache()
    scale = max(float(t.abs().max()) for t in state["f64"])
    err = max(float((a - b).abs().max()) for a, b in zip(state["f32"], state["f64"])) / scale
    log(f"4096^2 after {nsteps} steps: FP32 vs FP64 normwise {err:.2e}")
    assert err <= 1e-5
    for i, md in enumerate(probes):
        k = S.lattice_k(md["n"], (n, n))
        exact = S.omega_numeric(k, (1.0, 1.0), w.dt, w.sweeps)
        w32, w64 = _omega_fit(series["f32"][i], w.dt), _omega_fit(series["f64"][i], w.dt)
        ex = float(exact[np.argmin(np.abs(exact - w64))])
        log(f"mode {md['n']} {md['pol']}: omega fp32 {w32:.12f} fp64 {w64:.12f} T(k) {ex:.12f}; "
            f"fp32 vs fp64 {abs(w32 - w64) / w64:.2e}, fp64 vs T(k) {abs(w64 - ex) / ex:.2e}")
        assert abs(w64 - ex) <= 1e-9 * ex
        assert abs(w32 - w64) <= 1e-6 * w64


@pytest.mark.timeout(900)
def test_planewave_3d_512_fp32_within_1e5_of_fp64_after_200_steps():
    import torch
    w = I.planewave_3d()    # 512^3, 32 pulses, p = 1, tol 1e-7, m_max 300, 200 steps, FP32 inputs
    nsteps = w.steps
    env = [float(x) for x in w.env]
    n = w.shape[::-1]
    log(f"512^3 x {nsteps} steps, FP32 delta form to tol {w.tol}")
    g = mx.Grid(mx.make_config(3, n, w.dt, w.d, "f32", 3, w.sweeps, w.tol, w.filter_passes, form=mx.FORM_DELTA))
    E = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in w.E]
    B = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in w.B]
    J = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in w.J0]
    g.bind(E, B)
    g.set_current(J)
    st = []
    for s0 in range(0, nsteps, 50):
        st += g.step(50, env[s0:s0 + 50], stats=True)
        log(f"  fp32 step {s0 + 50}: sweeps {st[-1].sweeps[0]}")
    torch.cuda.synchronize()
    assert not any(s.nonconverged[0] for s in st)
    counts = [s.sweeps for s in st]
    log(f"sweeps per step: mean {np.mean([c[0] for c in counts]):.1f}, range {min(c[0] for c in counts)}.."
        f"{max(c[0] for c in counts)}")
    f32 = [t.clone() for t in E + B]
    del g, E, B, J
    torch.cuda.empty_cache()
    log("FP64 run replaying the FP32 counts")
    g = mx.Grid(mx.make_config(3, n, w.dt, w.d, "f64", 3, w.sweeps, w.tol, w.filter_passes))
    E = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in w.E]
    B = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in w.B]
    J = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in w.J0]
    g.bind(E, B)
    g.set_current(J)
    for s0 in range(0, nsteps, 50):
        g.step(50, env[s0:s0 + 50], replay=counts[s0:s0 + 50])
        torch.cuda.synchronize()
        log(f"  fp64 step {s0 + 50}")
    scale = max(float(t.abs().max()) for t in E + B)
    err = max(float((a.double() - b).abs().max()) for a, b in zip(f32, E + B)) / scale
    log(f"512^3 after {nsteps} steps: FP32 vs FP64 normwise {err:.2e}")
    assert err <= 1e-5
