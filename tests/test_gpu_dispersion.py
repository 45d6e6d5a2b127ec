"""The paper's 2D dispersion experiment for electromagnetic waves (Sec. 5.1)
on the HIP path: a point source in E_z on a 128 x 128 grid, m = 20, time
steps 0.1, 0.5, 0.7 and 1.0 of the CFL limit, run to t_max = 256 dx / c; the
recorded E_z(t, x, y) is multiplied by the Hann window sin^2(pi t / t_max),
Fourier transformed in space and time, and the frequency of each lattice
wavevector is the power-weighted mean of the non-negative frequencies.

Checks: the recorded history equals the FP64 oracle's (first steps, 1e-12);
the measured frequencies equal the scheme's exact TM dispersion relation at
m = 20 (the closed form of the per-k step matrix) to 1e-6 wherever the
window's main lobe stays below the Nyquist frequency, and they differ from
the converged (m = infinity) relation, so the test resolves the finite
sweep count; the fastest phase velocity grows as the time step shrinks
(the paper's observation that high-k waves become more superluminal)."""
import math

import numpy as np
import pytest

from oracle import ref, spectral as S
from paper_1907_13088_amd import mx

from gpu_helpers import log

pytestmark = pytest.mark.gpu

N_GRID, M = 128, 20


def _measure(frac):
    import torch
    n = N_GRID
    dt = frac / math.sqrt(2.0)
    nsteps = int(round(256.0 / dt))
    cfg = mx.make_config(2, (n, n), dt, (1.0, 1.0), "f64", mx.MX_TM, M, 0.0, 0)
    g = mx.Grid(cfg)
    E = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
    B = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
    E[2][n // 2, n // 2] = 1.0
    g.bind(E, B)
    rec = torch.empty((nsteps, n, n), dtype=torch.float64, device="cuda")
    for s in range(nsteps):
        g.step(1)
        rec[s].copy_(E[2])
    torch.cuda.synchronize()
    g.close()
    t = (torch.arange(nsteps, dtype=torch.float64, device="cuda") + 1) * dt
    w = torch.sin(math.pi * t / (nsteps * dt)) ** 2
    F = torch.fft.fft2(torch.fft.rfft(rec * w[:, None, None], dim=0), dim=(1, 2))
    P = F.real ** 2 + F.imag ** 2
    om = 2 * math.pi * torch.arange(P.shape[0], dtype=torch.float64, device="cuda") / (nsteps * dt)
    wnum = ((om[:, None, None] * P).sum(0) / P.sum(0)).cpu().numpy()
    return dt, nsteps, rec[:40].cpu().numpy(), wnum


def test_point_source_dispersion_matches_finite_m_relation():
    n = N_GRID
    kk = 2 * math.pi * np.fft.fftfreq(n)
    vmax = {}
    for frac in (1.0, 0.7, 0.5, 0.1):
        dt, nsteps, head, wnum = _measure(frac)
        # parity of the recorded history with the oracle
        cfg = ref.Config(ndim=2, shape=(n, n), dt=dt, blocks=2, sweeps=M)
        E = [np.zeros((n, n)) for _ in range(3)]
        B = [np.zeros((n, n)) for _ in range(3)]
        E[2][n // 2, n // 2] = 1.0
        err = 0.0
        for s in range(head.shape[0]):
            ref.step(cfg, E, B)
            err = max(err, float(np.abs(head[s] - E[2]).max()))
        assert err < 1e-12, (frac, err)
        dev20, devinf, vph = 0.0, 0.0, 0.0
        for jy in range(n):
            for ix in range(n):
                k = (kk[ix], kk[jy])
                kn = math.hypot(*k)
                if kn < 0.3:
                    continue
                w20 = S.omega_tm_closed(k, (1, 1), dt, M)
                if w20 * dt > 0.95 * math.pi:   # the window's lobe would wrap past Nyquist
                    continue
                winf = S.omega_tm_closed(k, (1, 1), dt, None)
                dev20 = max(dev20, abs(wnum[jy, ix] - w20))
                devinf = max(devinf, abs(wnum[jy, ix] - winf))
                vph = max(vph, wnum[jy, ix] / kn)
        vmax[frac] = vph
        log(f"dt = {frac} dt_CFL, {nsteps} steps: max |w - w_20| {dev20:.2e}, max |w - w_inf| {devinf:.2e}, "
            f"max v_ph {vph:.5f}, history vs oracle {err:.1e}")
        assert dev20 < 1e-6, (frac, dev20)
        assert devinf > 1e3 * dev20, (frac, devinf, dev20)
    assert vmax[0.1] > vmax[0.5] > vmax[0.7] > vmax[1.0] > 1.0, vmax
