"""Shared helpers for the oracle pin tests (CPU only)."""
import math

import numpy as np

from oracle import ref, spectral as S
from paper_1907_13088_amd.inputs import B_OFFSETS, E_OFFSETS


def plane(shape, k, off, phase=0.0):
    """cos(k.(x + off) + phase) on a periodic grid shaped (ny, nx) or (nz, ny, nx)."""
    nd = len(shape)
    acc = np.zeros(shape)
    for ax in range(nd):
        n = shape[nd - 1 - ax]
        x = np.arange(n) + off[ax]
        s = [1] * nd
        s[nd - 1 - ax] = n
        acc = acc + (k[ax] * x).reshape(s)
    return np.cos(acc + phase)


def omega_from_series(a, dt):
    """Angular frequency from a series a_n = c+ e^{i w n dt} + c- e^{-i w n dt}:
    a_{n+1} + a_{n-1} = 2 cos(w dt) a_n (least squares over the series)."""
    a = np.asarray(a)
    num = np.vdot(a[1:-1], a[2:] + a[:-2])
    den = 2.0 * np.vdot(a[1:-1], a[1:-1])
    c = (num / den).real
    return math.acos(max(-1.0, min(1.0, c))) / dt


def mode_2d(n, kidx, pol, amp=1.0):
    """Single lattice mode in 2D: pol 'TM' sets E_z, pol 'TE' sets the
    in-plane E transverse to k (continuum sense); B starts at zero."""
    ny, nx = n
    k = (2 * math.pi * kidx[0] / nx, 2 * math.pi * kidx[1] / ny)
    shape = (ny, nx)
    E = [np.zeros(shape) for _ in range(3)]
    B = [np.zeros(shape) for _ in range(3)]
    if pol == "TM":
        E[2] = amp * plane(shape, k, E_OFFSETS[2][2], 0.3)
    else:
        kk = math.hypot(*k)
        E[0] = -amp * k[1] / kk * plane(shape, k, E_OFFSETS[2][0], 0.3)
        E[1] = amp * k[0] / kk * plane(shape, k, E_OFFSETS[2][1], 0.3)
    return k, E, B


def measure_2d(cfg, E, B, k, pol, nsteps=8):
    """Run the oracle and return the measured frequency of the mode.  TM is
    read from E_z, TE from B_z: neither carries the static (w = 0) mode."""
    series = []
    for _ in range(nsteps):
        if pol == "TM":
            series.append(S.project(E[2], k, E_OFFSETS[2][2]))
        else:
            series.append(S.project(B[2], k, B_OFFSETS[2][2]))
        ref.step(cfg, E, B)
    return omega_from_series(series, cfg.dt)


def assemble_A(cfg, mask=7):
    """Dense matrix of the oracle's A over the components in `mask`."""
    shape = cfg.shape
    ncell = int(np.prod(shape))
    comps = [q for q in range(3) if mask & (1 << q)]
    N = ncell * len(comps)
    M = np.zeros((N, N))
    col = 0
    for qi, q in enumerate(comps):
        for o in range(ncell):
            x = [np.zeros(shape) for _ in range(3)]
            x[q].flat[o] = 1.0
            y = ref.apply_A(cfg, x, mask)
            M[:, col] = np.concatenate([y[p].ravel() for p in comps])
            col += 1
    return M


def div_B_2d(B):
    """Discrete div B (eq gauss_B), 2D, at nodes (i+1/2, j+1/2) of B_z's dual:
    (Bx[i+1,j] - Bx[i,j]) + (By[i,j+1] - By[i,j]) with unit cells."""
    Bx, By = B[0], B[1]
    return (np.roll(Bx, -1, axis=1) - Bx) + (np.roll(By, -1, axis=0) - By)


def div_B_3d(B):
    Bx, By, Bz = B
    return ((np.roll(Bx, -1, axis=2) - Bx) + (np.roll(By, -1, axis=1) - By)
            + (np.roll(Bz, -1, axis=0) - Bz))


def avg(f, axis):
    return (np.roll(f, 1, axis=axis) + 4 * f + np.roll(f, -1, axis=axis)) / 6.0


def gauss_E_lhs_2d(E):
    """D.(A_E E) of eq gauss_E in 2D (alpha_z = 1): A_E = diag(alpha_y, alpha_x, alpha_xy),
    evaluated at nodes (i, j): (aEx[i,j] - aEx[i-1,j]) + (aEy[i,j] - aEy[i,j-1])."""
    aEx = avg(E[0], 0)          # alpha_y on Ex (y is axis 0)
    aEy = avg(E[1], 1)          # alpha_x on Ey
    return (aEx - np.roll(aEx, 1, axis=1)) + (aEy - np.roll(aEy, 1, axis=0))


def div_node_2d(J):
    """D.J at nodes for a field placed like E."""
    return (J[0] - np.roll(J[0], 1, axis=1)) + (J[1] - np.roll(J[1], 1, axis=0))
