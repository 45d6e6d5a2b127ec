"""Per-wavevector (Fourier) analysis of the scheme, FP64 numpy.

TEST INFRASTRUCTURE ONLY.  Each field component is expanded in its own
staggered Fourier basis, f_c(x) = Re(a_c exp(i k . x_c)), in which the
operators of the paper become small matrices (Sec. 2 Fourier symbols,
Appendix C):

  alpha_i  -> 1 - (2/3) sin^2(k_i d_i / 2)                 (eq alphax)
  D_i      -> i [k]_i,  [k]_i = sin(k_i d_i / 2) / (d_i / 2)  (eq braket_k)
  Dbar_i   -> 2 i sin(k_i d_i / 2)                          (Appendix C)

so both discrete curls are i [k] x, Lambda = diag(alpha_x, alpha_y, alpha_z)
and A (eqs matrixA_*) is a real symmetric 3x3 matrix per k.  One vacuum
step maps (E^n, B^{n-1/2}) to (E^{n+1}, B^{n+1/2}) by

  T(k) = [[I + t^2 P X Lambda X,  i t P X Lambda],
          [-i t X,                I             ]],

X the cross-product matrix of [k], P = sum_{j<=m} A^j (Alg 1), or (1-A)^-1
for the exact solve.  With the averaging operators lumped, A = 0, Lambda = I
and T is the Yee step.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np


def _k3(k: Sequence[float]):
    k = list(k) + [0.0] * (3 - len(k))
    return np.array(k, dtype=np.float64)


def _d3(d: Sequence[float]):
    d = list(d) + [1.0] * (3 - len(d))
    return np.array(d, dtype=np.float64)


def alpha_hat(k, d):
    """Fourier symbol of the (1,4,1)/6 average along each axis (eq alphax)."""
    k, d = _k3(k), _d3(d)
    return 1.0 - (2.0 / 3.0) * np.sin(k * d / 2) ** 2


def bracket_k(k, d):
    """[k]_i = sin(k_i d_i / 2) / (d_i / 2) (eq braket_k)."""
    k, d = _k3(k), _d3(d)
    return np.sin(k * d / 2) / (d / 2)


def cross_matrix(v):
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def A_hat(k, d, dt):
    """Symbol of A: eqs matrixA_1st..matrixA_last with Dbar_ii -> -4 s_i^2,
    Dbar_i Dbar_j -> -4 s_i s_j and (1 + Dbar_ii/6) -> alpha_i (Appendix C)."""
    k, d = _k3(k), _d3(d)
    s = np.sin(k * d / 2)
    Dii = -4.0 * s * s
    al = 1.0 + Dii / 6.0
    r = dt * dt / (d * d)
    A = np.zeros((3, 3))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        A[a, a] = (r[b] - 1) / 6 * Dii[b] + (r[c] - 1) / 6 * Dii[c] + (r[b] + r[c] - 1) / 36 * Dii[b] * Dii[c]
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            c = 3 - a - b
            A[a, b] = -(dt * dt) / (6 * d[a] * d[b]) * (-4.0 * s[a] * s[b]) * al[c]
    return A


def P_hat(A, m: Optional[int]):
    """sum_{j=0}^{m} A^j, or (1 - A)^-1 when m is None (exact solve)."""
    if m is None:
        return np.linalg.inv(np.eye(A.shape[0]) - A)
    P = np.eye(A.shape[0])
    Aj = np.eye(A.shape[0])
    for _ in range(m):
        Aj = Aj @ A
        P = P + Aj
    return P


def step_matrix(k, d, dt, m: Optional[int] = None, lumped: bool = False):
    """T(k) (6x6 complex) on (E_x, E_y, E_z, B_x, B_y, B_z) amplitudes."""
    X = cross_matrix(bracket_k(k, d))
    if lumped:
        Lam = np.eye(3)
        P = np.eye(3)
    else:
        Lam = np.diag(alpha_hat(k, d))
        P = P_hat(A_hat(k, d, dt), m)
    T = np.zeros((6, 6), dtype=np.complex128)
    T[:3, :3] = np.eye(3) + dt * dt * P @ X @ Lam @ X
    T[:3, 3:] = 1j * dt * P @ X @ Lam
    T[3:, :3] = -1j * dt * X
    T[3:, 3:] = np.eye(3)
    return T


def omega_numeric(k, d, dt, m: Optional[int] = None, lumped: bool = False):
    """Frequencies |arg lambda| / dt of the propagating eigenvalues of T(k),
    sorted (the unit eigenvalues of static longitudinal fields dropped)."""
    ev = np.linalg.eigvals(step_matrix(k, d, dt, m, lumped))
    w = np.sort(np.abs(np.angle(ev)) / dt)
    return w[w > 1e-12 * max(1.0, w.max())]


def G(theta):
    """G(theta) = sin^2 theta / (1 - (2/3) sin^2 theta) (eq G)."""
    s2 = np.sin(theta) ** 2
    return s2 / (1.0 - (2.0 / 3.0) * s2)


def omega_exact(k, d, dt):
    """Converged-solve vacuum dispersion (eqs dispersion-em-F-2d/3d):
    G(w dt/2)/dt^2 = sum_i G(k_i d_i/2)/d_i^2 (c = 1), solved for w."""
    k, d = _k3(k), _d3(d)
    rhs = float(np.sum(G(k * d / 2) / (d * d))) * dt * dt   # = G(w dt / 2)
    # invert G: s2 = g / (1 + 2 g / 3)
    s2 = rhs / (1.0 + 2.0 * rhs / 3.0)
    return 2.0 * math.asin(math.sqrt(s2)) / dt


def omega_yee(k, d, dt):
    """Textbook Yee dispersion: sin^2(w dt/2)/dt^2 = sum_i sin^2(k_i d_i/2)/d_i^2."""
    k, d = _k3(k), _d3(d)
    s2 = float(np.sum(np.sin(k * d / 2) ** 2 / (d * d))) * dt * dt
    return 2.0 * math.asin(math.sqrt(s2)) / dt


def omega_tm_closed(k, d, dt, m: Optional[int]):
    """2D TM branch after m sweeps: sin^2(w dt/2) = (t^2/4)(alpha_y [k]_x^2 +
    alpha_x [k]_y^2) p, with p = (1 - a^{m+1})/(1 - a), a = A_zz(k)."""
    al = alpha_hat(k, d)
    bk = bracket_k(k, d)
    a = A_hat(k, d, dt)[2, 2]
    p = 1.0 / (1.0 - a) if m is None else (1.0 - a ** (m + 1)) / (1.0 - a)
    s2 = dt * dt / 4.0 * (al[1] * bk[0] ** 2 + al[0] * bk[1] ** 2) * p
    return 2.0 * math.asin(math.sqrt(s2)) / dt


def phase_speed_small_k(k, d, dt):
    """Second-order small-k phase speed (eqs phase-speed-3d/2d), c = 1."""
    k, d = _k3(k), _d3(d)
    kk2 = float(np.sum(k * k))
    return 1.0 + (float(np.sum(k ** 4 * d * d)) / kk2 - kk2 * dt * dt) / 24.0


def lattice_k(n_idx: Sequence[int], N: Sequence[int], d: Sequence[float] = (1.0, 1.0, 1.0)):
    return [2 * math.pi * n_idx[a] / (N[a] * d[a]) for a in range(len(N))]


def project(field: np.ndarray, k, offset, d=(1.0, 1.0, 1.0)) -> complex:
    """Complex amplitude a with field ~ Re(a exp(i k.(x + offset))) on a
    periodic grid: (2/N) sum field * exp(-i k.(x+offset)) (k not 0 or
    Nyquist on every axis)."""
    nd = field.ndim
    ph = np.zeros(field.shape)
    for ax in range(nd):
        n = field.shape[nd - 1 - ax]
        x = (np.arange(n) + offset[ax]) * d[ax]
        shp = [1] * nd
        shp[nd - 1 - ax] = n
        ph = ph + (k[ax] * x).reshape(shp)
    return complex(2.0 * np.sum(field * np.exp(-1j * ph)) / field.size)
