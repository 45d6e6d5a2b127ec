"""Seeded synthetic workloads for the finite-element Maxwell field step.

This module only *draws* inputs: initial fields, prescribed current shapes,
source envelopes and time steps.  It holds none of the step's arithmetic
(no Faraday or Ampere update, no averaging operator, no mass-matrix sweep,
no filter), so both the HIP path and the FP64 oracle can take their inputs
from here without sharing any of the method's code.  Two input properties
are built in from the grid alone: mode polarisations use the discrete
wavenumber [k]_i = 2 sin(k_i d_i / 2) / d_i, and the current is the exact
difference of a sampled potential, so that the initial fields and the
current are divergence-free on the staggered grid (Appendix A).

Conventions
-----------
* Light speed c = 1; cell sizes default to 1.
* Arrays are numpy float64, shaped ``(ny, nx)`` in 2D and ``(nz, ny, nx)`` in
  3D, so that x is the fastest (contiguous) index.
* Component positions follow the paper's staggered variable list (Sec. 2):
  E_x at (i+1/2, j, k), E_y at (i, j+1/2, k), E_z at (i, j, k+1/2);
  B_x at (i, j+1/2, k+1/2), B_y at (i+1/2, j, k+1/2), B_z at (i+1/2, j+1/2, k);
  J is placed like E.  In 2D the z offsets are dropped.
* "Courant C" is read as dt = C * dt_CFL, with dt_CFL the Yee-type stability
  limit the paper derives for this scheme (Sec. 2.1, CFL equations).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

E_OFFSETS = {
    3: ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5)),
    2: ((0.5, 0.0), (0.0, 0.5), (0.0, 0.0)),
}
B_OFFSETS = {
    3: ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)),
    2: ((0.0, 0.5), (0.5, 0.0), (0.5, 0.5)),
}

FOUR_PI = 4.0 * math.pi


def cfl_dt(d: Sequence[float]) -> float:
    """Largest stable time step (c = 1): (sum 1/d_i^2)^(-1/2) (Sec. 2.1)."""
    return 1.0 / math.sqrt(sum(1.0 / (x * x) for x in d))


def courant_dt(courant: float, d: Sequence[float]) -> float:
    return courant * cfl_dt(d)


def round_to(dtype, x):
    """Round a scalar or array to the run dtype, returned as float64."""
    if np.isscalar(x):
        return float(np.asarray(x, dtype=dtype))
    return np.asarray(x, dtype=dtype).astype(np.float64)


def _coords(shape: Tuple[int, ...], offset: Sequence[float]):
    """Per-axis coordinate vectors (x, y[, z]) of a staggered component."""
    nd = len(shape)
    out = []
    for ax in range(nd):  # ax 0 = x
        n = shape[nd - 1 - ax]
        out.append(np.arange(n, dtype=np.float64) + offset[ax])
    return out


# --------------------------------------------------------------------------
# Fourier-mode fields
# --------------------------------------------------------------------------

@dataclass
class Mode:
    n: Tuple[int, ...]   # integer lattice wavevector (n_x, n_y[, n_z])
    amp: float
    phase: float


def mode_sum(shape: Tuple[int, ...], modes: Sequence[Mode], offset: Sequence[float],
             weights: Optional[Sequence[float]] = None) -> np.ndarray:
    """sum_s w_s a_s cos(2 pi n_s . (x + offset) / N + phi_s) on the grid.

    Evaluated with one inverse FFT (all n_s lie on the periodic lattice)."""
    nd = len(shape)
    N = shape[::-1]  # (nx, ny[, nz])
    spec = np.zeros(shape, dtype=np.complex128)
    for s, md in enumerate(modes):
        w = 1.0 if weights is None else weights[s]
        if w == 0.0 or md.amp == 0.0:
            continue
        ph = md.phase + 2.0 * math.pi * sum(md.n[a] * offset[a] / N[a] for a in range(nd))
        idx = tuple(md.n[a] % N[a] for a in reversed(range(nd)))
        spec[idx] += w * md.amp * complex(math.cos(ph), math.sin(ph))
    total = 1
    for x in shape:
        total *= x
    return np.real(np.fft.ifftn(spec)) * total


def draw_modes(rng: np.random.Generator, N: Sequence[int], count: int, kmax: float) -> List[Mode]:
    """`count` distinct lattice wavevectors with 0 < |k| <= kmax (k = 2 pi n / N)."""
    nd = len(N)
    lim = [int(math.floor(kmax * N[a] / (2 * math.pi))) for a in range(nd)]
    ncand = 1
    for a in range(nd):
        ncand *= 2 * lim[a] + 1
    if ncand <= 64 * max(count, 1):
        # small lattice: enumerate the admissible wavevectors (one of each
        # mirror pair) and draw without replacement; fewer than `count` may exist
        cand = []
        for n in np.ndindex(*[2 * lim[a] + 1 for a in range(nd)]):
            v = tuple(int(n[a]) - lim[a] for a in range(nd))
            k2 = sum((2 * math.pi * v[a] / N[a]) ** 2 for a in range(nd))
            if k2 == 0.0 or k2 > kmax * kmax or tuple(-x for x in v) in cand:
                continue
            cand.append(v)
        pick = rng.permutation(len(cand))[:count]
        return [Mode(n=cand[j], amp=float(rng.normal()), phase=float(rng.uniform(0, 2 * math.pi))) for j in pick]
    seen = set()
    out: List[Mode] = []
    while len(out) < count:
        n = tuple(int(rng.integers(-lim[a], lim[a] + 1)) for a in range(nd))
        k2 = sum((2 * math.pi * n[a] / N[a]) ** 2 for a in range(nd))
        if k2 == 0.0 or k2 > kmax * kmax or n in seen:
            continue
        # a mode and its mirror image would alias onto one real field
        mirror = tuple(-x for x in n)
        if mirror in seen:
            continue
        seen.add(n)
        out.append(Mode(n=n, amp=float(rng.normal()), phase=float(rng.uniform(0, 2 * math.pi))))
    return out


def _kbracket(n_int: int, N: int, d: float = 1.0) -> float:
    """Discrete wavenumber [k] = 2 sin(k d / 2) / d of lattice mode n on N cells:
    a centred difference across one cell multiplies e^{ikx} by i [k]."""
    return 2.0 * math.sin(math.pi * n_int / N) / d


def em_wave_fields(shape: Tuple[int, ...], te_modes: Sequence[Mode], tm_modes: Sequence[Mode]):
    """Discretely transverse 2D plane waves: TE modes set (E_x, E_y, B_z) with
    E = a (-[k]_y, [k]_x)/|[k]|, B_z = a; TM modes set (E_z, B_x, B_y) with
    E_z = a, B = a ([k]_y, -[k]_x)/|[k]|.  With the discrete wavenumber the
    staggered divergences of E and B vanish for every mode (up to rounding),
    not only in the continuum limit.  Returns (E[3], B[3])."""
    assert len(shape) == 2
    ny, nx = shape
    def unit(md):
        kx, ky = _kbracket(md.n[0], nx), _kbracket(md.n[1], ny)
        kk = math.hypot(kx, ky)
        return kx / kk, ky / kk
    te_u = [unit(m) for m in te_modes]
    tm_u = [unit(m) for m in tm_modes]
    eo, bo = E_OFFSETS[2], B_OFFSETS[2]
    E = [mode_sum(shape, te_modes, eo[0], [-u[1] for u in te_u]),
         mode_sum(shape, te_modes, eo[1], [u[0] for u in te_u]),
         mode_sum(shape, tm_modes, eo[2])]
    B = [mode_sum(shape, tm_modes, bo[0], [u[1] for u in tm_u]),
         mode_sum(shape, tm_modes, bo[1], [-u[0] for u in tm_u]),
         mode_sum(shape, te_modes, bo[2])]
    return E, B


# --------------------------------------------------------------------------
# Prescribed currents: Gaussian pulses, divergence-free on the staggered grid
# --------------------------------------------------------------------------

@dataclass
class Pulse:
    centre: Tuple[float, ...]
    sigma: float
    phi: float                     # 2D polarisation angle
    pol: Tuple[float, float, float] = (0.0, 0.0, 1.0)  # 3D unit vector
    amp: float = 1.0


def _min_image(x: np.ndarray, c: float, n: int) -> np.ndarray:
    d = x - c
    return d - n * np.round(d / n)


def pulse_current(shape: Tuple[int, ...], pulses: Sequence[Pulse], scale: float = 1.0 / FOUR_PI,
                  window: float = 6.0):
    """J0 = sum of pulses (three components, positioned like E), divergence-free
    on the staggered grid.

    Each pulse has a potential psi sampled at the B positions (one cell
    corner per pair of axes): 2D psi = cos(phi) sigma g at B_z, and
    J_x = psi(i+1/2, j+1/2) - psi(i+1/2, j-1/2), J_y = -(psi(i+1/2, j+1/2) -
    psi(i-1/2, j+1/2)), J_z = sin(phi) g at E_z; 3D psi = p sigma g with
    psi_x, psi_y, psi_z at B_x, B_y, B_z and J = the difference-curl of psi,
    e.g. J_x = (psi_z(j+1/2) - psi_z(j-1/2)) - (psi_y(k+1/2) - psi_y(k-1/2)).
    The staggered divergence of J then telescopes to zero at every node
    (each psi sample enters it twice with opposite signs), so the charge
    density the current transports stays constant (Appendix A).
    g = exp(-|x - c|^2 / 2 sigma^2) with periodic minimum image; each pulse's
    potential is evaluated in a window of +-window*sigma cells."""
    nd = len(shape)
    N = shape[::-1]
    bo = B_OFFSETS[nd]

    def sampled(offset, weight_of):
        """sum over pulses of weight_of(pulse) * amp * sigma-scaled g at one
        staggered position (offset per axis), on the whole grid"""
        out = np.zeros(shape)
        for p in pulses:
            w = weight_of(p)
            if w == 0.0:
                continue
            s = p.sigma
            h = int(math.ceil(window * s))
            idx, dist = [], []
            for ax in range(nd):
                c = p.centre[ax]
                base = int(math.floor(c - offset[ax]))
                ii = np.arange(base - h, base + h + 2) if 2 * h + 2 < N[ax] else np.arange(N[ax])
                dist.append(_min_image(ii + offset[ax], c, N[ax]))
                idx.append(np.mod(ii, N[ax]))
            if nd == 2:
                dx, dy = np.meshgrid(dist[0], dist[1], indexing="xy")  # (ny, nx)
                g = np.exp(-(dx * dx + dy * dy) / (2 * s * s))
                np.add.at(out, np.ix_(idx[1], idx[0]), w * p.amp * scale * g)
            else:
                dz, dy, dx = np.meshgrid(dist[2], dist[1], dist[0], indexing="ij")
                g = np.exp(-(dx * dx + dy * dy + dz * dz) / (2 * s * s))
                np.add.at(out, np.ix_(idx[2], idx[1], idx[0]), w * p.amp * scale * g)
        return out

    def back(f, ax):
        """f(x) - f(x - e_ax) along grid axis ax (0 = x), periodic"""
        return f - np.roll(f, 1, axis=nd - 1 - ax)

    if nd == 2:
        psi = sampled(bo[2], lambda p: math.cos(p.phi) * p.sigma)
        return [back(psi, 1), -back(psi, 0), sampled(E_OFFSETS[2][2], lambda p: math.sin(p.phi))]
    psi = [sampled(bo[q], lambda p, q=q: p.pol[q] * p.sigma) for q in range(3)]
    return [back(psi[2], 1) - back(psi[1], 2),
            back(psi[0], 2) - back(psi[2], 0),
            back(psi[1], 0) - back(psi[0], 1)]


def draw_pulses(rng: np.random.Generator, N: Sequence[int], count: int, sigma: float = 8.0) -> List[Pulse]:
    nd = len(N)
    out = []
    for _ in range(count):
        c = tuple(float(rng.uniform(0, N[a])) for a in range(nd))
        phi = float(rng.uniform(0, 2 * math.pi))
        v = rng.normal(size=3)
        v = v / np.linalg.norm(v)
        out.append(Pulse(centre=c, sigma=sigma, phi=phi, pol=(float(v[0]), float(v[1]), float(v[2]))))
    return out


def envelope(nsteps: int, dt: float, omega: float = 0.3, start: int = 0) -> np.ndarray:
    """env_n = sin(omega (n + 1/2) dt): the current acts at half steps."""
    n = np.arange(start, start + nsteps, dtype=np.float64)
    return np.sin(omega * (n + 0.5) * dt)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ndim: int
    shape: Tuple[int, ...]          # (ny, nx) or (nz, ny, nx)
    d: Tuple[float, ...]
    dt: float
    dtype: str                      # "f32" | "f64"
    blocks: int                     # bit0 TE, bit1 TM (2D); 3 in 3D
    sweeps: int                     # m, or m_max when tol > 0
    tol: float
    filter_passes: int
    steps: int
    E: List[np.ndarray]
    B: List[np.ndarray]
    J0: Optional[List[np.ndarray]]
    env: Optional[np.ndarray]
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        c = 1
        for x in self.shape:
            c *= x
        return c


def _finish(w: Workload) -> Workload:
    """Round every input to the run dtype (both sides see identical values)."""
    np_dt = np.float32 if w.dtype == "f32" else np.float64
    w.dt = round_to(np_dt, w.dt)
    w.E = [round_to(np_dt, a) for a in w.E]
    w.B = [round_to(np_dt, a) for a in w.B]
    if w.J0 is not None:
        w.J0 = [round_to(np_dt, a) for a in w.J0]
    return w


def planewave_te_2d(n: int = 128, courant: float = 0.5, kidx: int = 4, noise: float = 1e-6,
                    seed: int = 1001, steps: int = 200, tol: float = 1e-12, m_max: int = 200,
                    dtype: str = "f64") -> Workload:
    """2D TE plane wave along x (E_y, B_z) plus N(0, noise) on E_x, E_y, B_z."""
    rng = np.random.default_rng(seed)
    shape = (n, n)
    md = [Mode(n=(kidx, 0), amp=1.0, phase=0.0)]
    E = [np.zeros(shape), mode_sum(shape, md, E_OFFSETS[2][1]), np.zeros(shape)]
    B = [np.zeros(shape), np.zeros(shape), mode_sum(shape, md, B_OFFSETS[2][2])]
    for a in (E[0], E[1], B[2]):
        a += rng.normal(0.0, noise, shape)
    return _finish(Workload("te_planewave_2d", 2, shape, (1.0, 1.0), courant_dt(courant, (1, 1)), dtype,
                            1, m_max, tol, 0, steps, E, B, None, None, {"seed": seed, "courant": courant}))


def modes_2d(n: Tuple[int, int] = (4096, 4096), courant: float = 0.5, nmodes: int = 256,
             npulses: int = 64, sigma: float = 8.0, filter_passes: int = 3, m: int = 20,
             steps: int = 1000, seed: int = 1002, dtype: str = "f32", kmax: float = math.pi / 2,
             omega: float = 0.3) -> Workload:
    """2D TE+TM: nmodes random plane waves (|k| <= kmax, N(0,1) amplitudes, TE or
    TM with probability 1/2) and npulses Gaussian current pulses."""
    rng = np.random.default_rng(seed)
    ny, nx = n[1], n[0]
    shape = (ny, nx)
    modes = draw_modes(rng, (nx, ny), nmodes, kmax)
    is_te = rng.uniform(size=nmodes) < 0.5
    te = [md for md, t in zip(modes, is_te) if t]
    tm = [md for md, t in zip(modes, is_te) if not t]
    E, B = em_wave_fields(shape, te, tm)
    J0 = None
    env = None
    dt = courant_dt(courant, (1, 1))
    if npulses > 0:
        J0 = pulse_current(shape, draw_pulses(rng, (nx, ny), npulses, sigma))
        env = envelope(steps, round_to(np.float32 if dtype == "f32" else np.float64, dt), omega)
    return _finish(Workload("modes_2d", 2, shape, (1.0, 1.0), dt, dtype, 3, m, 0.0,
                            filter_passes if npulses > 0 else 0, steps, E, B, J0, env,
                            {"seed": seed, "courant": courant, "nmodes": nmodes, "npulses": npulses,
                             "modes": [{"n": md.n, "amp": md.amp, "phase": md.phase, "pol": "TE" if t else "TM"}
                                       for md, t in zip(modes, is_te)]}))


def planewave_3d(n: int = 512, courant: float = 0.4, kidx: int = 16, noise: float = 1e-3,
                 npulses: int = 32, sigma: float = 8.0, filter_passes: int = 1, tol: float = 1e-7,
                 m_max: int = 300, steps: int = 200, seed: int = 1003, dtype: str = "f32",
                 omega: float = 0.3) -> Workload:
    """3D plane wave along x (E_y, B_z) plus N(0, noise) on all six components,
    and npulses solenoidal Gaussian current pulses."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    k = 2 * math.pi * kidx / n
    x_ey = np.arange(n) + E_OFFSETS[3][1][0]
    x_bz = np.arange(n) + B_OFFSETS[3][2][0]
    E = [np.zeros(shape), np.broadcast_to(np.cos(k * x_ey), shape).copy(), np.zeros(shape)]
    B = [np.zeros(shape), np.zeros(shape), np.broadcast_to(np.cos(k * x_bz), shape).copy()]
    for a in E + B:
        a += rng.normal(0.0, noise, shape)
    dt = courant_dt(courant, (1, 1, 1))
    J0 = pulse_current(shape, draw_pulses(rng, (n, n, n), npulses, sigma)) if npulses > 0 else None
    env = envelope(steps, round_to(np.float32 if dtype == "f32" else np.float64, dt), omega) if npulses > 0 else None
    return _finish(Workload("planewave_3d", 3, shape, (1.0, 1.0, 1.0), dt, dtype, 3, m_max, tol,
                            filter_passes if npulses > 0 else 0, steps, E, B, J0, env,
                            {"seed": seed, "courant": courant}))


def batch_2d(ngrids: int = 64, sizes: Sequence[int] = (256, 512, 1024, 2048), courant=(0.3, 0.7),
             nmodes: int = 16, m: int = 20, steps: int = 500, seed: int = 1004, dtype: str = "f32",
             kmax: float = math.pi / 2) -> List[Workload]:
    """Independent periodic 2D grids of uneven size and Courant number, no current."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(ngrids):
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        c = float(rng.uniform(*courant))
        sub = int(rng.integers(0, 2**31 - 1))
        w = modes_2d((nx, ny), courant=c, nmodes=nmodes, npulses=0, m=m, steps=steps, seed=sub,
                     dtype=dtype, kmax=kmax)
        w.name = f"batch_{g}"
        w.meta["batch_seed"] = seed
        out.append(w)
    return out


def adjoint_sources_2d(n: int = 2048, nsrc: int = 256, sigma: float = 8.0, seed: int = 1005,
                       window: float = 4.0):
    """Per-source current shapes g_s (the cfg2 polarisation recipe, unit
    amplitude) stored as local windows: returns (origins[s, 2] as (x0, y0),
    shapes[s, 3, W, W]) where window cell (a, b) sits at grid cell
    ((x0 + b) mod n, (y0 + a) mod n), plus amplitudes a_s ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    pulses = draw_pulses(rng, (n, n), nsrc, sigma)
    amps = rng.normal(size=nsrc)
    h = int(math.ceil(window * sigma))
    W = 2 * h + 2
    origins = np.zeros((nsrc, 2), dtype=np.int64)
    shapes = np.zeros((nsrc, 3, W, W))
    for s, p in enumerate(pulses):
        x0 = int(math.floor(p.centre[0])) - h
        y0 = int(math.floor(p.centre[1])) - h
        origins[s] = (x0 % n, y0 % n)
        # evaluate this pulse on a small periodic patch large enough for the window
        sub = pulse_current((W, W), [Pulse(centre=(p.centre[0] - x0, p.centre[1] - y0), sigma=sigma,
                                           phi=p.phi)], window=window)
        for c in range(3):
            shapes[s, c] = sub[c]
    return origins, shapes, amps


def assemble_sources(n: int, origins, shapes, amps) -> List[np.ndarray]:
    """J0 = sum_s a_s g_s on an n x n periodic grid (host-side, float64)."""
    J = [np.zeros((n, n)) for _ in range(3)]
    W = shapes.shape[-1]
    for s in range(shapes.shape[0]):
        xs = (origins[s, 0] + np.arange(W)) % n
        ys = (origins[s, 1] + np.arange(W)) % n
        for c in range(3):
            np.add.at(J[c], np.ix_(ys, xs), amps[s] * shapes[s, c])
    return J


# --------------------------------------------------------------------------
# Particles for the coupled step: a drifting pair plasma
# --------------------------------------------------------------------------

@dataclass
class Species:
    q: float
    m: float
    w: float                     # macro-particle weight (charge q w)
    x: np.ndarray
    y: np.ndarray
    u: List[np.ndarray]          # gamma v, three components


def drifting_pair_plasma(n: Tuple[int, int] = (256, 128), ppc: int = 256, gamma: float = 1000.0,
                         temperature: float = 0.01, skin_depth: float = 16.0, seed: int = 1006,
                         dtype: str = "f32") -> List[Species]:
    """Electrons and positrons (q = -1, +1, m = 1, c = 1) drifting along +x,
    the shape of the paper's NCI test problem (Table 1: 256 x 128 cells, 256
    particles per cell and species, drift Lorentz factor 1000, temperature
    0.01 m c^2, domain 16 x 8 skin depths, so 16 cells per skin depth).
    Positions are uniform over the periodic domain (unit cells).  Momenta:
    a Maxwellian of temperature T in the rest frame (u_i ~ N(0, T/m) per
    axis, gamma from |u|), boosted along x with the drift Lorentz factor
    (u_x' = gamma_d (u_x + beta_d gamma), u_y, u_z unchanged); a synthetic
    stand-in for the relativistic shifted-Maxwellian loader the paper uses.
    The weight makes the skin depth c / omega_p with
    omega_p^2 = 4 pi q^2 n / (gamma m) equal `skin_depth` cells:
    n = gamma / (4 pi skin_depth^2) per species and cell."""
    rng = np.random.default_rng(seed)
    nx, ny = n
    npart = nx * ny * ppc
    np_dt = np.float32 if dtype == "f32" else np.float64
    dens = gamma / (FOUR_PI * skin_depth * skin_depth)
    beta = math.sqrt(1.0 - 1.0 / (gamma * gamma))
    out = []
    for q in (-1.0, 1.0):
        x = rng.uniform(0.0, nx, npart)
        y = rng.uniform(0.0, ny, npart)
        th = math.sqrt(temperature)
        u0 = [rng.normal(0.0, th, npart) for _ in range(3)]
        g0 = np.sqrt(1.0 + u0[0] ** 2 + u0[1] ** 2 + u0[2] ** 2)
        ux = gamma * (u0[0] + beta * g0)
        # positions strictly inside [0, L) after rounding to the run dtype
        x = np.minimum(round_to(np_dt, x), np.nextafter(np.asarray(nx, np_dt), np_dt(0)).astype(np.float64))
        y = np.minimum(round_to(np_dt, y), np.nextafter(np.asarray(ny, np_dt), np_dt(0)).astype(np.float64))
        # particles in cell order (row-major), as particle codes keep them
        order = np.argsort(np.floor(y).astype(np.int64) * nx + np.floor(x).astype(np.int64), kind="stable")
        u = [ux, u0[1], u0[2]]
        out.append(Species(q=q, m=1.0, w=float(round_to(np_dt, dens / ppc)), x=x[order], y=y[order],
                           u=[round_to(np_dt, c[order]) for c in u]))
    return out
