"""Particle coupling on the GPU (through the C-ABI) against the FP64 oracle:
one push with its charge-conserving current, coupled particle-field steps,
the charge density, FP32 against FP64, and Gauss's law on the GPU's own
output (D.(A_E E) - 4 pi F rho conserved with a converged solve)."""
import math

import numpy as np
import pytest

from oracle import ref
from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import log, to_np, torch_fields

pytestmark = pytest.mark.gpu


def _setup(shape, d, dtype, sweeps=20, tol=0.0, p=0, seed=0, nspec=2, npart=500, umax=3.0, field=0.2):
    ny, nx = shape
    dt = 0.6 / math.sqrt(1.0 / d[0] ** 2 + 1.0 / d[1] ** 2)
    np_dt = np.float32 if dtype == "f32" else np.float64
    rng = np.random.default_rng(seed)
    E = [I.round_to(np_dt, rng.normal(0, field, shape)) for _ in range(3)]
    B = [I.round_to(np_dt, rng.normal(0, field, shape)) for _ in range(3)]
    species = []
    for s in range(nspec):
        q, m = (1.0, 1.0) if s % 2 == 0 else (-1.0, 1.7)
        x = I.round_to(np_dt, rng.uniform(0, nx * d[0], npart))
        y = I.round_to(np_dt, rng.uniform(0, ny * d[1], npart))
        # boundary cases: on nodes, on the seam, just below L
        x[:3] = [0.0, d[0] * 2, float(np.nextafter(np_dt(nx * d[0]), np_dt(0)))]
        y[:3] = [d[1] * 1.5, 0.0, float(np.nextafter(np_dt(ny * d[1]), np_dt(0)))]
        u = [I.round_to(np_dt, rng.uniform(-umax, umax, npart)) for _ in range(3)]
        species.append(I.Species(q=q, m=m, w=0.05, x=x, y=y, u=u))
    cfg_o = ref.Config(ndim=2, shape=shape, dt=float(I.round_to(np_dt, dt)), d=d, sweeps=sweeps, tol=tol,
                       filter_passes=p)
    cfg_g = mx.make_config(2, (nx, ny), cfg_o.dt, d, dtype, mx.MX_ALL, sweeps, tol, p)
    return cfg_o, cfg_g, E, B, species


def _gpu_state(sp, dtype):
    return torch_fields([sp.x, sp.y], dtype), torch_fields(sp.u, dtype)


def _rel(got, want):
    scale = max(float(np.abs(w).max()) for w in want) or 1.0
    return max(float(np.abs(g - w).max()) for g, w in zip(got, want)) / scale


def _cell_order(sp, d, nx):
    o = np.argsort(np.floor(sp.y / d[1]).astype(np.int64) * nx + np.floor(sp.x / d[0]).astype(np.int64),
                   kind="stable")
    return I.Species(q=sp.q, m=sp.m, w=sp.w, x=sp.x[o].copy(), y=sp.y[o].copy(), u=[a[o].copy() for a in sp.u])


@pytest.mark.parametrize("d,ordered,npart", [((1.0, 1.0), False, 1500), ((0.9, 1.2), False, 1500),
                                             ((0.9, 1.2), True, 1500), ((0.9, 1.2), True, 60000),
                                             ((0.9, 1.2), True, 150000)])
def test_push_and_deposit_match_oracle_fp64(d, ordered, npart):
    """One push of two species on a ragged grid: positions, momenta and the
    accumulated current within 1e-12 of the oracle, with the particles in
    random order (every contribution added to J directly) and in cell order:
    at 1.4 particles per cell a workgroup's 256 particles span whole rows, so
    they still go to J directly; at 56 per cell they span a few cells and
    their contributions are summed in the LDS tile first (except where they
    straddle the periodic seam); at 140 per cell most wavefronts share one
    start cell, so many lanes add to the same LDS nodes at once."""
    import torch
    cfg_o, cfg_g, E, B, species = _setup((29, 37), d, "f64", seed=1, npart=npart)
    if ordered:
        species = [_cell_order(sp, d, 37) for sp in species]
    g = mx.Grid(cfg_g)
    Et, Bt = torch_fields(E, "f64"), torch_fields(B, "f64")
    g.bind(Et, Bt)
    Jt = [torch.full(E[0].shape, 7.0, dtype=torch.float64, device="cuda") for _ in range(3)]   # overwritten
    Jo = [np.zeros(E[0].shape) for _ in range(3)]
    states = []
    for k, sp in enumerate(species):
        pos, u = _gpu_state(sp, "f64")
        g.pic_push(sp.q, sp.m, sp.w, pos, u, Jt, accumulate=k > 0)
        states.append((pos, u))
        xo, yo, uo = sp.x.copy(), sp.y.copy(), [a.copy() for a in sp.u]
        ref.pic_push_deposit(cfg_o, E, B, sp.q, sp.m, sp.w, xo, yo, *uo, Jo)
        torch.cuda.synchronize()
        e_pos = max(float(np.abs(a - b).max()) for a, b in zip(to_np(pos), [xo, yo]))
        e_u = _rel(to_np(u), uo)
        log(f"species {k}: positions {e_pos:.2e}, momenta {e_u:.2e}")
        assert e_pos <= 1e-12 * max(E[0].shape) * max(d) and e_u <= 1e-12
    e_j = _rel(to_np(Jt), Jo)
    log(f"current {e_j:.2e}")
    assert e_j <= 1e-12
    # the bound fields are read only
    for a, b in zip(to_np(Et + Bt), E + B):
        assert np.array_equal(a, b)
    g.close()


def test_charge_density_matches_oracle():
    import torch
    cfg_o, cfg_g, E, B, species = _setup((24, 40), (0.8, 1.1), "f64", seed=2)
    g = mx.Grid(cfg_g)
    g.bind(torch_fields(E, "f64"), torch_fields(B, "f64"))
    rho = torch.zeros(E[0].shape, dtype=torch.float64, device="cuda")
    ro = np.zeros(E[0].shape)
    for k, sp in enumerate(species):
        pos, _ = _gpu_state(sp, "f64")
        g.pic_charge(sp.q, sp.w, pos, rho, accumulate=k > 0)
        ref.pic_deposit_charge(cfg_o, sp.q, sp.w, sp.x, sp.y, ro)
    torch.cuda.synchronize()
    assert _rel(to_np([rho]), [ro]) <= 1e-13
    g.close()


def _coupled(dtype, nsteps, p, tol, seed, shape=(30, 34), d=(1.0, 1.0), sweeps=20):
    """nsteps coupled steps on the GPU and in the oracle (same inputs)."""
    import torch
    cfg_o, cfg_g, E, B, species = _setup(shape, d, dtype, sweeps=sweeps, tol=tol, p=p, seed=seed)
    g = mx.Grid(cfg_g)
    Et, Bt = torch_fields(E, dtype), torch_fields(B, dtype)
    g.bind(Et, Bt)
    Jt = torch_fields([np.zeros(shape)] * 3, dtype)
    g.set_current(Jt)
    gs = [_gpu_state(sp, dtype) for sp in species]
    Eo, Bo = [a.copy() for a in E], [a.copy() for a in B]
    os_ = [(sp.x.copy(), sp.y.copy(), [a.copy() for a in sp.u]) for sp in species]
    counts = []
    for n in range(nsteps):
        for k, (sp, (pos, u)) in enumerate(zip(species, gs)):
            g.pic_push(sp.q, sp.m, sp.w, pos, u, Jt, accumulate=k > 0)
        st = g.step(1, env=[1.0], stats=True)
        counts.append(st[0].sweeps)
        Jo = [np.zeros(shape) for _ in range(3)]
        for sp, (xo, yo, uo) in zip(species, os_):
            ref.pic_push_deposit(cfg_o, Eo, Bo, sp.q, sp.m, sp.w, xo, yo, *uo, Jo)
        ref.step(cfg_o, Eo, Bo, Jo, 1.0, st[0].sweeps if tol > 0 else None)
    torch.cuda.synchronize()
    return dict(g=g, Et=Et, Bt=Bt, gs=gs, Eo=Eo, Bo=Bo, os=os_, species=species, counts=counts, cfg_o=cfg_o,
                shape=shape)


@pytest.mark.parametrize("p", [0, 2])
def test_coupled_steps_match_oracle_fp64(p):
    """Ten coupled steps (push, deposit, filtered field step at m = 20):
    fields, positions and momenta within 1e-12 of the oracle."""
    r = _coupled("f64", 10, p, 0.0, seed=3 + p)
    e_f = _rel(to_np(r["Et"] + r["Bt"]), r["Eo"] + r["Bo"])
    e_u = max(_rel(to_np(u), uo) for (pos, u), (xo, yo, uo) in zip(r["gs"], r["os"]))
    e_x = max(float(np.abs(a - b).max()) for (pos, u), (xo, yo, uo) in zip(r["gs"], r["os"])
              for a, b in zip(to_np(pos), [xo, yo]))
    log(f"coupled fp64 p={p}: fields {e_f:.2e}, momenta {e_u:.2e}, positions {e_x:.2e}")
    assert e_f <= 1e-12 and e_u <= 1e-12 and e_x <= 1e-12 * 34
    r["g"].close()


def test_coupled_steps_fp32_within_1e5():
    """The same coupled steps in FP32 (atomics in FP32) against the FP64
    oracle on the same FP32-rounded inputs."""
    r = _coupled("f32", 10, 2, 0.0, seed=7)
    e_f = _rel(to_np(r["Et"] + r["Bt"]), r["Eo"] + r["Bo"])
    e_u = max(_rel(to_np(u), uo) for (pos, u), (xo, yo, uo) in zip(r["gs"], r["os"]))
    log(f"coupled fp32: fields {e_f:.2e}, momenta {e_u:.2e}")
    assert e_f <= 1e-5 and e_u <= 1e-5
    r["g"].close()


def test_gauss_law_on_gpu_output():
    """A converged solve (tol 1e-14) with a filtered current: on the GPU's own
    fields and charge, g = D.(A_E E) - 4 pi F rho keeps its initial value to
    1e-11 over six coupled steps, with the oracle's filter applied to the
    GPU's rho (the GPU filters only the current inside the step)."""
    import torch
    shape, p = (26, 30), 1
    cfg_o, cfg_g, E, B, species = _setup(shape, (1.0, 1.0), "f64", sweeps=400, tol=1e-14, p=p, seed=9)
    g = mx.Grid(cfg_g)
    Et, Bt = torch_fields(E, "f64"), torch_fields(B, "f64")
    g.bind(Et, Bt)
    Jt = torch_fields([np.zeros(shape)] * 3, "f64")
    g.set_current(Jt)
    gs = [_gpu_state(sp, "f64") for sp in species]
    rho = torch.zeros(shape, dtype=torch.float64, device="cuda")

    def gauss():
        for k, (sp, (pos, u)) in enumerate(zip(species, gs)):
            g.pic_charge(sp.q, sp.w, pos, rho, accumulate=k > 0)
        torch.cuda.synchronize()
        Ex, Ey = to_np(Et[:2])
        aEx = (np.roll(Ex, 1, 0) + 4 * Ex + np.roll(Ex, -1, 0)) / 6.0
        aEy = (np.roll(Ey, 1, 1) + 4 * Ey + np.roll(Ey, -1, 1)) / 6.0
        div = (aEx - np.roll(aEx, 1, 1)) + (aEy - np.roll(aEy, 1, 0))
        return div - 4 * math.pi * ref.filt(cfg_o, to_np([rho])[0])

    g0 = gauss()
    for _ in range(6):
        for k, (sp, (pos, u)) in enumerate(zip(species, gs)):
            g.pic_push(sp.q, sp.m, sp.w, pos, u, Jt, accumulate=k > 0)
        st = g.step(1, env=[1.0], stats=True)
        assert not any(st[0].nonconverged)
    drift = float(np.abs(gauss() - g0).max() / np.abs(g0).max())
    log(f"Gauss law drift over 6 coupled steps: {drift:.2e}")
    assert drift <= 1e-11
    g.close()


def test_no_particles_and_argument_checks():
    """np = 0 clears J (accumulate = 0) and launches no push; a 3D grid and a
    single-block grid are refused on the host."""
    import torch
    cfg_o, cfg_g, E, B, species = _setup((16, 20), (1.0, 1.0), "f64", seed=4)
    g = mx.Grid(cfg_g)
    g.bind(torch_fields(E, "f64"), torch_fields(B, "f64"))
    J = [torch.ones((16, 20), dtype=torch.float64, device="cuda") for _ in range(3)]
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    g.pic_push(1.0, 1.0, 1.0, [empty, empty], [empty, empty, empty], J)
    torch.cuda.synchronize()
    assert all(float(t.abs().max()) == 0.0 for t in J)
    with pytest.raises(mx.MxError):
        g.pic_push(1.0, 0.0, 1.0, [empty, empty], [empty, empty, empty], J)
    g.close()
    te = mx.make_config(2, (20, 16), cfg_o.dt, (1.0, 1.0), "f64", mx.MX_TE, 20, 0.0, 0)
    g = mx.Grid(te)
    g.bind(torch_fields(E, "f64"), torch_fields(B, "f64"))
    with pytest.raises(mx.MxError):
        g.pic_push(1.0, 1.0, 1.0, [empty, empty], [empty, empty, empty], J)
    g.close()


def test_drifting_pair_plasma_reduced_fp32():
    """The benchmark's plasma (gamma 1000 drift, T = 0.01) on a 32 x 16 grid
    with 16 particles per cell and species, FP32 against the FP64 oracle
    over 8 coupled steps."""
    import torch
    shape = (16, 32)
    sps = I.drifting_pair_plasma(n=(32, 16), ppc=16, dtype="f32", seed=11)
    dt = float(I.round_to(np.float32, 0.5 / math.sqrt(2)))
    cfg_o = ref.Config(ndim=2, shape=shape, dt=dt, sweeps=20, filter_passes=3)
    g = mx.Grid(mx.make_config(2, (32, 16), dt, (1.0, 1.0), "f32", mx.MX_ALL, 20, 0.0, 3))
    Et = torch_fields([np.zeros(shape)] * 3, "f32")
    Bt = torch_fields([np.zeros(shape)] * 3, "f32")
    g.bind(Et, Bt)
    Jt = torch_fields([np.zeros(shape)] * 3, "f32")
    g.set_current(Jt)
    gs = [_gpu_state(sp, "f32") for sp in sps]
    Eo, Bo = [np.zeros(shape) for _ in range(3)], [np.zeros(shape) for _ in range(3)]
    os_ = [(sp.x.copy(), sp.y.copy(), [a.copy() for a in sp.u]) for sp in sps]
    for n in range(8):
        for k, (sp, (pos, u)) in enumerate(zip(sps, gs)):
            g.pic_push(sp.q, sp.m, sp.w, pos, u, Jt, accumulate=k > 0)
        g.step(1, env=[1.0])
        Jo = [np.zeros(shape) for _ in range(3)]
        for sp, (xo, yo, uo) in zip(sps, os_):
            ref.pic_push_deposit(cfg_o, Eo, Bo, sp.q, sp.m, sp.w, xo, yo, *uo, Jo)
        ref.step(cfg_o, Eo, Bo, Jo, 1.0)
    torch.cuda.synchronize()
    e_f = _rel(to_np(Et + Bt), Eo + Bo)
    e_u = max(_rel(to_np(u), uo) for (pos, u), (xo, yo, uo) in zip(gs, os_))
    log(f"pair plasma fp32 vs oracle: fields {e_f:.2e}, momenta {e_u:.2e}")
    assert e_f <= 1e-4 and e_u <= 1e-5
    g.close()
