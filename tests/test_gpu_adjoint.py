"""Transposed step on the GPU against the FP64 oracle's transposed step,
dot-product identities, the source-window kernels, and the differentiable
multi-step wrapper (gradients against the oracle adjoint and against
central finite differences; the objective is quadratic, so central
differences are exact up to rounding for any step)."""
import math

import numpy as np
import pytest

from oracle import ref
from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import log, torch_fields, to_np

pytestmark = pytest.mark.gpu


def _grid(ndim, shape, dt, dtype, sweeps, p, blocks=3, solver=0):
    import torch
    n = shape[::-1]
    cfg = mx.make_config(ndim, n, dt, (1.0, 1.0, 1.0)[:ndim], dtype, blocks, sweeps, 0.0, p, solver=solver)
    return mx.Grid(cfg)


@pytest.mark.parametrize("ndim,shape,solver", [(2, (80, 96), 0), (3, (12, 16, 20), 0), (2, (80, 96), 1)])
def test_adjoint_matches_oracle(ndim, shape, solver):
    """The transposed step (with the Chebyshev solve too: its result is a
    polynomial in the symmetric A applied to dE', so v = q_m(A) E-bar)."""
    rng = np.random.default_rng(60 + ndim)
    dt = 0.55 / math.sqrt(ndim)
    m, p, nsteps = 4, (2 if ndim == 2 else 1), 4
    envs = [math.sin(0.3 * (n + 0.5) * dt) for n in range(nsteps)]
    counts = [(m, m)] * nsteps
    Eb = [rng.normal(size=shape) for _ in range(3)]
    Bb = [rng.normal(size=shape) for _ in range(3)]
    cfg = ref.Config(ndim=ndim, shape=shape, dt=dt, sweeps=m, filter_passes=p, solver=solver)
    Eo, Bo, Jo = [a.copy() for a in Eb], [a.copy() for a in Bb], [np.zeros(shape) for _ in range(3)]
    for n in reversed(range(nsteps)):
        ref.adjoint_step(cfg, Eo, Bo, Jo, envs[n], counts[n])
    g = _grid(ndim, shape, dt, "f64", m, p, solver=solver)
    Et, Bt = torch_fields(Eb, "f64"), torch_fields(Bb, "f64")
    Jt = torch_fields([np.zeros(shape)] * 3, "f64")
    g.adjoint(nsteps, envs, counts, Et, Bt, Jt)
    got = to_np(Et + Bt + Jt)
    want = Eo + Bo + Jo
    scale = max(np.abs(x).max() for x in want)
    err = max(np.abs(a - b).max() for a, b in zip(got, want)) / scale
    log(f"adjoint {ndim}D solver {solver} vs oracle: {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("solver", [0, 1])
def test_adjoint_dot_product_on_gpu(solver):
    """<T x, y> = <x, T^T y> with T the GPU's multi-step map (E, B, J0) -> (E, B)."""
    import torch
    rng = np.random.default_rng(70)
    shape = (72, 88)
    dt = 0.5 / math.sqrt(2)
    m, p, nsteps = 6, 3, 5
    envs = [math.sin(0.3 * (n + 0.5) * dt) for n in range(nsteps)]
    x = [rng.normal(size=shape) for _ in range(9)]
    y = [rng.normal(size=shape) for _ in range(6)]
    g = _grid(2, shape, dt, "f64", m, p, solver=solver)
    E, B, J = torch_fields(x[:3], "f64"), torch_fields(x[3:6], "f64"), torch_fields(x[6:], "f64")
    g.bind(E, B)
    g.set_current(J)
    st = g.step(nsteps, env=envs, stats=True)
    lhs = sum(float((a.cpu().double() * torch.tensor(b)).sum()) for a, b in zip(E + B, y))
    Eb, Bb = torch_fields(y[:3], "f64"), torch_fields(y[3:], "f64")
    Jb = torch_fields([np.zeros(shape)] * 3, "f64")
    g.adjoint(nsteps, envs, [s.sweeps for s in st], Eb, Bb, Jb)
    rhs = sum(float((a.cpu() * torch.tensor(b)).sum()) for a, b in zip(Eb + Bb + Jb, x))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_source_windows_assemble_and_project():
    import torch
    n = 96
    origins, shapes, amps = I.adjoint_sources_2d(n=n, nsrc=12, sigma=3.0, seed=9, window=3.0)
    g = _grid(2, (n, n), 0.3, "f64", 0, 0)
    ot = torch.tensor(origins, dtype=torch.int64, device="cuda")
    st = torch.tensor(shapes, dtype=torch.float64, device="cuda")
    at = torch.tensor(amps, dtype=torch.float64, device="cuda")
    J = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
    g.sources_assemble(ot, st, at, J)
    want = I.assemble_sources(n, origins, shapes, amps)
    for a, b in zip(to_np(J), want):
        assert np.abs(a - b).max() < 1e-14
    rng = np.random.default_rng(3)
    G = [rng.normal(size=(n, n)) for _ in range(3)]
    grad = torch.empty(12, dtype=torch.float64, device="cuda")
    g.sources_project(ot, st, torch_fields(G, "f64"), grad)
    W = shapes.shape[-1]
    ref_grad = []
    for s in range(12):
        xs = (origins[s, 0] + np.arange(W)) % n
        ys = (origins[s, 1] + np.arange(W)) % n
        ref_grad.append(sum(np.sum(shapes[s, c] * G[c][np.ix_(ys, xs)]) for c in range(3)))
    assert np.allclose(grad.cpu().numpy(), ref_grad, rtol=1e-13, atol=1e-13)


def _probe_loss(E, win):
    return (E[2][win] ** 2).sum()


def _run_autograd(n, nsrc, nsteps, ck, dtype, seed=1005, sigma=8.0, window=4.0, win_half=32, verify=True):
    import torch
    from paper_1907_13088_amd.adjoint import SourceSet, field_steps
    w = I.modes_2d((n, n), nmodes=64, npulses=0, steps=nsteps, seed=seed, dtype=dtype)
    origins, shapes, amps = I.adjoint_sources_2d(n=n, nsrc=nsrc, sigma=sigma, seed=seed, window=window)
    td = torch.float64 if dtype == "f64" else torch.float32
    shapes = np.asarray(I.round_to(np.float32 if dtype == "f32" else np.float64, shapes))
    amps = np.asarray(I.round_to(np.float32 if dtype == "f32" else np.float64, amps))
    dt = w.dt
    env = [math.sin(0.3 * (s + 0.5) * dt) for s in range(nsteps)]
    g = _grid(2, (n, n), dt, dtype, 20, 3)
    src = SourceSet(torch.tensor(origins, device="cuda"), torch.tensor(shapes, dtype=td, device="cuda"))
    a = torch.tensor(amps, dtype=td, device="cuda", requires_grad=True)
    E0 = [torch.tensor(x, dtype=td, device="cuda", requires_grad=True) for x in w.E]
    B0 = [torch.tensor(x, dtype=td, device="cuda", requires_grad=True) for x in w.B]
    E, B = field_steps(a, E0, B0, g, src, env, nsteps, checkpoint_every=ck, verify=verify)
    c0 = n // 2 - win_half
    win = (slice(c0, c0 + 2 * win_half), slice(c0, c0 + 2 * win_half))
    L = _probe_loss(E, win)
    L.backward()
    return dict(w=w, origins=origins, shapes=shapes, amps=amps, env=env, g=g, src=src, win=win, L=float(L),
                ga=a.grad.detach().cpu().double().numpy(),
                gE=[x.grad.detach().cpu().double().numpy() for x in E0],
                gB=[x.grad.detach().cpu().double().numpy() for x in B0])


def test_autograd_matches_oracle_adjoint_and_fd_fp64():
    """Reduced problem: 128^2, 32 sources, 40 steps, checkpoint every 10."""
    import torch
    from paper_1907_13088_amd.adjoint import field_steps
    n, nsrc, nsteps = 128, 32, 40
    r = _run_autograd(n, nsrc, nsteps, 10, "f64", window=3.0, win_half=16)
    w = r["w"]
    # oracle: forward with J0 = sum a_s g_s, then the transposed steps
    J0 = I.assemble_sources(n, r["origins"], r["shapes"], r["amps"])
    cfg = ref.Config(ndim=2, shape=(n, n), dt=w.dt, sweeps=20, filter_passes=3)
    E = [x.copy() for x in w.E]
    B = [x.copy() for x in w.B]
    ref.run(cfg, E, B, nsteps, J0, r["env"])
    Eb = [np.zeros((n, n)) for _ in range(3)]
    Eb[2][r["win"]] = 2 * E[2][r["win"]]
    Bb = [np.zeros((n, n)) for _ in range(3)]
    Jb = [np.zeros((n, n)) for _ in range(3)]
    for s in reversed(range(nsteps)):
        ref.adjoint_step(cfg, Eb, Bb, Jb, r["env"][s], (20, 20))
    W = r["shapes"].shape[-1]
    ga = []
    for s in range(nsrc):
        xs = (r["origins"][s, 0] + np.arange(W)) % n
        ys = (r["origins"][s, 1] + np.arange(W)) % n
        ga.append(sum(np.sum(r["shapes"][s, c] * Jb[c][np.ix_(ys, xs)]) for c in range(3)))
    ga = np.array(ga)
    assert np.abs(r["ga"] - ga).max() <= 1e-10 * np.abs(ga).max()
    for a, b in zip(r["gE"] + r["gB"], Eb + Bb):
        assert np.abs(a - b).max() <= 1e-10 * max(np.abs(x).max() for x in Eb + Bb)
    # central finite differences on the GPU path (L is quadratic: exact up to rounding)
    rng = np.random.default_rng(4)
    td = torch.float64

    def L_of(amps, E0, B0):
        Ev, _ = field_steps(torch.tensor(amps, dtype=td, device="cuda"),
                            [torch.tensor(x, dtype=td, device="cuda") for x in E0],
                            [torch.tensor(x, dtype=td, device="cuda") for x in B0],
                            r["g"], r["src"], r["env"], nsteps, checkpoint_every=10, verify=False)
        return float(_probe_loss(Ev, r["win"]))

    h = 1e-2
    for s in rng.choice(nsrc, 4, replace=False):
        ap, am = r["amps"].copy(), r["amps"].copy()
        ap[s] += h
        am[s] -= h
        fd = (L_of(ap, w.E, w.B) - L_of(am, w.E, w.B)) / (2 * h)
        assert fd == pytest.approx(r["ga"][s], rel=1e-7, abs=1e-9 * abs(r["L"]))
    # a random direction in the initial fields
    dE = [rng.normal(size=(n, n)) for _ in range(3)]
    Ep = [a + h * d for a, d in zip(w.E, dE)]
    Em = [a - h * d for a, d in zip(w.E, dE)]
    fd = (L_of(r["amps"], Ep, w.B) - L_of(r["amps"], Em, w.B)) / (2 * h)
    dir_grad = sum(np.sum(a * d) for a, d in zip(r["gE"], dE))
    assert fd == pytest.approx(dir_grad, rel=1e-7)


def test_autograd_full_size_fp32():
    """2048^2, 256 sources with learnable amplitudes, 500 steps, checkpoint every
    50, objective sum of E_z^2 over a 64 x 64 window: the FP32 gradient agrees
    with the FP64 GPU gradient (pinned to the oracle adjoint above) within
    1e-4 relative, and FP64 central differences confirm the FP64 gradient."""
    import torch
    n, nsrc, nsteps = 2048, 256, 500
    log("full-size adjoint fp32")
    r32 = _run_autograd(n, nsrc, nsteps, 50, "f32")
    log("full-size adjoint fp64")
    r64 = _run_autograd(n, nsrc, nsteps, 50, "f64")
    ga32, ga64 = r32["ga"], r64["ga"]
    rel = np.linalg.norm(ga32 - ga64) / np.linalg.norm(ga64)
    log(f"amplitude gradient fp32 vs fp64: {rel:.2e}")
    assert rel < 1e-4
    for a, b in zip(r32["gE"], r64["gE"]):
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-30
    from paper_1907_13088_amd.adjoint import field_steps
    td = torch.float64
    w = r64["w"]

    def L_of(amps):
        Ev, _ = field_steps(torch.tensor(amps, dtype=td, device="cuda"),
                            [torch.tensor(x, dtype=td, device="cuda") for x in w.E],
                            [torch.tensor(x, dtype=td, device="cuda") for x in w.B],
                            r64["g"], r64["src"], r64["env"], nsteps, checkpoint_every=50, verify=False)
        return float(_probe_loss(Ev, r64["win"]))

    order = np.argsort(-np.abs(ga64))[:3]
    h = 1e-2
    for s in order:
        ap, am = r64["amps"].copy(), r64["amps"].copy()
        ap[s] += h
        am[s] -= h
        fd = (L_of(ap) - L_of(am)) / (2 * h)
        log(f"source {s}: fd {fd:.10e} adjoint {ga64[s]:.10e}")
        assert fd == pytest.approx(ga64[s], rel=1e-6)
