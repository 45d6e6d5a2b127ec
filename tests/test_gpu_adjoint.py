"""Transposed step on the GPU against the FP64 oracle's transposed step,
dot-product identities, the source-window kernels, and the differentiable
multi-step wrapper (gradients against the oracle adjoint and against
central finite differences; the objective is quadratic, so central
differences are exact up to rounding for any step)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ref
from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import log, torch_fields, to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_2048_grad.json")


def _grid(ndim, shape, dt, dtype, sweeps, p, blocks=3, solver=0):
    import torch
    n = shape[::-1]
    cfg = mx.make_config(ndim, n, dt, (1.0, 1.0, 1.0)[:ndim], dtype, blocks, sweeps, 0.0, p, solver=solver)
    return mx.Grid(cfg)


@pytest.mark.parametrize("ndim,shape,solver", [(2, (80, 96), 0), (3, (12, 16, 20), 0), (2, (80, 96), 1),
                                                (3, (12, 16, 20), 1)])
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


@pytest.mark.parametrize("ndim,solver", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_adjoint_dot_product_on_gpu(ndim, solver):
    """<T x, y> = <x, T^T y> with T the GPU's multi-step map (E, B, J0) -> (E, B)
    (3D on cubic cells, where the Chebyshev solve is defined)."""
    import torch
    rng = np.random.default_rng(70 + ndim)
    shape = (72, 88) if ndim == 2 else (14, 18, 22)
    dt = 0.5 / math.sqrt(ndim)
    m, p, nsteps = 6, (3 if ndim == 2 else 1), 5
    envs = [math.sin(0.3 * (n + 0.5) * dt) for n in range(nsteps)]
    x = [rng.normal(size=shape) for _ in range(9)]
    y = [rng.normal(size=shape) for _ in range(6)]
    g = _grid(ndim, shape, dt, "f64", m, p, solver=solver)
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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_source_assembly_wrapped_overlapping_windows_bitwise(dtype):
    """J0 = sum_s a_s shape_s with more sources than one chunk of a
    workgroup's list (600), origins far outside the grid on both sides, a
    window as wide as the grid's short side and a grid that is not a multiple
    of the 64 x 4 cell blocks: every cell must equal, bitwise, the sum taken
    one source after another in source order."""
    import torch
    ny, nx, nsrc, W = 37, 150, 600, 37
    npd = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(77)
    origins = np.stack([rng.integers(-5 * nx, 5 * nx, size=nsrc), rng.integers(-5 * ny, 5 * ny, size=nsrc)], axis=1)
    shapes = rng.normal(size=(nsrc, 3, W, W)).astype(npd)
    amps = rng.normal(size=nsrc).astype(npd)
    want = [np.zeros((ny, nx), dtype=npd) for _ in range(3)]
    for k in range(nsrc):
        ys = (origins[k, 1] + np.arange(W)) % ny
        xs = (origins[k, 0] + np.arange(W)) % nx
        for c in range(3):
            want[c][np.ix_(ys, xs)] += amps[k] * shapes[k, c]
    g = _grid(2, (ny, nx), 0.3, dtype, 0, 0)
    td = torch.float64 if dtype == "f64" else torch.float32
    J = [torch.full((ny, nx), float("nan"), dtype=td, device="cuda") for _ in range(3)]
    g.sources_assemble(torch.tensor(origins, dtype=torch.int64, device="cuda"),
                       torch.tensor(shapes, device="cuda"), torch.tensor(amps, device="cuda"), J)
    for a, b in zip(to_np(J), want):
        assert np.array_equal(a, b)


def _probe_loss(E, win):
    return (E[2][win] ** 2).sum()


def _run_autograd(n, nsrc, nsteps, ck, dtype, seed=1005, sigma=8.0, window=4.0, win_half=32, verify=True,
                  inputs_dtype=None):
    """inputs_dtype: the dtype every input is rounded to (default: the run's)."""
    import torch
    from paper_1907_13088_amd.adjoint import SourceSet, field_steps
    idt = inputs_dtype or dtype
    w = I.modes_2d((n, n), nmodes=64, npulses=0, steps=nsteps, seed=seed, dtype=idt)
    origins, shapes, amps = I.adjoint_sources_2d(n=n, nsrc=nsrc, sigma=sigma, seed=seed, window=window)
    td = torch.float64 if dtype == "f64" else torch.float32
    shapes = np.asarray(I.round_to(np.float32 if idt == "f32" else np.float64, shapes))
    amps = np.asarray(I.round_to(np.float32 if idt == "f32" else np.float64, amps))
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


def test_autograd_full_size_against_oracle_golden():
    """2048^2, 256 sources with learnable amplitudes, 500 steps, checkpoint every
    50, objective sum of E_z^2 over a 64 x 64 window, every input rounded to
    FP32: the FP64 GPU gradients agree with the FP64 oracle's
    (tests/golden/adjoint_2048_grad.json, written by the committed script
    beside it from oracle/ alone) within 1e-10, the FP32 GPU gradients within
    1e-4 (amplitudes normwise and per entry on the scale of the largest,
    initial fields in norm and at 512 sampled cells), and FP64 central
    differences confirm three amplitude gradients."""
    import torch
    with open(GOLDEN) as f:
        gold = json.load(f)
    n, nsrc, nsteps = 2048, 256, 500
    ga_gold = np.array(gold["grad_amps"])
    cells = np.array(gold["sample_cells_yx"])
    runs = {}
    for dtype, tol in (("f64", 1e-10), ("f32", 1e-4)):
        log(f"full-size adjoint {dtype}")
        r = _run_autograd(n, nsrc, nsteps, 50, dtype, inputs_dtype="f32")
        runs[dtype] = r
        e_L = abs(r["L"] - gold["L"]) / abs(gold["L"])
        e_norm = np.linalg.norm(r["ga"] - ga_gold) / np.linalg.norm(ga_gold)
        e_ent = np.abs(r["ga"] - ga_gold).max() / np.abs(ga_gold).max()
        # the objective is E_z only: the TE components' gradients are exactly 0
        norms = gold["grad_E0_norm"] + gold["grad_B0_norm"]
        gmax = max(norms)
        e_fn = max(abs(np.linalg.norm(x) - g) / (g if g > 0 else gmax) for x, g in zip(r["gE"] + r["gB"], norms))
        assert all(np.linalg.norm(x) == 0.0 for x, g in zip(r["gE"] + r["gB"], norms) if g == 0.0)
        samp = [x[cells[:, 0], cells[:, 1]] for x in r["gE"] + r["gB"]]
        gs = [np.array(v) for v in gold["grad_E0_samples"] + gold["grad_B0_samples"]]
        e_s = max(np.abs(a - b).max() for a, b in zip(samp, gs)) / max(np.abs(b).max() for b in gs)
        log(f"{dtype} vs oracle golden: L {e_L:.2e}, amplitude gradient normwise {e_norm:.2e}, per entry "
            f"{e_ent:.2e}, field gradient norms {e_fn:.2e}, sampled field gradient {e_s:.2e}")
        assert max(e_L, e_norm, e_ent, e_fn, e_s) <= tol
    from paper_1907_13088_amd.adjoint import field_steps
    td = torch.float64
    r64 = runs["f64"]
    w = r64["w"]
    ga64 = r64["ga"]

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
