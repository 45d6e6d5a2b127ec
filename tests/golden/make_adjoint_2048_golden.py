"""Write tests/golden/adjoint_2048_grad.json: the FP64 oracle's gradients of
the full-size adjoint workload.

Workload (the GPU test in tests/test_gpu_adjoint.py takes the same inputs):
2048^2 periodic grid, Courant 0.5, m = 20 sweeps, 3 filter passes, 500
steps, initial fields 64 seeded Fourier modes (seed 1005), 256 seeded
Gaussian current sources with amplitudes a_s (seed 1005, sigma 8, windows of
4 sigma), envelope sin(0.3 (n + 1/2) dt); every input rounded to FP32 first,
so the FP32 and the FP64 GPU runs see the values the oracle sees.
Objective L = sum of E_z^2 over the 64 x 64 window [992, 1056)^2 after the
last step.

The oracle runs the forward steps with J0 = sum_s a_s g_s, seeds E_z-bar =
2 E_z on the window, runs the transposed steps (the adjoint of Alg 1 with the
same counts, eqs faraday_* and ampere_aux_* transposed) and projects the
current gradient on the source shapes: dL/da_s = <g_s, dL/dJ0>.  Stored: L,
the 256 amplitude gradients, the L2 norm of each initial-field gradient
component, and the initial-field gradient at 512 seeded cells.

Calls only oracle/ and the input generators; about an hour on 8 host cores:
    python tests/golden/make_adjoint_2048_golden.py
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ref  # noqa: E402
from paper_1907_13088_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_2048_grad.json")
N, NSRC, NSTEPS, M, P = 2048, 256, 500, 20, 3
SEED, SIGMA, WINDOW, WIN_HALF = 1005, 8.0, 4.0, 32


def inputs():
    """The workload's inputs, rounded to FP32 (returned as float64)."""
    w = I.modes_2d((N, N), nmodes=64, npulses=0, steps=NSTEPS, seed=SEED, dtype="f32")
    origins, shapes, amps = I.adjoint_sources_2d(n=N, nsrc=NSRC, sigma=SIGMA, seed=SEED, window=WINDOW)
    shapes = np.asarray(I.round_to(np.float32, shapes))
    amps = np.asarray(I.round_to(np.float32, amps))
    env = [math.sin(0.3 * (s + 0.5) * w.dt) for s in range(NSTEPS)]
    c0 = N // 2 - WIN_HALF
    win = (slice(c0, c0 + 2 * WIN_HALF), slice(c0, c0 + 2 * WIN_HALF))
    return w, origins, shapes, amps, env, win


def sample_cells(count=512, seed=77):
    rng = np.random.default_rng(seed)
    return rng.integers(0, N, size=(count, 2))   # (y, x)


def main():
    w, origins, shapes, amps, env, win = inputs()
    cfg = ref.Config(ndim=2, shape=(N, N), dt=w.dt, sweeps=M, filter_passes=P)
    J0 = I.assemble_sources(N, origins, shapes, amps)
    E = [a.copy() for a in w.E]
    B = [a.copy() for a in w.B]
    t0 = time.time()
    for s in range(NSTEPS):
        ref.step(cfg, E, B, J0, env[s])
        if s % 25 == 24:
            print(f"forward {s + 1}/{NSTEPS} {time.time() - t0:.0f}s", flush=True)
    L = float((E[2][win] ** 2).sum())
    Eb = [np.zeros((N, N)) for _ in range(3)]
    Eb[2][win] = 2.0 * E[2][win]
    Bb = [np.zeros((N, N)) for _ in range(3)]
    Jb = [np.zeros((N, N)) for _ in range(3)]
    del E, B
    for s in reversed(range(NSTEPS)):
        ref.adjoint_step(cfg, Eb, Bb, Jb, env[s], (M, M))
        if s % 25 == 0:
            print(f"adjoint {NSTEPS - s}/{NSTEPS} {time.time() - t0:.0f}s", flush=True)
    W = shapes.shape[-1]
    ga = []
    for s in range(NSRC):
        xs = (origins[s, 0] + np.arange(W)) % N
        ys = (origins[s, 1] + np.arange(W)) % N
        ga.append(float(sum(np.sum(shapes[s, c] * Jb[c][np.ix_(ys, xs)]) for c in range(3))))
    cells = sample_cells()
    out = {
        "what": "FP64 oracle gradients of L = sum E_z^2 over [992,1056)^2 after 500 steps; "
                "2048^2, Courant 0.5, m=20, p=3, 64 modes and 256 sources (seed 1005), inputs rounded to FP32",
        "script": "tests/golden/make_adjoint_2048_golden.py",
        "L": L,
        "grad_amps": ga,
        "grad_E0_norm": [float(np.linalg.norm(x)) for x in Eb],
        "grad_B0_norm": [float(np.linalg.norm(x)) for x in Bb],
        "sample_cells_yx": cells.tolist(),
        "grad_E0_samples": [[float(x[y, i]) for y, i in cells] for x in Eb],
        "grad_B0_samples": [[float(x[y, i]) for y, i in cells] for x in Bb],
        "oracle_threads": ref.num_threads(),
        "seconds": round(time.time() - t0, 1),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}: L = {L:.12e}, |grad a| = {np.linalg.norm(ga):.6e}", flush=True)


if __name__ == "__main__":
    main()
