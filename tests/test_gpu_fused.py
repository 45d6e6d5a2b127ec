"""The front fused with the first sweep pass (variant 4, the FP32 default).

One row-streaming pass runs the Faraday update, the current filter and the
auxiliary increment dE' (Sec. 2.2.2), and at once the first K sweeps of
Alg 1 from x_0 = dE'.  It performs the same floating-point operations as
the separate front and first pass, so every fused depth K (3..6) and filter
depth p (0..4) must give bitwise the fields of the separate schedule
(variant 2), which the other 2D tests pin to the FP64 oracle; the library
profile shows that the fused kernel ran.  FP32 results are also checked
against the FP64 oracle directly.
"""
import numpy as np
import pytest

from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import gpu_config, log, rel_err, run_oracle, to_np, torch_fields

pytestmark = pytest.mark.gpu


def run(w, nsteps, variant, spp=0, sweeps=None, current=True):
    import torch
    g = mx.Grid(gpu_config(w, dtype="f32", spp=spp, sweeps=sweeps, variant=variant))
    E, B = torch_fields(w.E, "f32"), torch_fields(w.B, "f32")
    g.bind(E, B)
    if current and w.J0 is not None:
        g.set_current(torch_fields(w.J0, "f32"))
    g.profile_enable(True)
    g.step(nsteps, env=None if w.env is None else list(w.env[:nsteps]))
    prof = g.profile_read()
    torch.cuda.synchronize()
    out = to_np(E) + to_np(B)
    g.close()
    return out, prof["front_sweep"]["launches"]


# (grid, m, sweeps per pass): first passes of m // ceil(m / spp) = 6, 3, 4, 5, 6, 6 sweeps
CASES = [((203, 141), 20, 0), ((203, 141), 9, 3), ((203, 141), 8, 4), ((203, 141), 10, 5),
         ((97, 70), 12, 6), ((700, 41), 20, 7)]


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_fused_front_bitwise_equal_to_separate_passes(p):
    for shape, m, spp in CASES:
        w = I.modes_2d(shape, nmodes=24, npulses=6, filter_passes=p, m=m, steps=4, seed=4000 + p, dtype="f32")
        k = m // -(-m // (spp or 9))
        got, nf = run(w, 3, mx.VARIANT_STREAM_FUSED, spp=spp)
        want, n0 = run(w, 3, mx.VARIANT_STREAM, spp=spp)
        log(f"fused p={p} {shape} m={m} spp={spp} K={k}: fused launches {nf}")
        assert n0 == 0
        assert nf == 3
        for a, b in zip(got, want):
            assert np.array_equal(a, b), (p, shape, m, spp)


def test_fused_front_tiny_grids():
    """Grids smaller than one strip and than the pipeline depth (halos wrap
    many times over), with a random current."""
    for n in ((1, 1), (2, 3), (5, 4), (7, 1), (300, 2), (3, 40)):
        w = I.modes_2d(n, nmodes=0, npulses=0, steps=3, seed=3, dtype="f32")
        rng = np.random.default_rng(1)
        w.E = [rng.normal(size=w.shape).astype(np.float32) for _ in range(3)]
        w.B = [rng.normal(size=w.shape).astype(np.float32) for _ in range(3)]
        w.J0 = [rng.normal(size=w.shape).astype(np.float32) for _ in range(3)]
        w.env = np.ones(3)
        w.filter_passes = 3
        got, nf = run(w, 3, mx.VARIANT_STREAM_FUSED)
        want, _ = run(w, 3, mx.VARIANT_STREAM)
        assert nf == 3, n
        for a, b in zip(got, want):
            assert np.array_equal(a, b), n


def test_fused_front_without_current_and_with_replayed_counts():
    """No current (the kernel without the filter); per-step counts that
    fuse only when both blocks take the same count in more than one pass."""
    import torch
    w = I.modes_2d((330, 97), nmodes=24, npulses=6, filter_passes=3, m=20, steps=4, seed=4100, dtype="f32")
    got, nf = run(w, 3, mx.VARIANT_STREAM_FUSED, current=False)
    want, _ = run(w, 3, mx.VARIANT_STREAM, current=False)
    assert nf == 3
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    counts = [(20, 20), (6, 6), (9, 11), (13, 13)]   # fused (6 + 7 + 7), single pass, unequal, fused (6 + 7)
    outs = []
    for variant in (mx.VARIANT_STREAM_FUSED, mx.VARIANT_STREAM):
        g = mx.Grid(gpu_config(w, dtype="f32", variant=variant))
        E, B = torch_fields(w.E, "f32"), torch_fields(w.B, "f32")
        g.bind(E, B)
        g.set_current(torch_fields(w.J0, "f32"))
        g.profile_enable(True)
        g.step(len(counts), env=list(w.env[:len(counts)]), replay=counts)
        nf = g.profile_read()["front_sweep"]["launches"]
        torch.cuda.synchronize()
        outs.append((to_np(E) + to_np(B), nf))
        g.close()
    assert outs[0][1] == 2 and outs[1][1] == 0
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)


def test_fused_front_fp32_against_fp64_oracle():
    """A ragged grid (cfg2 recipe): FP32 within 1e-5 of the FP64 oracle
    after 40 steps (at this size the library's own choice is the LDS-tile
    kernel, so the fused variant is asked for)."""
    w = I.modes_2d((300, 211), nmodes=32, npulses=8, filter_passes=3, m=20, steps=40, seed=4200, dtype="f32")
    got, nf = run(w, 40, mx.VARIANT_STREAM_FUSED)
    assert nf == 40
    Eo, Bo, _ = run_oracle(w, 40)
    e = rel_err(got, Eo + Bo)
    log(f"fused FP32 vs oracle after 40 steps: {max(e):.2e}")
    assert max(e) < 1e-5
