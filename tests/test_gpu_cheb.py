"""Chebyshev-accelerated solve of the 2D mass-matrix system (the paper's
future-work direction) on the HIP path against the FP64 oracle's Chebyshev
semi-iteration, through the C-ABI.

Bars as for Alg 1: FP64 within 1e-12 (counts replayed under a tolerance),
FP32 within 1e-5; the GPU's stop decisions within one check of the oracle's;
every pass depth and both streaming variants give bitwise identical FP32
iterates."""
import numpy as np
import pytest

from paper_1907_13088_amd import inputs as I
from paper_1907_13088_amd import mx

from gpu_helpers import gpu_config, log, rel_err, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
CHEB = mx.SOLVER_CHEBYSHEV
# deepest Chebyshev pass (TE, TM) in FP64: both blocks in one pass, each on its own
KMAX_F64 = {mx.VARIANT_STREAM: (2, 2), mx.VARIANT_STREAM_BLOCK: (4, 8)}


@pytest.fixture(scope="module")
def small_modes():
    return I.modes_2d((200, 136), nmodes=48, npulses=8, filter_passes=3, m=13, steps=40, seed=2102,
                      dtype="f64")


@pytest.mark.parametrize("variant,spp", [(mx.VARIANT_STREAM, 1), (mx.VARIANT_STREAM, 2),
                                         (mx.VARIANT_STREAM_BLOCK, 1), (mx.VARIANT_STREAM_BLOCK, 2),
                                         (mx.VARIANT_STREAM_BLOCK, 3), (mx.VARIANT_STREAM_BLOCK, 6),
                                         (mx.VARIANT_STREAM_BLOCK, 8), (mx.VARIANT_STREAM_BLOCK, 0)])
def test_cheb_fp64_fixed_m_every_pass_depth(small_modes, variant, spp):
    w = small_modes
    nsteps = 8
    g = mx.Grid(gpu_config(w, spp=spp, variant=variant, solver=CHEB))
    want = tuple(min(spp, k) if spp else k for k in KMAX_F64[variant])
    assert g.block_sweeps_per_pass == want
    g.close()
    Eg, Bg, stg, _ = run_gpu(w, nsteps, spp=spp, variant=variant, solver=CHEB)
    Eo, Bo, sto = run_oracle(w, nsteps, solver=CHEB)
    assert all(list(s.sweeps) == [13, 13] for s in stg)
    e = rel_err(Eg + Bg, Eo + Bo)
    log(f"chebyshev variant={variant} spp={spp} fp64 errors {max(e):.3e}")
    assert max(e) < 1e-12


def test_cheb_fp32_fixed_m_and_bitwise_schedule_invariance(small_modes):
    """FP32 within 1e-5 of the FP64 oracle after 40 steps, and identical bits
    for every pass depth of both streaming variants."""
    w = small_modes
    nsteps = 40
    Eo, Bo, _ = run_oracle(w, nsteps, solver=CHEB)
    ref = None
    for variant, spp in ((mx.VARIANT_STREAM, 0), (mx.VARIANT_STREAM, 3), (mx.VARIANT_STREAM, 1),
                         (mx.VARIANT_STREAM_BLOCK, 0), (mx.VARIANT_STREAM_BLOCK, 4), (mx.VARIANT_STREAM_BLOCK, 7)):
        Eg, Bg, _, _ = run_gpu(w, nsteps, dtype="f32", spp=spp, variant=variant, solver=CHEB)
        e = rel_err(Eg + Bg, Eo + Bo)
        log(f"chebyshev fp32 variant={variant} spp={spp}: {max(e):.2e}")
        assert max(e) < 1e-5
        if ref is None:
            ref = Eg + Bg
        else:
            assert all(np.array_equal(a, b) for a, b in zip(ref, Eg + Bg)), (variant, spp)


def test_cheb_tolerance_te_planewave_decisions_and_replay():
    """128^2 TE plane wave + noise, FP64, tol 1e-12 (the Alg 1 tolerance
    workload): the GPU stops within one check of the oracle, replaying the
    oracle's counts matches it to FP64 rounding, and the Chebyshev solve
    takes fewer sweeps than Alg 1 (the smooth plane wave sits where the
    Chebyshev error polynomial peaks, at the zero end of the spectrum of A,
    so the saving is smaller here than for white noise)."""
    w = I.planewave_te_2d()
    nsteps = 30
    Eg, Bg, stg, spp = run_gpu(w, nsteps, solver=CHEB)
    Eo, Bo, sto = run_oracle(w, nsteps, check_every=spp, solver=CHEB)
    diffs = [abs(a.sweeps[0] - b.sweeps[0]) for a, b in zip(stg, sto)]
    assert max(diffs) <= spp and sum(d > 0 for d in diffs) <= 2
    Eg, Bg, _, _ = run_gpu(w, nsteps, replay=[s.sweeps for s in sto], solver=CHEB)
    e = rel_err(Eg[:2] + [Bg[2]], Eo[:2] + [Bo[2]])
    log(f"chebyshev te planewave replay errors {max(e):.2e}")
    assert max(e) < 1e-12
    _, _, sta = run_oracle(w, nsteps, check_every=1)
    _, _, stc = run_oracle(w, nsteps, check_every=1, solver=CHEB)
    alg1 = np.mean([s.sweeps[0] for s in sta])
    cheb = np.mean([s.sweeps[0] for s in stc])
    log(f"sweeps per step to 1e-12: Alg 1 {alg1:.1f}, Chebyshev {cheb:.1f}")
    assert cheb < 0.75 * alg1


def test_cheb_tolerance_both_blocks_stop_independently():
    """TE+TM to tol 1e-10 in FP64 with currents: the blocks stop on their own
    counts (TM converges more slowly); replayed counts give 1e-12 agreement."""
    w = I.modes_2d((72, 88), nmodes=24, npulses=4, filter_passes=2, m=200, steps=10, seed=2103, dtype="f64")
    w.tol = 1e-10
    nsteps = 6
    Eg, Bg, stg, spp = run_gpu(w, nsteps, solver=CHEB)
    Eo, Bo, sto = run_oracle(w, nsteps, check_every=spp, solver=CHEB)
    for a, b in zip(stg, sto):
        assert all(abs(a.sweeps[q] - b.sweeps[q]) <= spp for q in range(2))
    assert any(s.sweeps[0] != s.sweeps[1] for s in sto)
    Eg, Bg, _, _ = run_gpu(w, nsteps, replay=[s.sweeps for s in sto], solver=CHEB)
    e = rel_err(Eg + Bg, Eo + Bo)
    log(f"chebyshev TE+TM tolerance replay errors {max(e):.2e}")
    assert max(e) < 1e-12


def test_cheb_rejections():
    w = I.modes_2d((32, 32), nmodes=4, npulses=0, m=5, steps=1, seed=1, dtype="f64")
    with pytest.raises(mx.MxError):
        mx.Grid(gpu_config(w, variant=mx.VARIANT_TILE, solver=CHEB))
    with pytest.raises(mx.MxError):
        mx.Grid(gpu_config(w, lumped=True, solver=CHEB))


def test_cheb_fp32_tolerance_1e6():
    """FP32 Chebyshev solve to tol 1e-6 (above the FP32 rounding floor of
    the residual b + A x - x): every step converges, and the fields agree
    with the FP64 oracle run on the GPU's own counts within 1e-5."""
    w = I.modes_2d((136, 120), nmodes=32, npulses=4, filter_passes=2, m=200, steps=12, seed=2104, dtype="f32")
    w.tol = 1e-6
    nsteps = 10
    Eg, Bg, stg, _ = run_gpu(w, nsteps, solver=CHEB)
    assert all(tuple(s.nonconverged) == (0, 0) for s in stg)
    assert all(0 < s.sweeps[0] < 200 and 0 < s.sweeps[1] < 200 for s in stg)
    Eo, Bo, _ = run_oracle(w, nsteps, replay=[s.sweeps for s in stg], solver=CHEB)
    e = rel_err(Eg + Bg, Eo + Bo)
    log(f"chebyshev fp32 tol 1e-6: sweeps {[tuple(s.sweeps) for s in stg][:3]}, errors {max(e):.2e}")
    assert max(e) < 1e-5
