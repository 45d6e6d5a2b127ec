#!/usr/bin/env python3
"""Throughput of the finite-element Maxwell field step on one MI355X.

Workload: 2D periodic 4096 x 4096 grid, FP32, TE+TM (six components),
Courant 0.5 (dt = 0.5 dt_CFL), initial fields = 256 seeded Fourier modes
with |k| <= pi/2 and N(0,1) amplitudes, prescribed current = 64 seeded
Gaussian pulses (sigma = 8 cells, sin(0.3 t) envelope), 3-pass binomial
current filter every step, m = 20 mass-matrix sweeps per step.

A step is one full time step: filter + Faraday + auxiliary increment, the
20 sweeps, and the E increment.  Inputs are resident in HBM before timing.
Reported: Gcell-steps/s (cells x steps / s) in FP32, the same for the FP64
path and the FP32 error against it after the same steps, per-kernel times
from HIP events recorded on the library stream inside the timed region, the
roofline of the dominant kernel (the sweep pass that stores its iterate)
with HBM traffic read from the committed rocprofv3 counter summary when the
kernel sources still match it, and the FP64 CPU oracle timed on this
host's cores on a bounded sample.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
# FP32 FMA issue rate without the packed two-wide forms (not used in this
# build): 256 CUs x 64 lanes x 2 flops x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 78.6
HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE_SUMMARY = os.path.join(HERE, "profiles", "step_2d_4096sq_f32.md")
# per-launch timing events are recorded on the last steps of the timed
# region: all of it below PSTRIDE steps, else an even count near K / 4 (the
# event records cost about 3 us per launch; even step counts per call let
# the library hand B back in the caller's buffer without a copy)
PSTRIDE = 20
# single steps after the timed region whose two probed lattice modes give
# the fitted frequencies omega(k) of the FP32 and FP64 runs
OMEGA_TAIL = 8


def sampled_steps(K):
    return K if K < PSTRIDE else max(2, (K // 4) & ~1)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--spp", type=int, default=0, help="sweeps per pass (0 = library choice)")
    ap.add_argument("--variant", type=int, default=0,
                    help="2D sweep kernel: 0 library choice, 1 LDS tile, 2 row streaming, "
                         "3 row streaming per block, 4 row streaming with the front fused into the first pass")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="minimum CPU time of the oracle sample (whole steps, at most 8)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run 4 plain device copies of this many bytes (counter calibration)")
    ap.add_argument("--workload", default="modes2d",
                    choices=["modes2d", "planewave_te", "planewave_3d", "batch", "adjoint", "chebyshev", "chebyshev_3d",
                             "pic"],
                    help="modes2d (default): the 4096^2 line above; the others time the 128^2 TE "
                         "tolerance solve, the 512^3 3D solve, the 64-grid batch, the adjoint and the "
                         "Chebyshev solve against Alg 1 in 2D (chebyshev) and 3D (chebyshev_3d)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the field step runs on one GPU; a multi-GPU run (spatial domain "
              "decomposition with halo exchange) is not part of this library", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    from paper_1907_13088_amd import profsum

    mx.lib()  # raises if the HIP library is missing: no fallback path exists
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)

    global SPP
    SPP = args.spp
    if args.copy_probe > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the HBM traffic read for the field kernels
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 4 x {args.copy_probe} bytes")
        del src, dst

    if args.workload != "modes2d":
        steps = args.steps if "--steps" in sys.argv else None
        warm = args.warmup if "--warmup" in sys.argv else None
        print(json.dumps(OTHER_WORKLOADS[args.workload](steps, warm)), flush=True)
        return

    K, W = args.steps, args.warmup
    n = args.n
    t0 = time.time()
    w = I.modes_2d((n, n), steps=W + K + OMEGA_TAIL, dtype="f32")
    log(f"inputs generated in {time.time() - t0:.1f}s")
    env = [float(x) for x in w.env]
    env_tail = env[W + K:]
    ncell = n * n

    def make(dtype):
        td = torch.float64 if dtype == "f64" else torch.float32
        cfg = mx.make_config(2, (n, n), w.dt, (1.0, 1.0), dtype, mx.MX_ALL, w.sweeps, 0.0,
                             w.filter_passes, sweeps_per_pass=args.spp, variant=args.variant)
        g = mx.Grid(cfg)
        E = [torch.tensor(a, dtype=td, device="cuda") for a in w.E]
        B = [torch.tensor(a, dtype=td, device="cuda") for a in w.B]
        J = [torch.tensor(a, dtype=td, device="cuda") for a in w.J0]
        g.bind(E, B)
        g.set_current(J)
        return g, E, B, J

    # two probed lattice modes for the frequency fit: the largest amplitudes
    # with |k| > 1, where the pulses' spectrum (sigma = 8) is negligible
    import math
    probes = sorted([md for md in w.meta["modes"]
                     if math.hypot(*[2 * math.pi * md["n"][a] / n for a in range(2)]) > 1.0],
                    key=lambda md: -abs(md["amp"]))[:2]

    def project(F, md):
        """(2/N) sum F exp(-i k.(x + offset)) in FP64 on the device"""
        off = I.B_OFFSETS[2][2] if md["pol"] == "TE" else I.E_OFFSETS[2][2]
        k = [2 * math.pi * md["n"][a] / n for a in range(2)]
        ar = torch.arange(n, dtype=torch.float64, device=F.device)
        ex, ey = torch.exp(-1j * k[0] * (ar + off[0])), torch.exp(-1j * k[1] * (ar + off[1]))
        return complex(2.0 * (ey @ (F.double().to(torch.complex128) @ ex)) / F.numel())

    def omega_fit(a, dt):
        """w from a_{n+1} + a_{n-1} = 2 cos(w dt) a_n (least squares)"""
        import numpy as np
        a = np.asarray(a)
        c = (np.vdot(a[1:-1], a[2:] + a[:-2]) / (2.0 * np.vdot(a[1:-1], a[1:-1]))).real
        return math.acos(max(-1.0, min(1.0, c))) / dt

    def timed(dtype):
        g, E, B, J = make(dtype)
        g.step(W, env[:W])
        torch.cuda.synchronize()
        # per-launch HIP events on the library stream over the last ps steps
        # of the timed region
        ps = sampled_steps(K)
        g.profile_enable(True)
        g.profile_enable(False)
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sm = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        s0.record()
        if K > ps:
            g.step(K - ps, env[W:W + K - ps])
        sm.record()
        g.profile_resume()
        g.step(ps, env[W + K - ps:W + K])
        g.profile_enable(False)
        s1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        prof = g.profile_read()
        ms = s0.elapsed_time(s1)
        prof["sampled_ms"] = sm.elapsed_time(s1)
        log(f"{dtype}: {K} steps in {ms:.1f} ms (wall {wall * 1e3:.1f} ms), "
            f"sweeps per pass {g.block_sweeps_per_pass}, events on the last {ps}")
        state = [t.clone() for t in E + B]
        # frequency probe: single steps after the timed region
        ser = [[] for _ in probes]
        for s in range(OMEGA_TAIL + 1):
            for i, md in enumerate(probes):
                ser[i].append(project(B[2] if md["pol"] == "TE" else E[2], md))
            if s < OMEGA_TAIL:
                g.step(1, [env_tail[s]])
        omegas = [omega_fit(x, w.dt) for x in ser]
        return g, state, ms, prof, ps, omegas

    g32, st32, ms32, prof, nprof, om32 = timed("f32")
    value = ncell * K / (ms32 / 1e3) / 1e9

    fp64 = None
    if not args.no_fp64:
        g64, st64, ms64, _, _, om64 = timed("f64")
        scale = max(float(t.abs().max()) for t in st64)
        err = max(float((a.double() - b).abs().max()) for a, b in zip(st32, st64)) / scale
        om = [{"mode_n": list(md["n"]), "pol": md["pol"], "omega_fp32": a, "omega_fp64": b,
               "rel_err": abs(a - b) / b} for md, a, b in zip(probes, om32, om64)]
        fp64 = {"value": round(ncell * K / (ms64 / 1e3) / 1e9, 3), "ms_per_step": round(ms64 / K, 5),
                "fp32_vs_fp64_rel_err": err, "err_steps": W + K,
                "err_metric": "max |FP32 - FP64| over the six components / max |FP64|",
                "omega": om, "omega_rel_err_max": max((x["rel_err"] for x in om), default=None),
                "omega_metric": f"frequency of two lattice modes (|k| > 1, largest amplitudes) fitted from "
                                f"their Fourier amplitudes over {OMEGA_TAIL} steps after the timed region"}
        log(f"f64: {fp64['value']:.2f} Gcell-steps/s; FP32 vs FP64 normwise rel err after {W + K} steps: "
            f"{err:.2e}; omega rel err {fp64['omega_rel_err_max']:.2e}")
        g64.close()
        del st64

    sampled_ms = prof.pop("sampled_ms")
    total_ms = sum(v["ms"] for v in prof.values())
    kernels = {}
    for name, v in prof.items():
        if v["launches"]:
            kernels[name] = {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / v["launches"], 2),
                             "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                             "share": round(v["ms"] / total_ms, 4)}
    log(f"kernels: {json.dumps(kernels)}")
    k = g32.block_sweeps_per_pass[0]
    # pass depths of a fixed count: the fewest passes, deeper ones last
    depths, rem = [], w.sweeps
    while rem > 0:
        kk = rem // -(-rem // k)
        depths.append(kk)
        rem -= kk
    fused = prof["front_sweep"]["launches"] > 0
    store = depths[1:-1] if fused else depths[:-1]
    # FP32 flops per cell of the implemented stencils (an FMA counts 2): a
    # sweep 33 (TE 18, TM 15); the front about 120 (Faraday 12, the 7-tap x
    # filter 42 and 3 cascaded y passes 36 of the current, dE' 30)
    FRONT_FLOPS, SWEEP_FLOPS = 120.0, 33.0
    desc = {
        "front_sweep": (f"k2_front_sweep<float,P=3,K={depths[0]}>: Faraday, current filter and dE' fused with the "
                        f"first {depths[0]} sweeps (stores B, dE' and the iterate)",
                        FRONT_FLOPS + SWEEP_FLOPS * depths[0],
                        "row streaming with one LDS exchange and barrier per row step, two waves per SIMD "
                        "(234 VGPRs): the sweep levels' latency chain overlaps the front's HBM streams"),
        "sweep": (f"k2_stream<float,3,K> row-streaming sweep passes storing their iterate "
                  f"(K = {'+'.join(map(str, store))})",
                  SWEEP_FLOPS * sum(store) / max(len(store), 1),
                  "the 6- and 7-sweep passes are bound neither by HBM nor by VALU: each row step waits on an "
                  "LDS neighbour exchange and barrier (measured against memory-only twins of the passes)"),
        "sweep_last": (f"k2_stream<float,3,{depths[-1]}> final pass adding the result into E",
                       SWEEP_FLOPS * depths[-1], "as the other sweep passes; reads three arrays more"),
        "front": ("k2_front_stream<float,3,P=3>: Faraday, current filter and dE'", FRONT_FLOPS,
                  "HBM streams with halo rows of the chunked strips"),
    }
    dom = max((c for c in desc if prof[c]["launches"] > 0), key=lambda c: prof[c]["ms"])
    dv = prof[dom]
    nl = max(dv["launches"], 1)
    avg_s = dv["ms"] / 1e3 / nl
    bytes_per_launch = dv["bytes"] / nl
    achieved = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = profsum.traffic_per_launch(PROFILE_SUMMARY, dom)
    flops_per_launch = desc[dom][1] * ncell
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": desc[dom][0], "category": dom,
                "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2), "launches": nl,
                "timed_launches": f"HIP events on every launch of the last {nprof} of the {K} timed steps",
                "limiter": desc[dom][2],
                "valu_tflops": round(flops_per_launch / avg_s / 1e12, 2) if avg_s > 0 else None,
                "valu_peak_tflops": VALU_FP32_PEAK_TFLOPS,
                "step_hbm_GBps": round(sum(v["bytes"] for v in prof.values()) / (total_ms / 1e3) / 1e9, 1),
                "sampled_kernel_us_per_step": round(1e3 * total_ms / max(nprof, 1), 2),
                "sampled_us_per_step": round(1e3 * sampled_ms / max(nprof, 1), 2),
                "kernel_sum_over_sampled_step": round(total_ms / sampled_ms, 4) if sampled_ms > 0 else None,
                "kernel_sum_over_ms_per_step": round(total_ms / max(nprof, 1) / (ms32 / K), 4)}

    # bytes per cell-step: this schedule's (the per-launch algorithmic bytes of
    # every kernel category) against the unfused schedule (Faraday 9 words,
    # each filter pass 6 words per axis, auxiliary increment 9, each sweep 9,
    # E increment 9; FP32 words)
    fused_b = sum(v["bytes"] for v in prof.values()) / (ncell * nprof)
    unfused_b = 4.0 * (9 + 12 * w.filter_passes + 9 + 9 * w.sweeps + 9)
    bytes_model = {"fused_B_per_cell_step": round(fused_b, 1), "unfused_B_per_cell_step": unfused_b,
                   "unfused_equivalent_GBps": round(unfused_b * value, 1)}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import ref
        cfg = ref.Config(ndim=2, shape=w.shape, dt=w.dt, sweeps=w.sweeps, filter_passes=w.filter_passes)
        E = [a.astype("float64") for a in w.E]
        B = [a.astype("float64") for a in w.B]
        J0 = [a.astype("float64") for a in w.J0]
        c0 = time.perf_counter()
        steps = 0
        while steps < 8 and (steps == 0 or time.perf_counter() - c0 < args.cpu_seconds):
            ref.step(cfg, E, B, J0, env[steps])
            steps += 1
        ct = time.perf_counter() - c0
        threads = ref.num_threads()
        cpu = {"value": ncell * steps / ct / 1e9, "unit": "Gcell-steps/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {steps} steps of the same {n}x{n} workload, FP64 C oracle, {ct:.1f} s"}
        # one thread: the next step of the same run
        ref.set_num_threads(1)
        try:
            c0 = time.perf_counter()
            ref.step(cfg, E, B, J0, env[steps])
            ct1 = time.perf_counter() - c0
        finally:
            ref.set_num_threads(threads)
        cpu["single_thread"] = {"value": ncell / ct1 / 1e9, "unit": "Gcell-steps/s", "cores": 1,
                                "sample": f"step {steps + 1} of the same {n}x{n} run on one thread, {ct1:.1f} s"}
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": "Gcell-steps/s incl. mass-matrix sweeps, FP32 vs FP64 @ stated error; %HBM",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms32 / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D periodic {n}x{n} TE+TM FP32, Courant 0.5, 256 Fourier modes |k|<=pi/2, "
                               f"64 Gaussian current pulses, 3-pass binomial filter, m=20 sweeps",
                   "grid": [n, n], "sweeps": w.sweeps, "filter_passes": w.filter_passes,
                   "sweeps_per_pass": list(g32.block_sweeps_per_pass), "pass_depths": depths,
                   "front_fused": fused, "parallelism": "single GPU"},
        "fp64": fp64,
        "roofline": roofline,
        "kernels": kernels,
        "bytes_model": bytes_model,
        "cpu_baseline": cpu,
    }
    g32.close()
    print(json.dumps(out), flush=True)


# --------------------------------------------------------------------------
# The other workloads (not the headline line): each prints one JSON object
# --------------------------------------------------------------------------

SPP = 0   # sweeps per pass of the other workloads' grids (0: library choice), from --spp


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _line(name, value, unit, extra):
    out = {"metric": "Gcell-steps/s incl. mass-matrix sweeps" if unit == "Gcell-steps/s" else name,
           "value": round(value, 4), "unit": unit, "n_gpus": 1, "data": "synthetic", "workload": name}
    out.update(extra)
    return out


def bench_planewave_te(steps, warm):
    """128^2 TE plane wave + noise, FP64, solve to 1e-12 (checked every pass)."""
    import torch
    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    # 1000 steps: over 200 the per-step time of this latency-bound case
    # varies twofold with the GPU clock ramping up
    steps = steps or 1000
    w = I.planewave_te_2d(steps=steps)
    cfg = mx.make_config(2, w.shape[::-1], w.dt, w.d, "f64", w.blocks, w.sweeps, w.tol, 0, sweeps_per_pass=SPP)
    g = mx.Grid(cfg)
    E = [torch.tensor(a, device="cuda") for a in w.E]
    B = [torch.tensor(a, device="cuda") for a in w.B]
    g.bind(E, B)
    g.step(warm or 5)
    torch.cuda.synchronize()
    # five repeats, the median reported: the step time of this latency-bound
    # case follows the GPU clock, which does not stay at its peak under a
    # launch of 64 workgroups (the same 1000 steps took 62-121 us per step)
    times, sweeps = [], 0.0
    for _ in range(5):
        t0 = time.perf_counter()
        st = g.step(steps, stats=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        sweeps = sum(s.sweeps[0] for s in st) / steps
    dt = sorted(times)[2]
    return _line("128x128 TE plane wave, FP64, tol 1e-12", w.cells * steps / dt / 1e9, "Gcell-steps/s",
                 {"steps": steps, "repeats": 5, "us_per_step": round(dt / steps * 1e6, 1),
                  "us_per_step_range": [round(min(times) / steps * 1e6, 1), round(max(times) / steps * 1e6, 1)],
                  "mean_sweeps": round(sweeps, 1), "sweeps_per_pass": g.sweeps_per_pass, "dtype": "f64",
                  "note": "latency bound: one cooperative launch runs up to 64 steps, the stop test on the device; "
                          "the median of 5 repeats"})


def _run_3d(steps, warm, solver, form, dtype="f32"):
    """Step the 512^3 plane-wave workload (tol 1e-7) with one solver;
    returns (Gcell-steps/s, details)."""
    import torch
    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    t0 = time.time()
    w = I.planewave_3d(steps=steps + warm, dtype=dtype)
    log(f"3D inputs generated in {time.time() - t0:.1f}s")
    cfg = mx.make_config(3, w.shape[::-1], w.dt, w.d, dtype, 3, w.sweeps, w.tol, w.filter_passes,
                         form=form, solver=solver, sweeps_per_pass=SPP)
    g = mx.Grid(cfg)
    td = torch.float64 if dtype == "f64" else torch.float32
    E = [torch.tensor(a, dtype=td, device="cuda") for a in w.E]
    B = [torch.tensor(a, dtype=td, device="cuda") for a in w.B]
    J = [torch.tensor(a, dtype=td, device="cuda") for a in w.J0]
    del w.E, w.B, w.J0
    g.bind(E, B)
    g.set_current(J)
    env = [float(x) for x in w.env]
    if warm:
        g.step(warm, env[:warm])
    torch.cuda.synchronize()
    g.profile_enable(True)
    t0 = time.perf_counter()
    st = g.step(steps, env[warm:warm + steps], stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = g.profile_read()
    g_spp = g.sweeps_per_pass
    g.close()
    del E, B, J
    torch.cuda.empty_cache()
    sw = prof["sweep"]
    sweeps = sum(s.sweeps[0] for s in st) / steps
    return w.cells * steps / dt / 1e9, {
        "steps": steps, "ms_per_step": round(dt / steps * 1e3, 2), "mean_sweeps": round(sweeps, 1),
        "sweeps_per_pass": g_spp,
        "nonconverged_steps": sum(s.nonconverged[0] for s in st),
        "front_us": round(1e3 * prof["front"]["ms"] / max(prof["front"]["launches"], 1), 1),
        "front_GBps": round(prof["front"]["bytes"] / (prof["front"]["ms"] / 1e3) / 1e9, 1) if prof["front"]["ms"] else None,
        "sweep_pass_us": round(1e3 * sw["ms"] / max(sw["launches"], 1), 1),
        "sweep_pass_GBps": round(sw["bytes"] / (sw["ms"] / 1e3) / 1e9, 1) if sw["ms"] else None}


def bench_planewave_3d(steps, warm):
    """512^3, FP32, all six components, tol 1e-7 (delta form); the same in
    FP64 beside it (two steps)."""
    from paper_1907_13088_amd import mx
    v, det = _run_3d(steps or 5, 1 if warm is None else warm, mx.SOLVER_ALG1, mx.FORM_DELTA)
    v64, d64 = _run_3d(2, 1, mx.SOLVER_ALG1, mx.FORM_DELTA, "f64")
    return _line("512^3 plane wave + 32 pulses, FP32, tol 1e-7", v, "Gcell-steps/s",
                 {**det, "dtype": "f32", "fp64": {**d64, "Gcell_steps_per_s": round(v64, 4)}})


def bench_chebyshev_3d(steps, warm):
    """The 512^3 FP32 workload to tol 1e-7 with the Chebyshev solve (cubic
    cells, 1 - A on [1/9, 1], one sweep per pass), beside Alg 1 (delta form)."""
    from paper_1907_13088_amd import mx
    steps, warm = steps or 5, 1 if warm is None else warm
    v1, d1 = _run_3d(steps, warm, mx.SOLVER_ALG1, mx.FORM_DELTA)
    vc, dc = _run_3d(steps, warm, mx.SOLVER_CHEBYSHEV, mx.FORM_STANDARD)
    return _line("512^3 plane wave + 32 pulses, FP32, tol 1e-7, Chebyshev solve", vc, "Gcell-steps/s",
                 {"dtype": "f32", "chebyshev": dc, "alg1_delta": {**d1, "Gcell_steps_per_s": round(v1, 4)},
                  "speedup": round(vc / v1, 3)})


def _batch_run(ws, steps, warm, persistent, dtype):
    """Step the batch with one schedule; returns its result record."""
    import torch
    from paper_1907_13088_amd import mx
    cells = sum(w.cells for w in ws)
    td = torch.float64 if dtype == "f64" else torch.float32
    cfgs = [mx.make_config(2, w.shape[::-1], w.dt, (1.0, 1.0), dtype, mx.MX_ALL, w.sweeps, 0.0, 0) for w in ws]
    b = mx.Batch(cfgs)
    fields = []
    for gi, w in enumerate(ws):
        E = [torch.tensor(a, dtype=td, device="cuda") for a in w.E]
        B = [torch.tensor(a, dtype=td, device="cuda") for a in w.B]
        b.bind(gi, E, B)
        fields.append((E, B))
    b.step(warm or 2, persistent=persistent)
    torch.cuda.synchronize()
    s0, s1 = _events()
    s0.record()
    b.step(steps, persistent=persistent)
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1)
    rec = {"Gcell_steps_per_s": round(cells * steps / ms / 1e6, 3), "ms": round(ms, 1),
           "plan": {**b.schedule(persistent), "persistent_blocks": b.plan()["persistent_blocks"]}}
    b.close()
    del fields
    torch.cuda.empty_cache()
    return rec


def bench_batch(steps, warm):
    """64 grids of uneven size and Courant number, FP32, m = 20, one persistent
    launch (and the grouped schedule beside it; both again in FP64 over 100
    steps)."""
    import torch
    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    steps = steps or 500
    t0 = time.time()
    ws = I.batch_2d(steps=steps)
    log(f"batch inputs generated in {time.time() - t0:.1f}s")
    cells = sum(w.cells for w in ws)
    res = {}
    for persistent in (True, False):
        res["persistent" if persistent else "grouped"] = _batch_run(ws, steps, warm, persistent, "f32")
    ws64 = I.batch_2d(steps=100, dtype="f64")
    res["fp64"] = {("persistent" if p else "grouped"): _batch_run(ws64, 100, warm, p, "f64") for p in (True, False)}
    return _line("64 batched 2D grids, FP32, m = 20", res["persistent"]["Gcell_steps_per_s"], "Gcell-steps/s",
                 {"steps": steps, "cells": cells, "dtype": "f32", "schedules": res})


def _adjoint_run(steps, dtype):
    """Forward and backward of the 2048^2 adjoint workload; returns
    (forward s, backward s)."""
    import math
    import numpy as np
    import torch
    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    from paper_1907_13088_amd.adjoint import SourceSet, field_steps
    n, nsrc = 2048, 256
    td = torch.float64 if dtype == "f64" else torch.float32
    npd = np.float64 if dtype == "f64" else np.float32
    w = I.modes_2d((n, n), nmodes=64, npulses=0, steps=steps, seed=1005, dtype=dtype)
    origins, shapes, amps = I.adjoint_sources_2d(n=n, nsrc=nsrc, seed=1005)
    shapes = np.asarray(I.round_to(npd, shapes))
    amps = np.asarray(I.round_to(npd, amps))
    env = [math.sin(0.3 * (s + 0.5) * w.dt) for s in range(steps)]
    cfg = mx.make_config(2, (n, n), w.dt, (1.0, 1.0), dtype, mx.MX_ALL, 20, 0.0, 3)
    g = mx.Grid(cfg)
    src = SourceSet(torch.tensor(origins, device="cuda"), torch.tensor(shapes, dtype=td, device="cuda"))
    a = torch.tensor(amps, device="cuda", requires_grad=True)
    E0 = [torch.tensor(x, dtype=td, device="cuda", requires_grad=True) for x in w.E]
    B0 = [torch.tensor(x, dtype=td, device="cuda", requires_grad=True) for x in w.B]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E, B = field_steps(a, E0, B0, g, src, env, steps, checkpoint_every=50, verify=False)
    c0 = n // 2 - 32
    L = (E[2][c0:c0 + 64, c0:c0 + 64] ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.close()
    del E, B, E0, B0, a, src
    torch.cuda.empty_cache()
    return t1 - t0, t2 - t1


def bench_adjoint(steps, warm):
    """2048^2 FP32, 256 learnable sources, forward + backward with checkpoints
    every 50 steps (and the same in FP64 beside it)."""
    steps = steps or 500
    cells = 2048 * 2048
    # an untimed short run of each dtype first: kernel loading and the
    # library's per-device set-up are not part of a step
    for dt in ("f32", "f64"):
        _adjoint_run(2 if warm is None else max(1, warm), dt)
    tf, tb = _adjoint_run(steps, "f32")
    tf64, tb64 = _adjoint_run(steps, "f64")
    return _line(f"2048^2 adjoint, 256 sources, FP32, {steps} steps", cells * steps / (tf + tb) / 1e9, "Gcell-steps/s",
                 {"steps": steps, "dtype": "f32", "forward_s": round(tf, 3), "backward_s": round(tb, 3),
                  "forward_Gcell_steps_per_s": round(cells * steps / tf / 1e9, 3),
                  "backward_Gcell_steps_per_s": round(cells * steps / tb / 1e9, 3),
                  "fp64": {"forward_s": round(tf64, 3), "backward_s": round(tb64, 3),
                           "Gcell_steps_per_s": round(cells * steps / (tf64 + tb64) / 1e9, 3)},
                  "note": "value counts forward and backward (transposed steps and source projection) "
                          "over the same steps; the step is linear, so the backward needs no forward "
                          "state and runs without re-verifying the checkpointed segments"})


def _cheb_sweeps_matching_alg1(dt, d, m):
    """Fewest Chebyshev sweeps whose worst-case error factor 1/T_k(theta/delta)
    is at most Alg 1's rho^(m+1), for the TE and the TM block of a 2D grid
    (the spectrum of A on a block is [0, rho]: TE 2/3, TM the largest corner
    of its bilinear symbol)."""
    import math
    rx, ry = dt * dt / (d[0] * d[0]), dt * dt / (d[1] * d[1])
    rhos = (2 / 3, max(2 / 3 * (1 - rx), 2 / 3 * (1 - ry), 8 / 9 - 2 / 9 * (rx + ry)))
    need, bounds = 1, []
    for rho in rhos:
        x = (1 - rho / 2) / (rho / 2)
        k = 1
        while 1 / math.cosh(k * math.acosh(x)) > rho ** (m + 1):
            k += 1
        need = max(need, k)
        bounds.append(rho ** (m + 1))
    return need, rhos, bounds


def bench_chebyshev(steps, warm):
    """The Chebyshev solve against Alg 1: the 4096^2 FP32 TE+TM workload with
    a sweep count of equal worst-case solve error per block, and the 128^2
    FP64 TE plane wave to 1e-12."""
    import math
    import torch
    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    steps = steps or 200
    warm = 5 if warm is None else warm
    out = {}
    # (a) 4096^2 FP32, fixed counts
    n = 4096
    w = I.modes_2d((n, n), steps=steps + warm, dtype="f32")
    env = [float(x) for x in w.env]
    kc, rhos, bounds = _cheb_sweeps_matching_alg1(w.dt, (1.0, 1.0), w.sweeps)
    res = {}
    for name, solver, m in (("alg1", mx.SOLVER_ALG1, w.sweeps), ("chebyshev", mx.SOLVER_CHEBYSHEV, kc)):
        cfg = mx.make_config(2, (n, n), w.dt, (1.0, 1.0), "f32", mx.MX_ALL, m, 0.0, w.filter_passes, solver=solver)
        g = mx.Grid(cfg)
        E = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in w.E]
        B = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in w.B]
        J = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in w.J0]
        g.bind(E, B)
        g.set_current(J)
        g.step(warm, env[:warm])
        torch.cuda.synchronize()
        s0, s1 = _events()
        s0.record()
        g.step(steps, env[warm:warm + steps])
        s1.record()
        torch.cuda.synchronize()
        ms = s0.elapsed_time(s1)
        res[name] = {"sweeps": m, "sweeps_per_pass": list(g.block_sweeps_per_pass),
                     "Gcell_steps_per_s": round(n * n * steps / (ms / 1e3) / 1e9, 3),
                     "ms_per_step": round(ms / steps, 4)}
        g.close()
        del E, B, J
    res["solve_error_factor_bound"] = {"alg1_rho^(m+1)": [float(f"{b:.3g}") for b in bounds],
                                       "chebyshev_1/T_k": [float(f"{1 / math.cosh(kc * math.acosh((1 - r / 2) / (r / 2))):.3g}")
                                                           for r in rhos]}
    out["4096sq_f32_equal_worst_case_error"] = res
    # (b) 128^2 FP64 TE to 1e-12
    wt = I.planewave_te_2d(steps=steps + warm)
    res = {}
    for name, solver in (("alg1", mx.SOLVER_ALG1), ("chebyshev", mx.SOLVER_CHEBYSHEV)):
        cfg = mx.make_config(2, wt.shape[::-1], wt.dt, wt.d, "f64", wt.blocks, wt.sweeps, wt.tol, 0, solver=solver)
        g = mx.Grid(cfg)
        E = [torch.tensor(a, device="cuda") for a in wt.E]
        B = [torch.tensor(a, device="cuda") for a in wt.B]
        g.bind(E, B)
        g.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = g.step(steps, stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"mean_sweeps": round(sum(s.sweeps[0] for s in st) / steps, 2),
                     "us_per_step": round(dt / steps * 1e6, 1), "sweeps_per_pass": g.sweeps_per_pass}
        g.close()
    out["128sq_te_f64_tol1e-12"] = res
    a = out["4096sq_f32_equal_worst_case_error"]
    return _line("Chebyshev vs Alg 1 solve, 4096^2 FP32 at equal worst-case solve error", 
                 a["chebyshev"]["Gcell_steps_per_s"], "Gcell-steps/s", {"steps": steps, "results": out})


def bench_pic(steps, warm):
    """Coupled particle-field steps on a drifting pair plasma shaped like the
    paper's NCI test problem (Table 1): 256 x 128 cells, 256 particles per
    cell and species (16.8 M in all), drift Lorentz factor 1000, temperature
    0.01 m c^2, dt = 0.5 dt_CFL, linear shapes; field step m = 20 with a
    3-pass filter of the deposited current; FP32."""
    import math
    import torch
    from paper_1907_13088_amd import inputs as I
    from paper_1907_13088_amd import mx
    steps = steps or 200
    warm = 5 if warm is None else warm
    nx, ny = 256, 128
    t0 = time.time()
    sps = I.drifting_pair_plasma(n=(nx, ny), ppc=256, dtype="f32")
    log(f"plasma generated in {time.time() - t0:.1f}s")
    dt = 0.5 / math.sqrt(2.0)
    g = mx.Grid(mx.make_config(2, (nx, ny), dt, (1.0, 1.0), "f32", mx.MX_ALL, 20, 0.0, 3))
    E = [torch.zeros((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
    B = [torch.zeros((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
    J = [torch.zeros((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
    g.bind(E, B)
    g.set_current(J)
    parts = [([torch.tensor(sp.x, dtype=torch.float32, device="cuda"),
               torch.tensor(sp.y, dtype=torch.float32, device="cuda")],
              [torch.tensor(a, dtype=torch.float32, device="cuda") for a in sp.u]) for sp in sps]
    npart = sum(int(p[0][0].numel()) for p in parts)

    def one_step():
        for k, (sp, (pos, u)) in enumerate(zip(sps, parts)):
            g.pic_push(sp.q, sp.m, sp.w, pos, u, J, accumulate=k > 0)
        g.step(1, env=[1.0])

    for _ in range(warm):
        one_step()
    torch.cuda.synchronize()
    g.profile_enable(True)
    s0, s1 = _events()
    s0.record()
    for _ in range(steps):
        one_step()
    s1.record()
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1)
    prof = g.profile_read()
    g.close()
    pp = prof["particles"]
    field_ms = sum(v["ms"] for k, v in prof.items() if k != "particles")
    return _line("coupled particle-field step, drifting pair plasma 256x128, 16.8M particles, FP32",
                 npart * steps / (ms / 1e3) / 1e9, "Gparticle-steps/s",
                 {"steps": steps, "dtype": "f32", "particles": npart, "ms_per_step": round(ms / steps, 4),
                  "push_deposit_us_per_species": round(1e3 * pp["ms"] / max(pp["launches"], 1), 1),
                  "push_share_of_kernel_time": round(pp["ms"] / max(pp["ms"] + field_ms, 1e-9), 4),
                  "field_step_us": round(1e3 * field_ms / steps, 1),
                  "push_phase_space_GBps": round(pp["bytes"] / (pp["ms"] / 1e3) / 1e9, 1) if pp["ms"] else None,
                  "note": "kernel times from HIP events on every launch (profiling on)"})


OTHER_WORKLOADS = {"planewave_te": bench_planewave_te, "planewave_3d": bench_planewave_3d, "pic": bench_pic,
                   "batch": bench_batch, "adjoint": bench_adjoint, "chebyshev": bench_chebyshev,
                   "chebyshev_3d": bench_chebyshev_3d}


if __name__ == "__main__":
    main()
