#!/usr/bin/env python3
"""Throughput of the weighted adjoint NFFT on one MI355X.

Workload: polar grid with signed radius, R = T = 512 (N = 262144 nodes), d = 2,
M = 256, sigma = 2, Kaiser-Bessel m = 6, geometric area weights, one
right-hand side of complex samples per step. A step is one reconstruction
fhat = D^* F^* B^* W f (spreading, FFT, deconvolution and crop) with the plan,
the weights and the samples already resident in device memory.

Plans are made by the library's autotuner (plan-time work, outside the timed
region). Prints one JSON line: points/s of the float32 path (value), per-step
latency percentiles, the float64 path's figures, per-stage times with their
HBM rates from algorithmic bytes, the roofline position of the spreading
kernel (timed with HIP events on the library's stream inside the timed
region, on every PROFILE_EVERY-th step), the batched form (spiral, 131072 nodes, 32 right-hand sides, one
fused float32 call against 32 float64 calls) and the FP64 CPU oracle timed
on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nonuniform points/s for weighted adjoint NFFT (2D M=256, rel err<=1e-5); p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# stage events are recorded on every PROFILE_EVERY-th step of a timed region
PROFILE_EVERY = 32
R_POLAR = T_POLAR = 512
M, SIGMA, MW, D = 256, 2.0, 6, 2


def spread_algorithmic_bytes(N, Ms, d, prec):
    """Minimum HBM bytes of one spreading launch: per node the encoded
    position (d offsets + one packed cell word), the weight and the sample;
    plus the M_sigma^d grid of cell sums once."""
    rb = 8 if prec == "f64" else 4
    cb = 2 * rb
    per_node = d * rb + 4 + cb + cb
    return N * per_node + Ms ** d * cb


def spread_flops(N, m, d):
    """Two real multiply-adds per complex-by-real cell update, (2m)^d cells."""
    return 4 * (2 * m) ** d * N


def stage_bytes(N, Ms, Mb, d, prec, nrhs=1):
    """Algorithmic HBM bytes of each adjoint stage (the least each stage must
    move): spreading reads the encoded nodes, weights and samples and writes
    the M_sigma^d grid of cell sums once; the first FFT pass reads that grid
    (the tile partials hold it spread over padded tiles) and writes
    M_sigma^(d-1) M values after the crop of its dimension; the remaining
    passes read that and write the M^d result."""
    rb = 8 if prec == "f64" else 4
    cb = 2 * rb
    spread = N * (d * rb + 4 + cb) + nrhs * (N * cb + Ms ** d * cb)
    merge = nrhs * (Ms ** d + Ms ** (d - 1) * Mb) * cb
    rest = nrhs * (Ms ** (d - 1) * Mb + Mb ** d) * cb
    return {"spread": spread, "fft_merge": merge, "fft_rest_deconv": rest}


def run_gpu(prec, x, w, f, steps, warmup, tuning="auto"):
    import torch
    from paper_2302_00414_amd.nfft import Plan

    dev = torch.device("cuda:0")
    plan = Plan(x, M, SIGMA, MW, precision=prec, device=dev, tuning=tuning)
    plan.set_weights(w)
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    fd = torch.from_numpy(f).to(device=dev, dtype=cdt)
    out = torch.empty(M ** D, dtype=cdt, device=dev)
    for _ in range(warmup):
        plan.adjoint(fd, out=out)
    torch.cuda.synchronize()

    # one untimed profiled pass fills the library's event pool, so the timed
    # region records stage events without creating any
    plan.set_profiling(True)
    for _ in range(steps // PROFILE_EVERY + 1):
        plan.adjoint(fd, out=out)
    torch.cuda.synchronize()
    plan.stage_times(reset=True)

    # timed region: K back-to-back steps; the library records its stage events
    # (HIP events on its stream around every kernel) on every PROFILE_EVERY-th
    # step, so that the events cost little of the measured throughput
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(steps):
        plan.set_profiling(i % PROFILE_EVERY == 0)
        plan.adjoint(fd, out=out)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    plan.set_profiling(False)
    stages = plan.stage_times(reset=True)

    # per-request latency: one call at a time, synchronised
    lat = []
    for _ in range(min(steps, 300)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.adjoint(fd, out=out)
        b.record()
        b.synchronize()
        lat.append(a.elapsed_time(b))
    # cold caches: a 512 MiB write (twice the Infinity Cache) before each
    # call evicts the plan's arrays, the weights and the samples from the
    # caches; only the call itself is between the events
    flush = torch.empty(128 << 20, dtype=torch.float32, device=dev)
    lat_cold = []
    for i in range(min(steps, 100)):
        flush.fill_(float(i))
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.adjoint(fd, out=out)
        b.record()
        b.synchronize()
        lat_cold.append(a.elapsed_time(b))
    del flush
    res = out.cpu().numpy().astype(np.complex128)
    info = plan.info()
    tuning = plan.tuning()
    plan.close()
    ms_per_step = max(gpu_ms, wall * 1e3) / steps
    return dict(ms_per_step=ms_per_step, gpu_ms=gpu_ms, wall_s=wall, stages=stages,
                lat=np.array(lat), lat_cold=np.array(lat_cold), out=res, info=info, tuning=tuning)


def run_forward(prec, x, steps, tuning="auto"):
    """Forward NFFT f = B F D fhat (Algorithm 2.1) on the same plan shape:
    milliseconds per call and per stage."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan

    cdt = torch.complex64 if prec == "f32" else torch.complex128
    plan = Plan(x, M, SIGMA, MW, precision=prec, tuning=tuning)
    fh = torch.from_numpy(wl.complex_normal(M ** D, 7)).to("cuda", cdt)
    out = torch.empty(x.shape[0], dtype=cdt, device="cuda")
    for _ in range(5):
        plan.forward(fh, out=out)
    plan.set_profiling(True)
    for _ in range(steps // PROFILE_EVERY + 1):
        plan.forward(fh, out=out)
    torch.cuda.synchronize()
    plan.stage_times(reset=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        plan.set_profiling(i % PROFILE_EVERY == 0)
        plan.forward(fh, out=out)
    e1.record()
    torch.cuda.synchronize()
    plan.set_profiling(False)
    st = plan.stage_times(reset=True)
    plan.close()
    ms = e0.elapsed_time(e1) / steps
    return dict(ms_per_call=ms, points_per_s=x.shape[0] / (ms / 1e3),
                stage_us={k: round(v[0] / max(v[1], 1) * 1e3, 3) for k, v in st.items() if v[1]})


def run_weights():
    """Algorithm 3.6 on the GPU (float64 CG with the library NFFT at 2M):
    d = 2, M = 32, N = 16384 uniform nodes (the setting of Example 5.2,
    |I_2M| = 4096 < N, branch (3.15))."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import compute_weights

    x = wl.uniform_nodes(16384, 2, 11)
    compute_weights(x, 32, 2.0, 8)  # warm-up (plan kernels, first launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, info = compute_weights(x, 32, 2.0, 8)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(workload="d=2, M=32, N=16384 uniform (Example 5.2 setting), m=8, tol 1e-13",
                seconds=dt, **info)


def run_bopt(steps):
    """Optimized sparse matrix (Algorithms 4.3 / 4.4): jittered 384 x 384 grid
    (N = 147456), d = 2, M = 256, sigma = 2, m = 4, float32 plan. Times the
    float64 device precompute of B_opt and the reconstruction D^* F^* B_opt^* f."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan

    x = wl.jittered_nodes((384, 384), 12)
    N = x.shape[0]
    plan = Plan(x, M, SIGMA, 4, precision="f32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = plan.build_bopt(x)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    f = torch.from_numpy(wl.complex_normal(N, 13)).to("cuda", torch.complex64)
    out = torch.empty(M * M, dtype=torch.complex64, device="cuda")
    for _ in range(5):
        plan.bopt_adjoint(f, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.bopt_adjoint(f, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.close()
    return dict(workload="jittered 384x384 (N=147456), d=2, M=256, sigma=2, m=4, float32",
                build_s=t_build, ms_per_reconstruction=ms, points_per_s=N / (ms / 1e3), **info)


def run_refine(steps, iters=4, tuning="auto"):
    """Weighted iterative refinement (nfft_refine) on the polar workload of
    the headline (512 x 512 nodes, M = 256, m = 6, area weights, float32):
    milliseconds per call of `iters` steps (each one forward, which forms the
    residual, and one weighted adjoint, which adds the correction; autotuned
    plan unless a tuning is given) and the relative residuals per step, for samples of a random trigonometric polynomial of degree M (made with the
    plan's forward transform)."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan

    x = wl.polar_nodes(512, 512)
    N = x.shape[0]
    plan = Plan(x, M, SIGMA, 6, precision="f32", tuning=tuning)
    plan.set_weights(wl.polar_area_weights(512, 512).astype(np.complex128))
    fh = torch.from_numpy(wl.complex_normal(M * M, 14)).to("cuda", torch.complex64)
    f = plan.forward(fh)
    out = torch.empty(M * M, dtype=torch.complex64, device="cuda")
    _, res = plan.refine(f, iters, out=out, residuals=True)
    for _ in range(3):
        plan.refine(f, iters, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.refine(f, iters, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.close()
    return dict(workload=f"polar 512x512 (N=262144), d=2, M=256, m=6, area weights, float32, "
                         f"{iters} refinement steps, samples of a random polynomial",
                ms_per_call=ms, ms_per_step=ms / iters, relative_residuals=[float(r) for r in res])


def run_bandlimited():
    """Example 5.5: the triangular pulse b = 24 sampled on a jittered 144 x 144
    grid, M = 64; largest pointwise error of the reconstructed fhat(k) for the
    weights of Algorithm 3.6, the optimized sparse matrix (sigma = 2, m = 4),
    the PCF weights (3.62) and an equispaced 144 x 144 grid (float64)."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan, compute_weights

    Mb, b, n = 64, 24, 144
    fh = wl.triangle_pulse_coefficients(Mb, 2, b)

    def rec(x, w):
        p = Plan(x, Mb, 2.0, 6, precision="f64")
        p.set_weights(w)
        h = p.adjoint(torch.from_numpy(wl.triangle_pulse_samples(x, b)).cuda()).cpu().numpy()
        p.close()
        return float(np.max(np.abs(h - fh)))

    xe = wl.equispaced_nodes(n, 2)
    out = {"equispaced": rec(xe, np.full(xe.shape[0], 1.0 / xe.shape[0], dtype=np.complex128))}
    x = wl.jittered_nodes((n, n), 5, jitter=1.0)
    t0 = time.perf_counter()
    w, _ = compute_weights(x, Mb, 2.0, 8, 1e-13, 2000)
    torch.cuda.synchronize()
    out["alg3.6_weights_s"] = time.perf_counter() - t0
    out["alg3.6"] = rec(x, w.cpu().numpy())
    wp, _ = compute_weights(x, Mb, 2.0, 8, scheme="pcf")
    out["pcf"] = rec(x, wp.cpu().numpy())
    p = Plan(x, Mb, 2.0, 4, precision="f64")
    p.build_bopt(x)
    h = p.bopt_adjoint(torch.from_numpy(wl.triangle_pulse_samples(x, b)).cuda()).cpu().numpy()
    p.close()
    out["bopt"] = float(np.max(np.abs(h - fh)))
    return dict(workload="Example 5.5: triangular pulse b=24, jittered 144x144, M=64, "
                         "max |fhat_rec(k) - fhat(k)|", **out)


def run_jittered3d(steps, precs=("f32", "f64"), tuning="auto"):
    """Jittered 128 x 64 x 64 grid (N = 524288), d = 3, M = 64, sigma = 2,
    m = 4, weights 1/N: the weighted adjoint in float32 and float64 on
    autotuned plans, milliseconds per call (plain events) and per stage
    (stage events on a separate loop)."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan

    M3, m3 = 64, 4
    x = wl.jittered_nodes((128, 64, 64), 4)
    N = x.shape[0]
    w = np.full(N, 1.0 / N)
    f = wl.complex_normal(N, 8)
    res = {}
    for prec in precs:
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        plan = Plan(x, M3, SIGMA, m3, precision=prec, tuning=tuning)
        plan.set_weights(w)
        fd = torch.from_numpy(f).to("cuda", cdt)
        out = torch.empty(M3 ** 3, dtype=cdt, device="cuda")
        for _ in range(5):
            plan.adjoint(fd, out=out)
        plan.set_profiling(True)
        for _ in range(max(5, steps // 4)):
            plan.adjoint(fd, out=out)
        torch.cuda.synchronize()
        st = plan.stage_times(reset=True)
        plan.set_profiling(False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.adjoint(fd, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[prec] = dict(ms_per_step=ms, points_per_s=N / (ms / 1e3), tuning=plan.tuning(),
                         stage_us={k: round(v[0] / max(v[1], 1) * 1e3, 3)
                                   for k, v in st.items() if v[1]})
        plan.close()
    return dict(workload="jittered 128x64x64 (N=524288), d=3, M=64, sigma=2, m=4, w=1/N", **res)


# Table 5.1 of the paper (linogram R = 2M, T = 2R, Shepp-Logan phantom,
# hardware not stated): Alg. 3.7 precomputation [s], reconstruction [s], e_2
PAPER_TABLE_5_1 = {64: (3.4324, 5.0420e-03, 2.5859e-14), 128: (9.4725, 2.9860e-02, 7.9006e-14),
                   256: (38.365, 6.6443e-02, 2.6386e-13), 512: (140.20, 2.1674e-01, 1.0917e-12),
                   1024: (721.53, 7.4896e-01, 4.2563e-12)}


def run_table51(steps, Ms=(64, 128, 256, 512, 1024)):
    """The setting of Table 5.1: linogram grids R = 2M, T = 2R (N = 8M^2),
    weights of Algorithm 3.6 on the GPU (float64, NFFT window m = 8) timed
    as the precomputation, the weighted adjoint of Algorithm 3.7 timed as the
    reconstruction (float64 with m = 8, and float32 with m = 6), and e_2 of
    (5.6) for random coefficients (the phantom is not available) whose
    samples the float64 forward transform makes."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan, compute_weights

    rows = {}
    for Mt in Ms:
        x = wl.linogram_nodes(2 * Mt, 4 * Mt)
        N = x.shape[0]
        fh = torch.from_numpy(wl.complex_normal(Mt * Mt, 160)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, info = compute_weights(x, Mt, 2.0, 8)
        torch.cuda.synchronize()
        t_pre = time.perf_counter() - t0
        row = dict(N=N, precompute_s=t_pre, cg_iterations=info["iterations"])
        for prec, m in (("f64", 8), ("f32", 6)):
            cdt = torch.complex64 if prec == "f32" else torch.complex128
            p = Plan(x, Mt, 2.0, m, precision=prec)
            p.set_weights(w)
            if prec == "f64":
                f = p.forward(fh)
            fd = f.to(cdt)
            out = torch.empty(Mt * Mt, dtype=cdt, device="cuda")
            for _ in range(5):
                p.adjoint(fd, out=out)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                p.adjoint(fd, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            e2 = float(torch.linalg.norm(out.to(torch.complex128) - fh) / torch.linalg.norm(fh))
            row[prec] = dict(reconstruction_ms=ms, points_per_s=N / (ms / 1e3), e2=e2, m=m)
            p.close()
        if Mt in PAPER_TABLE_5_1:
            pre, rec, e2p = PAPER_TABLE_5_1[Mt]
            row["paper"] = dict(precompute_s=pre, reconstruction_s=rec, e2=e2p,
                                note="Shepp-Logan phantom, hardware not stated")
        rows[str(Mt)] = row
    # Example 5.4's second setting, R = M, T = 2R (N = 2M^2 < |I_2M|): the
    # weights are not exact there; Algorithm 4.4 and the refinement compared
    Mr = 64
    x = wl.linogram_nodes(Mr, 2 * Mr)
    fh = torch.from_numpy(wl.complex_normal(Mr * Mr, 170)).cuda()
    p = Plan(x, Mr, 2.0, 8, precision="f64")
    f = p.forward(fh)
    w, _ = compute_weights(x, Mr, 2.0, 8)
    p.set_weights(w)
    err = lambda h: float(torch.linalg.norm(h - fh) / torch.linalg.norm(fh))
    r_m = dict(N=x.shape[0], alg3_7=err(p.adjoint(f)), alg3_7_refined_20=err(p.refine(f, 20)))
    p.close()
    q = Plan(x, Mr, 2.0, 4, precision="f64")
    q.build_bopt(x)
    r_m["alg4_4_sigma2_m4"] = err(q.bopt_adjoint(f))
    q.close()
    r_m["paper_M1024_phantom"] = dict(alg3_7=0.50585, alg4_4=2.2737e-3, voronoi=0.5304)
    return dict(workload="linogram R=2M, T=2R (N=8M^2), d=2, sigma=2, Alg. 3.6 weights, "
                         "random coefficients", **rows, R_equals_M_64=r_m)


def run_batched(steps, precs=("f32", "f64"), tuning="auto"):
    """Spiral trajectory, N = 131072, 32 right-hand sides, M = 256, m = 6: one
    fused float32 adjoint of all 32 against 32 float64 single calls."""
    import torch
    from paper_2302_00414_amd import workloads as wl
    from paper_2302_00414_amd.nfft import Plan

    N, R = 131072, 32
    x = wl.spiral_nodes(N, M)
    w = wl.spiral_area_weights(N, M)
    F = wl.complex_normal((R, N), 5)
    res = {}
    for prec, nrhs in (("f32", R), ("f64", 1)):
        if prec not in precs:
            continue
        cdt = torch.complex64 if prec == "f32" else torch.complex128
        plan = Plan(x, M, SIGMA, MW, precision=prec, max_rhs=nrhs, tuning=tuning)
        plan.set_weights(w)
        fd = torch.from_numpy(F).to("cuda", cdt)
        out = torch.empty((nrhs, M * M), dtype=cdt, device="cuda")
        calls = (lambda: plan.adjoint(fd, out=out)) if nrhs == R else \
                (lambda: [plan.adjoint(fd[r:r + 1], out=out) for r in range(R)])
        for _ in range(3):
            calls()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            calls()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[prec] = dict(ms_per_32_rhs=ms, points_per_s=N * R / (ms / 1e3), tuning=plan.tuning())
        plan.close()
    if len(res) < 2:
        return dict(workload="spiral N=131072, d=2, M=256, sigma=2, m=6, 32 rhs, area weights", **res)
    return dict(workload="spiral N=131072, d=2, M=256, sigma=2, m=6, 32 rhs, area weights",
                f32_fused=res["f32"], f64_separate_calls=res["f64"],
                speedup=res["f64"]["ms_per_32_rhs"] / res["f32"]["ms_per_32_rhs"])


def cpu_baseline(x, w, f, gpu_out32, gpu_out64, budget_s=12.0):
    """The FP64 oracle on the host: the step-by-step NFFT (O2) on the whole
    workload, repeated up to the time budget; the exact sums (O1) at sampled
    frequencies for the accuracy of the GPU results."""
    from oracle import ndft, nfft as onfft, metrics
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    c = w * f
    reps, t0 = 0, time.perf_counter()
    while True:
        ref = onfft.adjoint(x, c, M, SIGMA, MW)
        reps += 1
        if time.perf_counter() - t0 > budget_s or reps >= 20:
            break
    dt = (time.perf_counter() - t0) / reps
    # the same oracle on one thread (BLAS and FFT pools limited to one)
    dt1 = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t2 = time.perf_counter()
            onfft.adjoint(x, c, M, SIGMA, MW)
            dt1 = time.perf_counter() - t2
    except Exception:
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    K = ndft.index_set(M, D)
    rng = np.random.default_rng(17)
    sel = np.unique(np.concatenate([rng.choice(K.shape[0], 256, replace=False), [0, K.shape[0] - 1]]))
    t1 = time.perf_counter()
    exact = ndft.adjoint_at(x, c, K[sel])
    t_exact = time.perf_counter() - t1
    return dict(
        baseline=dict(value=x.shape[0] / dt, unit="points/s", cores=int(cores), kind="oracle",
                      sample=f"step-by-step FP64 NFFT oracle on the full polar 512x512 workload, "
                             f"{reps} run(s), {dt:.2f} s each; exact sums at {len(sel)} sampled "
                             f"frequencies took {t_exact:.2f} s",
                      cpu_model=model, nproc=os.cpu_count(),
                      single_thread_points_per_s=(x.shape[0] / dt1) if dt1 else None),
        err32_vs_exact=metrics.rel_err(gpu_out32[sel], exact),
        err64_vs_exact=metrics.rel_err(gpu_out64[sel], exact),
        err32_vs_nfft_oracle=metrics.rel_err(gpu_out32, ref),
        err64_vs_nfft_oracle=metrics.rel_err(gpu_out64, ref),
    )


def traffic_record(kernel):
    """HBM bytes per launch from committed counter summaries, if they were taken
    on this kernel and the current kernel source (sha256 of the spreading
    sources recorded with them)."""
    path = os.path.join(ROOT, "profiles", "spread_traffic_polar512.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != spread_source_sha() or rec.get("kernel", "").replace(" ", "") \
            != ("nfft::" + kernel).replace(" ", ""):
        return None
    return rec.get("bytes_per_launch")


# sources of the d = 2 single-rhs spreading kernels
SPREAD_SOURCES = ("spread.hip", "spread_common.hpp", "spread_group.hpp", "spread_pre.hip", "spread_late.hip",
                  "spread_rows.hip")


def spread_kernel_name(t):
    """Name of the spreading kernel the library launches for this tuning
    (d = 2, m = 6, float32, one right-hand side), as the profiler prints it."""
    T, mode = t["tile_edge"], t["spread_mode"]
    if mode == 2 and T + 2 * MW <= 32:
        return f"spread_rows_kernel<float, {MW}, {T if T == 16 else 0}, 1>"
    ws = {3: 1, 4: 2}.get(mode, 0)   # window source of the group kernel
    return (f"spread_group_kernel<float, 2, {MW}, {t['spread_threads']}, "
            f"{T if T in (8, 16) else 0}, {'true' if t['spread_planes'] == 2 else 'false'}, {ws}>")


def spread_source_sha():
    h = hashlib.sha256()
    for name in SPREAD_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2302_00414_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-rhs spiral figures")
    ap.add_argument("--tuning", default="auto",
                    help='profiling runs: "auto" (autotuner) or a JSON object of tuning keys')
    ap.add_argument("--precision", choices=["both", "f32", "f64"], default="both",
                    help="profiling runs: time one path only (the JSON line needs both)")
    ap.add_argument("--only", choices=["jittered3d", "batched", "forward", "refine", "table51"],
                    default=None,
                    help="profiling runs: run one secondary workload alone and print its JSON")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="profiling runs: also launch one device-to-device copy of this size, "
                         "a known-size reference for the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the reconstruction of one request runs on one "
              "device and the library has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_00414_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    x = wl.polar_nodes(R_POLAR, T_POLAR)
    w = wl.polar_area_weights(R_POLAR, T_POLAR)
    f = wl.complex_normal(x.shape[0], 3)
    N = x.shape[0]
    Ms = 2 * M

    if args.only:
        # one secondary workload, for profiling: --precision picks the path,
        # --tuning a fixed tuning (so that no autotuner runs are traced)
        k = max(10, args.steps // 5)
        precs = ("f32", "f64") if args.precision == "both" else (args.precision,)
        tun = "auto" if args.tuning == "auto" else json.loads(args.tuning)
        sec = {"jittered3d": lambda: run_jittered3d(k, precs, tun),
               "batched": lambda: run_batched(k, precs, tun),
               "forward": lambda: {p: run_forward(p, x, k, tun) for p in precs},
               "refine": lambda: run_refine(max(10, args.steps // 20), tuning=tun),
               "table51": lambda: run_table51(max(10, args.steps // 20))}[args.only]()
        print(json.dumps({args.only: sec}), flush=True)
        return

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration copy: {n * 4} bytes read, {n * 4} bytes written", file=sys.stderr)
    tuning = args.tuning if args.tuning == "auto" else json.loads(args.tuning)
    if args.precision != "both":
        r = run_gpu(args.precision, x, w, f, args.steps, args.warmup, tuning)
        print(json.dumps({"precision": args.precision, "ms_per_step": r["ms_per_step"],
                          "tuning": r["tuning"],
                          "points_per_s": N / (r["ms_per_step"] / 1e3),
                          "stage_us": {k: v[0] / max(v[1], 1) * 1e3 for k, v in r["stages"].items()
                                       if v[1]}}), flush=True)
        return
    r32 = run_gpu("f32", x, w, f, args.steps, args.warmup, tuning)
    r64 = run_gpu("f64", x, w, f, args.steps, args.warmup, tuning)

    sp_ms, sp_calls = r32["stages"]["spread"]
    sp_avg_s = sp_ms / max(sp_calls, 1) / 1e3
    alg = spread_algorithmic_bytes(N, Ms, D, "f32")
    flops = spread_flops(N, MW, D)
    achieved = flops / sp_avg_s / 1e12
    t = r32["tuning"]
    kname = spread_kernel_name(t)
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=FP32_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / FP32_PEAK_TFLOPS, 5),
                    traffic=traffic_record(kname),
                    kernel=kname,
                    avg_launch_us=round(sp_avg_s * 1e6, 3),
                    algorithmic_flops_per_launch=flops,
                    algorithmic_bytes_per_launch=alg,
                    hbm_view_gbs=round(alg / sp_avg_s / 1e9, 2),
                    hbm_view_frac=round(alg / sp_avg_s / 1e9 / HBM_PEAK_GBS, 5),
                    cell_updates_per_s=(2 * MW) ** D * N / sp_avg_s)
    if roofline["traffic"]:
        # the counters' HBM bytes per launch over the same launch time
        roofline["traffic_gbs"] = round(roofline["traffic"] / sp_avg_s / 1e9, 1)
        roofline["traffic_frac_of_hbm"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
    stage_us = {k: round(v[0] / max(v[1], 1) * 1e3, 3) for k, v in r32["stages"].items() if v[1]}
    stage_us64 = {k: round(v[0] / max(v[1], 1) * 1e3, 3) for k, v in r64["stages"].items() if v[1]}

    def hbm(stage_times, prec):
        b = stage_bytes(N, Ms, M, D, prec)
        return {k: dict(alg_bytes=b[k], gbs=round(b[k] / (stage_times[k] * 1e-6) / 1e9, 1),
                        frac=round(b[k] / (stage_times[k] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
                for k in b if k in stage_times}

    line = {
        "metric": METRIC,
        "value": N / (r32["ms_per_step"] / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "polar R=T=512 (N=262144), d=2, M=256, sigma=2, KB m=6, "
                               "area weights, 1 rhs complex64, weighted adjoint NFFT",
                   "global_batch": 1, "nodes": N, "M": M, "sigma": SIGMA, "m": MW},
        "latency_ms": {"p50": float(np.percentile(r32["lat"], 50)),
                       "p99": float(np.percentile(r32["lat"], 99))},
        "cold_latency_ms": {"p50": float(np.percentile(r32["lat_cold"], 50)),
                            "p99": float(np.percentile(r32["lat_cold"], 99)),
                            "flush": "512 MiB device write before each call"},
        "stage_us": stage_us,
        "stage_events": f"HIP events on the library stream, every {PROFILE_EVERY}th timed step",
        "stage_hbm": hbm(stage_us, "f32"),
        "tuning": r32["tuning"],
        "f64": {"value": N / (r64["ms_per_step"] / 1e3), "ms_per_step": r64["ms_per_step"],
                "latency_ms": {"p50": float(np.percentile(r64["lat"], 50)),
                               "p99": float(np.percentile(r64["lat"], 99))},
                "cold_latency_ms": {"p50": float(np.percentile(r64["lat_cold"], 50)),
                                    "p99": float(np.percentile(r64["lat_cold"], 99))},
                "stage_us": stage_us64, "stage_hbm": hbm(stage_us64, "f64"),
                "tuning": r64["tuning"]},
        "roofline": roofline,
        "plan": r32["info"],
        "paper_context": "Table 5.1, M=256 linogram N=524288: 6.6443e-02 s per reconstruction "
                         "(7.89e6 points/s), hardware not stated",
    }
    if not args.no_batched:
        line["batched"] = run_batched(max(10, min(args.steps // 10, 100)))
        line["forward"] = {"f32": run_forward("f32", x, max(10, args.steps // 5)),
                           "f64": run_forward("f64", x, max(10, args.steps // 5))}
        line["weights_gpu"] = run_weights()
        line["bopt"] = run_bopt(max(10, args.steps // 5))
        line["jittered3d"] = run_jittered3d(max(10, args.steps // 10))
        line["table51"] = run_table51(max(10, args.steps // 20))
        line["refine"] = run_refine(max(10, args.steps // 20))
        line["bandlimited"] = run_bandlimited()
    if not args.no_cpu_baseline:
        cb = cpu_baseline(x, w, f, r32["out"], r64["out"])
        line["cpu_baseline"] = cb["baseline"]
        line["rel_err"] = {"f32_vs_exact_sampled": cb["err32_vs_exact"],
                           "f64_vs_exact_sampled": cb["err64_vs_exact"],
                           "f32_vs_nfft_oracle": cb["err32_vs_nfft_oracle"],
                           "f64_vs_nfft_oracle": cb["err64_vs_nfft_oracle"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
