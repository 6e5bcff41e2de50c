#!/usr/bin/env python3
"""Benchmark: Hessian-free ray-Born frequency-step updates per second on one MI355X.

Workload (default): ring of 1024 transducers (R = 110 mm), 1024^2 grid at 0.22 mm, breast-like
phantom with 10 lesions, 1024 rays per transducer, frequencies 0.1-1.2 MHz (32, one per
step, low to high). A step is one pass of the whole hot path for one frequency: smoothing,
ray tracing + binning, Green's-function assembly, Born forward term, residual, Hessian-free
back-projection and model update (rb_frequency_step). Inputs are resident on the GPU before
the timed region; the synthetic data are made once, untimed, by the same library (ray-Born
prediction of the phantom plus 1 % complex Gaussian noise).

Prints one JSON line. Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hashlib
import re

FP32_MFMA_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix
HBM_PEAK_GBS = 8000.0
# FP32 vector arithmetic without packed FP32 instructions (the library is built without
# them): 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic units of the hot kernels
TRACE_FLOP_PER_SAMPLE = 550     # two spline value+gradient+Hessian evaluations, Heun, paraxial
TABLE_BYTES = {"f32": 21,       # one table entry: T 8, A 4, (u_x, u_y) 8, flags 1
               "bf16": 16, "f16": 16, "f16x": 16}   # compact record: dT, A, theta, flags
SAMPLE_BYTES = 24               # one ray sample: position 8, (dT, L, t_x, t_y) 16 (K only in folds)
# operand bytes written per (e, p): G (complex) + H, H_x, H_y; split form: G + H, b, a (FP16)
# + their low parts (FP8)
OPERAND_BYTES = {"f32": 32, "bf16": 16, "f16": 16, "f16x": 22}

CSRC = os.path.join(ROOT, "paper_2211_00316_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")

# stage -> kernels it launches (FP32 form, 16-bit forms)
PREC_CODES = {"f32": 1, "bf16": 2, "f16": 3, "f16x": 4}

STAGE_KERNELS = {
    "trace": (["trace_kernel"], ["trace_kernel"]),
    "resolve": (["tile_offset_kernel", "locate_kernel"], ["tile_offset_kernel", "locate_kernel"]),
    "build_green": (["green_kernel"], ["green_lp_rec_kernel"]),
    "forward_gemm": (["forward_kernel"], ["forward_pipe_kernel"]),
    "backproject_gemm": (["rowred_kernel"], ["rowred_lp_kernel"]),
}


def synthesize_data(ctx, w, grid, ring, tp, c_true, freq_idx, alpha0=None, y=1.4):
    """Measured data of the listed frequencies, made on the GPU by the library itself:
    ray-Born prediction of the phantom (window of that frequency) plus 1 % noise. alpha0
    (float64 [ny][nx], Np (rad/s)^-y m^-1): the absorbing, dispersive phantom (rays of each
    frequency on its map, A_abs, complex scattering potential)."""
    import numpy as np
    import torch

    import phantoms as ph
    from paper_2211_00316_amd import _lib

    N = w.n_trans
    c_t = torch.as_tensor(c_true, device="cuda:0")
    out = torch.empty(len(freq_idx), N, N, dtype=torch.complex64, device="cuda:0")
    zero = torch.zeros(N, N, dtype=torch.complex64, device="cuda:0")
    mask = _mask_index(w)
    a_t = None if alpha0 is None else torch.as_tensor(alpha0, device="cuda:0")
    for s, k in enumerate(freq_idx):
        om = 2 * math.pi * w.freqs[k]
        ns = ctx.refractive_index(grid, c_t, 1500.0, w.smooth_window(k))
        if a_t is None:
            tb = ctx.trace_rays(grid, ring, tp, ns)
        else:
            n_w, a_w = ctx.lossy_maps(grid, c_t, a_t, y, 1500.0, om, w.smooth_window(k))
            tb = ctx.trace_rays_lossy(grid, ring, tp, n_w, a_w)
            del n_w, a_w
        gr = ctx.build_green(tb, om, 1500.0)
        cm = c_t.reshape(-1)[mask]
        delta = (1.0 / cm ** 2 - (ns.reshape(-1)[mask].double() / 1500.0) ** 2).float()
        wv = torch.full((mask.numel(),), om * om * w.dx * w.dx, dtype=torch.complex64,
                        device="cuda:0")
        if a_t is not None:
            # scattering potential omega c k~ = omega^2 [1 + omega^(y-1) c alpha0 (tan + i)]
            t = om ** (y - 1.0) * cm * a_t.reshape(-1)[mask]
            wv = wv * (1.0 + t * math.tan(0.5 * math.pi * y) + 1j * t).to(torch.complex64)
        d = ctx.born_forward(gr, wv, delta)
        clean = ctx.residual(tb, om, 1500.0, zero, d)     # g_ray + Born term - 0
        keep = (clean != 0)
        rms = torch.sqrt(torch.mean(torch.abs(clean[keep]) ** 2)).item()
        noise = torch.as_tensor(ph.complex_noise((N, N), w.noise_seed + k).astype(np.complex64),
                                device="cuda:0")
        out[s] = clean + 0.01 * rms * noise
        del tb, gr, d, ns
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def _mask_index(w):
    import numpy as np
    import torch

    xs = w.x0 + w.dx * np.arange(w.nx)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    idx = np.flatnonzero((X * X + Y * Y <= w.mask_radius ** 2).ravel())
    return torch.as_tensor(idx, device="cuda:0")


def cpu_baseline(w):
    """The FP64 oracle timed on the host on a bounded sample of the same workload: trace +
    binning + receiver tables of a sample of transducers in a process pool over the host
    cores (two per worker, scaled by N), their Green's functions, and the Born forward /
    back-projection products on a block of mask columns on the BLAS threads (scaled by
    P_m / block); extrapolated to one frequency step."""
    import numpy as np

    import phantoms as ph
    from oracle import born, green, step as ostep
    from oracle.medium import Grid, Ring

    grid = Grid(w.nx, w.ny, w.dx, w.x0, w.y0, w.mask_radius)
    st = ostep.StepSetup(grid, Ring(w.n_trans, w.radius), w.n_rays, w.ds, w.max_steps())
    c = ph.phantom_for(w)
    N = w.n_trans
    Pm = grid.mask_index().size
    om = 2 * math.pi * w.freqs[0]
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    ns_sample = 2 * workers
    t0 = time.perf_counter()
    sample = [k * N // ns_sample for k in range(ns_sample)]
    tb, ns = ostep.tables_for(c, st, w.smooth_window(0), emitters=sample, workers=workers)
    t_tab = time.perf_counter() - t0
    t0 = time.perf_counter()
    green.build_green(tb, om)
    t_green = time.perf_counter() - t0
    block = 32768
    rng = np.random.default_rng(0)
    G = rng.standard_normal((N, block)) + 1j * rng.standard_normal((N, block))
    H = [rng.standard_normal((N, block)) + 1j * rng.standard_normal((N, block)) for _ in range(3)]
    R = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    t0 = time.perf_counter()
    born.forward(G, np.ones(block), rng.standard_normal(block))
    born.backproject(R, H[0], H[1], H[2], np.ones(block))
    t_gemm = time.perf_counter() - t0
    t_step = (t_tab + t_green) * N / len(sample) + t_gemm * Pm / block
    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    return {
        "value": 1.0 / t_step,
        "unit": "frequency-step updates/s",
        "cores": max(threads, workers),
        "kind": "oracle",
        "sample": (f"FP64 oracle: trace+bin+receivers of {len(sample)} of {N} transducers "
                   f"in {workers} processes and their Green's functions "
                   f"({t_tab + t_green:.1f} s, x{N / len(sample):.0f}) plus Born forward and "
                   f"back-projection on {block} of {Pm} mask columns on {threads} BLAS "
                   f"threads ({t_gemm:.1f} s, x{Pm / block:.1f}); extrapolated step "
                   f"{t_step:.0f} s"),
    }


PEAKS = {"f32": (FP32_MFMA_PEAK_TFLOPS, "fp32 MFMA"), "bf16": (2500.0, "bf16 MFMA dense"),
         "f16": (2500.0, "fp16 MFMA dense"), "f16x": (2500.0, "fp16 MFMA dense")}


def _pad(x, m):
    return (x + m - 1) // m * m


def contraction_flops(stage, N, Pm, prec):
    """(issued, own, dense) flop of one launch of a contraction. issued: what the kernel's
    tiles compute (the MFMA instructions it issues; in the split form the FP8 product counts
    half, its MFMA rate being twice the FP16 one); own: the symmetric products' unique
    entries, 8 flop per complex multiply-add over N (N + 1) / 2 pairs; dense: the plain
    complex GEMM count (8 N^2 P_m for the forward, three of them for the back-projection)."""
    own_pairs = N * (N + 1) // 2
    if stage == "forward_gemm":
        if prec == "f32":   # 128 x 128 upper tiles over K = P_m
            nT = _pad(N, 128) // 128
            issued = 8.0 * nT * (nT + 1) // 2 * 128 * 128 * Pm
        else:               # 256 x 128 upper tiles over K = P_m padded to 32
            nT = _pad(N, 128) // 128
            tiles = sum(nT - 2 * tm for tm in range((nT + 1) // 2))
            issued = 8.0 * tiles * 256 * 128 * _pad(Pm, 32)
        return issued, 8.0 * own_pairs * Pm, 8.0 * N * N * Pm
    # back-projection: row slabs of 256, K over the transducers (block upper triangle of R, or
    # the whole symmetric R in the split form), node tiles of 128 (64 in FP32)
    Np = _pad(N, 32)
    mb = _pad(N, 256) // 256
    cols = _pad(Pm, 64 if prec == "f32" else 128)
    tri = sum(256 * (Np - 256 * i) for i in range(mb))   # K values of the block triangle
    if prec == "f16x":
        # two FP16 products over all of Rs (H; b) and one FP8 product (b's low part, K rows
        # padded to 64)
        issued = 16.0 * mb * 256 * Np * cols + 0.5 * 8.0 * mb * 256 * _pad(N, 64) * cols
    elif prec == "f32":
        issued = 24.0 * tri * cols   # H, H u_x, H u_y over the block triangle
    else:
        # H over the block triangle, the bilinear form a^T Rs b over all of Rs
        issued = 8.0 * tri * cols + 8.0 * mb * 256 * Np * cols
    return issued, 24.0 * own_pairs * Pm, 24.0 * N * N * Pm


def start_model(w, start, c_true):
    """Model the timed steps start from: water (the first steps of the frequency
    continuation) or the true phantom (a late stage, with folded fans)."""
    import torch

    if start == "truth":
        return torch.as_tensor(c_true, dtype=torch.float64, device="cuda:0")
    return torch.full((w.ny, w.nx), 1500.0, dtype=torch.float64, device="cuda:0")


def run_form(ctx, w, grid, ring, tp, data, prec, steps, warmup, tag, c_start, alpha0=None,
             y=1.4, first=0):
    """Time `steps` frequency steps of one form from c_start (after `warmup`), at the
    frequencies first + warmup ... (data[k - first] is frequency k's); alpha0 (device float64
    map): the lossy, dispersive step (rb_frequency_step_lossy)."""
    import torch

    from paper_2211_00316_amd import _lib

    d_om = 2 * math.pi * (w.freqs[1] - w.freqs[0]) if len(w.freqs) > 1 else None
    c = c_start.clone()
    rn = torch.zeros(1, dtype=torch.float64, device="cuda:0")

    def one_step(k):
        om = 2 * math.pi * w.freqs[k]
        if alpha0 is not None:
            ctx.frequency_step_lossy(grid, ring, tp, c, alpha0, y, w.smooth_window(k), [om],
                                     [d_om or om], data[k - first], w.tau, residual_norm=rn,
                                     prec=prec)
            return
        ctx.frequency_step(grid, ring, tp, c, w.smooth_window(k), [om], [d_om or om],
                           data[k - first], w.tau, residual_norm=rn, prec=prec)

    for k in range(first, first + warmup):
        one_step(k)
        print(f"[bench] {tag} warmup step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(first + warmup, first + warmup + steps):
        one_step(k)
        print(f"[bench] {tag} step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = ctx.profile_read()
    ctx.profile_enable(False)
    return 1000.0 * elapsed / steps, stages, c


def run_sweep(ctx, w, grid, ring, tp, data, prec, steps, warmup, c_start):
    """The same `steps` frequency steps as one graph launch (rb_frequency_sweep): captured and
    run once from c_start (untimed), then replayed from c_start (timed)."""
    import torch

    d_om = 2 * math.pi * (w.freqs[1] - w.freqs[0]) if len(w.freqs) > 1 else None
    ks = list(range(warmup, warmup + steps))
    sets = [[2 * math.pi * w.freqs[k]] for k in ks]
    dsets = [[d_om or s[0]] for s in sets]
    wins = [w.smooth_window(k) for k in ks]
    sweep_data = data[warmup:warmup + steps]
    c = c_start.clone()
    ctx.frequency_sweep(grid, ring, tp, c, wins, sets, dsets, sweep_data, w.tau, prec=prec,
                        use_graph=True)
    print("[bench] graph sweep captured", file=sys.stderr, flush=True)
    c.copy_(c_start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.frequency_sweep(grid, ring, tp, c, wins, sets, dsets, sweep_data, w.tau, prec=prec,
                        use_graph=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print("[bench] graph sweep replayed", file=sys.stderr, flush=True)
    return 1000.0 * elapsed / steps, c


def source_hash(fname):
    with open(os.path.join(CSRC, fname), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload, prec):
    """HBM bytes per dispatch from the committed PMC summary, keyed by kernel; entries whose
    source file changed since the counters were taken are dropped."""
    path = os.path.join(PROFILES, f"hbm_traffic_{workload}_{prec}.md")
    out = {}
    if not os.path.exists(path):
        return out
    row = re.compile(r"^\|\s*(\w+)\s*\|\s*([\w.]+)\s*\|\s*([0-9a-f]{16})\s*\|"
                     r"\s*(\d+)\s*\|\s*([0-9.eE+]+)\s*\|\s*([0-9.eE+]+)\s*\|\s*([0-9.eE+]+)\s*\|")
    for line in open(path):
        m = row.match(line)
        if m and source_hash(m.group(2)) == m.group(3):
            out[m.group(1)] = float(m.group(7))
    return out


def kernel_rooflines(stages, steps, N, Pm, samples, prec, workload):
    """Per hot kernel: algorithmic work per launch / average launch time, against the peak
    of what bounds it. `samples` = ray samples per step."""
    peak, peak_name = PEAKS[prec]
    tab = TABLE_BYTES[prec]
    traffic = measured_traffic(workload, prec)
    work = {  # stage -> (bound, algorithmic units per step, unit, peak, peak name, what)
        "trace": ("alu", TRACE_FLOP_PER_SAMPLE * samples / 1e12, "TFLOP/s",
                  FP32_VECTOR_PEAK_TFLOPS, "fp32 vector (no packed FP32)",
                  f"{TRACE_FLOP_PER_SAMPLE} flop per ray sample"),
        "resolve": ("hbm", (tab * N * Pm + SAMPLE_BYTES * samples) / 1e9, "GB/s",
                    HBM_PEAK_GBS, "HBM3E",
                    f"{tab} B per table entry written + {SAMPLE_BYTES} B per ray sample read"),
        "build_green": ("hbm", (tab + OPERAND_BYTES[prec]) * N * Pm / 1e9, "GB/s",
                        HBM_PEAK_GBS, "HBM3E",
                        f"{tab} B read + {OPERAND_BYTES[prec]} B written per (e, p)"),
        "forward_gemm": ("mfma", contraction_flops("forward_gemm", N, Pm, prec)[0] / 1e12,
                         "TFLOP/s", peak, peak_name,
                         "flop the kernel issues (upper 256 x 128 tiles of the symmetric "
                         "N x N product, 8 per complex multiply-add over P_m)"),
        "backproject_gemm": ("mfma",
                             contraction_flops("backproject_gemm", N, Pm, prec)[0] / 1e12,
                             "TFLOP/s", peak, peak_name,
                             "flop the kernel issues (row slabs of 256; FP32: 3 complex "
                             "products over the block upper triangle of R; 16-bit: H over it "
                             "and the bilinear form a^T Rs b over all of Rs; split: 2 FP16 "
                             "products over all of Rs + 1 FP8 product counted at half)"),
    }
    out = {}
    for stage, (bound, units, unit, pk, pk_name, what) in work.items():
        if stage not in stages:
            continue
        ms, n = stages[stage]
        launches = n / steps
        avg_ms = ms / max(n, 1)
        achieved = units * steps / (ms * 1e-3)
        kernels = STAGE_KERNELS[stage][0 if prec == "f32" else 1]
        have = all(k in traffic for k in kernels)
        out[stage] = {
            "kernel": "+".join(kernels),
            "bound": bound, "achieved": round(achieved, 2), "peak": pk, "unit": unit,
            "frac": round(achieved / pk, 4),
            "traffic": round(sum(traffic[k] for k in kernels)) if have else None,
            "peak_is": pk_name, "per_unit": what, "avg_launch_ms": round(avg_ms, 3),
            "launches_per_step": round(launches, 2), "ms_per_step": round(ms / steps, 3),
        }
        if stage in ("forward_gemm", "backproject_gemm"):
            issued, own, dense = contraction_flops(stage, N, Pm, prec)
            t = ms * 1e-3 / steps
            out[stage]["own_work_frac"] = round(own / t / 1e12 / pk, 4)
            out[stage]["dense_equivalent_frac"] = round(dense / t / 1e12 / pk, 4)
    return out


def run_serve(args):
    """Serving mix: prints its own JSON line (serve_runs with the full report)."""
    print(json.dumps(serve_runs(args.requests, args.rate_frac, args.prec, full=True)),
          flush=True)


def serve_runs(n_requests, rate_frac, prec_name, full=False):
    """Serving mix: requests of three scan classes (ring 256 / 512 / 1024 on 256^2 / 512^2 /
    1024^2 grids), 8-32 frequency steps each, admitted by HBM budget and stepped with
    continuous batching (paper_2211_00316_amd.serve). A closed-loop run (every request
    waiting at time 0) measures the capacity; the reported run has Poisson arrivals at
    rate_frac of it. Some requests are then run alone and compared with their result in the
    mix. full=False (the bounded leg of the default run): one phantom per class, no
    one-at-a-time run."""
    import numpy as np
    import torch

    import phantoms as ph
    from paper_2211_00316_amd import _lib, serve, setup_for

    prec = PREC_CODES[prec_name]
    classes = ph.SERVE_CLASSES
    draws0 = ph.serve_draws(n_requests, seed=5, rate=None)
    if not full:   # one phantom per class
        draws0 = [ph.ServeDraw(d.rid, d.cls, 1, d.n_steps, d.arrival) for d in draws0]
    ctx = _lib.Context("cuda:0")
    store = {}
    for k, sd in sorted({(d.cls, d.phantom_seed) for d in draws0}):
        w = classes[k]
        grid, ring, tp = setup_for(w)
        print(f"[serve] data of {w.name} phantom {sd}", file=sys.stderr, flush=True)
        store[(k, sd)] = synthesize_data(ctx, w, grid, ring, tp, ph.phantom_for(w, seed=sd),
                                         list(range(len(w.freqs)))).cpu()
    ctx.close()

    def make(draws):
        reqs = []
        for d in draws:
            w = classes[d.cls]
            grid, ring, tp = setup_for(w)
            idx = ph.step_frequencies(d.n_steps, len(w.freqs))
            om = [2 * math.pi * w.freqs[i] for i in idx]
            dom = [2 * math.pi * (w.freqs[-1] - w.freqs[0]) / max(1, d.n_steps - 1)] * d.n_steps
            # host copy of the request's data: the server moves it to the device on admission
            data = store[(d.cls, d.phantom_seed)][torch.as_tensor(idx)].pin_memory()
            c0 = torch.full((w.ny, w.nx), ph.C_WATER, dtype=torch.float64)
            reqs.append(serve.Request(d.rid, d.arrival, grid, ring, tp, om, dom,
                                      [w.smooth_window(i) for i in idx], data, c0,
                                      w.tau, tag=w.name))
        return reqs

    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    budget = int(0.9 * torch.cuda.mem_get_info()[0])
    ex = serve.GpuExecutor(prec, budget=budget)
    last = [0.0]

    def progress(msg):   # at most one line every 5 s
        now = time.perf_counter()
        if now - last[0] >= 5.0:
            last[0] = now
            print(f"[serve] {msg}", file=sys.stderr, flush=True)

    # warm-up: one step of one request per class (module loads, first allocations)
    warm = []
    for k in range(len(classes)):
        first = next((d for d in draws0 if d.cls == k), None)
        if first is not None:
            warm.append(ph.ServeDraw(1000 + k, k, first.phantom_seed, 1, 0.0))
    serve.Server(ex, budget).run(make(warm))
    print("[serve] warm-up done", file=sys.stderr, flush=True)

    # one request at a time (no batching), then the closed loop with batching
    seq = None
    if full:
        seq = serve.Server(ex, budget, max_batch=1, log=progress).run(make(draws0))
        print(f"[serve] one at a time: {seq.summary()}", file=sys.stderr, flush=True)
    closed = serve.Server(ex, budget, log=progress).run(make(draws0))
    cap = len(draws0) / closed.makespan
    rate = rate_frac * cap
    print(f"[serve] closed loop: {closed.summary()}", file=sys.stderr, flush=True)
    draws = ph.serve_draws(n_requests, seed=5, rate=rate)
    if not full:
        draws = [ph.ServeDraw(d.rid, d.cls, 1, d.n_steps, d.arrival) for d in draws]
    mix = serve.Server(ex, budget, log=progress).run(make(draws))
    print(f"[serve] open loop at {rate:.3f} requests/s: {mix.summary()}", file=sys.stderr,
          flush=True)
    # alone vs in the mix: the first request of each class
    by_id = {r.rid: r for r in mix.requests}
    picks = [next(d for d in draws if d.cls == k) for k in range(len(classes))
             if any(d.cls == k for d in draws)]
    diffs = {}
    for d in picks:
        alone = serve.Server(ex, budget).run(make([ph.ServeDraw(d.rid, d.cls, d.phantom_seed,
                                                                d.n_steps, 0.0)]))
        a, m = alone.requests[0], by_id[d.rid]
        diffs[d.rid] = float((a.c - m.c).abs().max().item())
        print(f"[serve] request {d.rid} ({classes[d.cls].name}, {d.n_steps} steps): "
              f"max |c_alone - c_mix| = {diffs[d.rid]:.3e}", file=sys.stderr, flush=True)
    ex.drain()
    del store
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out = {
        "metric": "serving frequency-step updates/s (mixed scans, continuous batching)",
        "value": round(mix.steps_per_s, 3),
        "unit": "frequency-step updates/s",
        "n_gpus": 1,
        "steps": mix.steps,
        "warmup": len(warm),
        "ms_per_step": round(1000.0 / mix.steps_per_s, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec_name,
        "data": "synthetic",
        "p50_latency_s": round(mix.latency_pct(50), 4),
        "p99_latency_s": round(mix.latency_pct(99), 4),
        "config": {"workload": f"serve_mix{len(draws)}",
                   "classes": [c.name for c in classes],
                   "requests": len(draws), "steps_per_request": "8-32",
                   "phantoms_per_class": 3 if full else 1,
                   "arrivals": "poisson", "rate_per_s": round(rate, 4),
                   "rate_frac_of_capacity": rate_frac,
                   "budget_bytes": budget},
        "open_loop": mix.summary(),
        "closed_loop": closed.summary(),
        "alone_vs_mix_max_abs_diff": diffs,
    }
    if seq is not None:
        out["one_at_a_time"] = seq.summary()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ring1024_grid1024")
    ap.add_argument("--prec", default="f16x", choices=["f16x", "bf16", "f16", "f32"],
                    help="operand type of the headline (reduced-precision) form; f16x (FP16 "
                         "with the back-projection operand split into two parts) is the form "
                         "that meets the 2e-3 image tolerance")
    ap.add_argument("--fast-form", default="bf16", choices=["bf16", "f16", "none"],
                    help="plain 16-bit form timed beside the headline (faster, outside the "
                         "image tolerance)")
    ap.add_argument("--late-steps", type=int, default=3,
                    help="steps timed from the true phantom at the last frequencies (a late stage of the "
                         "continuation: bent rays, folded fans); 0 skips them")
    ap.add_argument("--no-gn", action="store_true",
                    help="skip the Gauss-Newton (Hessian-based) and prototype Born steps")
    ap.add_argument("--gn-inner", type=int, default=12, help="CG iterations of a Gauss-Newton step")
    ap.add_argument("--no-lossy", action="store_true",
                    help="skip the absorbing, dispersive (Szabo) form of the same steps")
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="requests of the bounded serving leg of the default run (0 skips it)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--start", default="water", choices=["water", "truth"],
                    help="model of the timed steps: water (first steps of the continuation) "
                         "or the true phantom (a late stage: heterogeneous, folded fans)")
    ap.add_argument("--no-graph", action="store_true",
                    help="report the eager per-step form only (no graph-captured sweep)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB read + 1 GiB write elementwise kernel first "
                         "(reference for the HBM byte counters)")
    ap.add_argument("--no-tune", action="store_true",
                    help="built-in forward launch configuration instead of the autotuner's")
    ap.add_argument("--linked", action="store_true",
                    help="also time the headline form with receiver tables by secant ray "
                         "linking (rb_set_receiver_linking)")
    ap.add_argument("--serve", action="store_true",
                    help="serving mix of scans of three sizes with continuous batching "
                         "(prints its own JSON line)")
    ap.add_argument("--requests", type=int, default=64, help="requests of the serving mix")
    ap.add_argument("--rate-frac", type=float, default=0.8,
                    help="arrival rate of the serving mix, as a fraction of its capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the frequency step on a single "
              "MI355X (see the sharding design); --gpus above 1 is not supported.",
              file=sys.stderr)
        sys.exit(2)

    if args.serve:
        run_serve(args)
        return

    import numpy as np
    import torch

    import phantoms as ph
    from paper_2211_00316_amd import _lib, setup_for

    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    w = ph.WORKLOADS[args.workload]
    grid, ring, tp = setup_for(w)
    ctx = _lib.Context("cuda:0")
    c_true = ph.phantom_for(w)
    n_total = args.warmup + args.steps
    if n_total > len(w.freqs):
        raise SystemExit(f"at most {len(w.freqs)} steps (one per frequency)")
    print(f"[bench] {w.name}: synthesizing data for {n_total} frequencies", file=sys.stderr,
          flush=True)
    data = synthesize_data(ctx, w, grid, ring, tp, c_true, list(range(n_total)))
    prec_code = PREC_CODES[args.prec]

    # forward tiles and K splits of each form from the autotuner (untimed)
    tuning = {}
    if not args.no_tune:
        for name, code in ([("f32", _lib.RB_F32)] if not args.no_fp32 and args.prec != "f32"
                           else []) + [(args.prec, prec_code)]:
            t = ctx.autotune(grid, ring, code)
            tuning[name] = {"forward_tile": "256x128" if t.fwd_tile == _lib.RB_TILE_256x128
                            else "128x128", "forward_splitk": t.fwd_splitk,
                            "forward_ms": round(t.fwd_ms, 3)}
            print(f"[bench] autotune {name}: {tuning[name]}", file=sys.stderr, flush=True)

    forms = {}
    c_start = start_model(w, args.start, c_true)
    if not args.no_fp32 and args.prec != "f32":
        ms32, st32, c32 = run_form(ctx, w, grid, ring, tp, data, _lib.RB_F32, args.steps,
                                   args.warmup, "f32", c_start)
        forms["f32"] = (ms32, st32, c32)
    ms, stages, c_lp = run_form(ctx, w, grid, ring, tp, data, prec_code, args.steps,
                                args.warmup, args.prec, c_start)
    forms[args.prec] = (ms, stages, c_lp)
    ms_eager = ms
    graph = None
    if not args.no_graph:
        ms_graph, _ = run_sweep(ctx, w, grid, ring, tp, data, prec_code, args.steps,
                                args.warmup, c_start)
        graph = {"ms_per_step": round(ms_graph, 2), "value": round(1000.0 / ms_graph, 4)}
        ms = ms_graph

    N = w.n_trans
    mask = _mask_index(w)
    Pm = mask.numel()
    samples = ctx.trace_samples()
    rl = kernel_rooflines(stages, args.steps, N, Pm, samples, args.prec, w.name)
    dominant = max(rl, key=lambda k: rl[k]["ms_per_step"])
    roofline = dict(rl[dominant], stage=dominant)
    line = {
        "metric": "frequency-step updates/s at 1024 elems, 1024^2 grid (reduced-precision form; "
                  "FP32 form alongside)",
        "value": round(1000.0 / ms, 4),
        "unit": "frequency-step updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "form": ("one HIP-graph launch of the steps (rb_frequency_sweep)" if graph else
                 "one rb_frequency_step call per step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic (seeded breast-like phantom, ray-Born data + 1% noise)",
        "config": {"workload": w.name, "transducers": N, "grid": f"{w.nx}x{w.ny}",
                   "dx_mm": w.dx * 1e3, "rays_per_transducer": w.n_rays,
                   "mask_nodes": int(Pm), "freqs_hz": [w.freqs[k] for k in
                                                        range(args.warmup, n_total)],
                   "start_model": args.start,
                   "parallelism": "single GPU",
                   "autotuned_forward": tuning or None},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
        "roofline": roofline,
        "rooflines": rl,
        "eager_form": {"ms_per_step": round(ms_eager, 2), "value": round(1000.0 / ms_eager, 4)},
        "graph_form": graph,
        "ray_samples_per_step": samples,
    }
    if "f32" in forms and args.prec != "f32":
        ms32, st32, c32 = forms["f32"]
        line["fp32_form"] = {
            "value": round(1000.0 / ms32, 4), "ms_per_step": round(ms32, 2),
            "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in st32.items()}}
        line["speedup_vs_fp32"] = round(ms32 / ms_eager, 3)   # both eager, per step
        # same frequencies, same start: image difference between the two forms on the mask
        a = c_lp.reshape(-1)[mask]
        b = c32.reshape(-1)[mask]
        line["image_rel_diff_vs_fp32"] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        da, db = a - 1500.0, b - 1500.0
        line["update_rel_diff_vs_fp32"] = float(torch.linalg.norm(da - db) / torch.linalg.norm(db))
    if args.linked:
        ctx.set_receiver_linking(12, 1e-8)
        msl, stl, _ = run_form(ctx, w, grid, ring, tp, data, prec_code, args.steps, args.warmup,
                               args.prec + "-linked", c_start)
        ctx.set_receiver_linking(0)
        line["linked_receivers_form"] = {
            "ms_per_step": round(msl, 2), "value": round(1000.0 / msl, 4),
            "linking": "secant, at most 12 rays per pair, exit-angle tolerance 1e-8 rad",
            "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stl.items()}}
    if args.fast_form != "none" and args.fast_form != args.prec:
        msf, stf, cf = run_form(ctx, w, grid, ring, tp, data, PREC_CODES[args.fast_form],
                                args.steps, args.warmup, args.fast_form, c_start)
        ff = {"ms_per_step": round(msf, 2), "value": round(1000.0 / msf, 4),
              "note": "plain 16-bit operands: faster, outside the 2e-3 image tolerance",
              "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stf.items()},
              "rooflines": kernel_rooflines(stf, args.steps, N, Pm, samples, args.fast_form,
                                            w.name)}
        if "f32" in forms:
            a, b = cf.reshape(-1)[mask] - 1500.0, forms["f32"][2].reshape(-1)[mask] - 1500.0
            ff["update_rel_diff_vs_fp32"] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        line[f"{args.fast_form}_form"] = ff
        del cf
    if args.late_steps > 0:
        # the last frequencies of the continuation (their narrowest smoothing windows), from
        # the true phantom: bent rays and folded fans
        c_late = start_model(w, "truth", c_true)
        n_late = min(args.late_steps, len(w.freqs) - 1)
        wl = min(1, len(w.freqs) - n_late)
        first = len(w.freqs) - n_late - wl
        late_data = synthesize_data(ctx, w, grid, ring, tp, c_true,
                                    list(range(first, len(w.freqs))))
        msl, stl, _ = run_form(ctx, w, grid, ring, tp, late_data, prec_code, n_late, wl,
                               args.prec + "-late", c_late, first=first)
        del late_data
        line["late_stage_form"] = {
            "ms_per_step": round(msl, 2), "value": round(1000.0 / msl, 4), "steps": n_late,
            "frequencies_hz": [round(w.freqs[k]) for k in range(first + wl, len(w.freqs))],
            "smoothing_windows": [w.smooth_window(k) for k in range(first + wl, len(w.freqs))],
            "start_model": "true phantom (bent rays, folded fans)",
            "stages_ms_per_step": {k: round(v[0] / n_late, 3) for k, v in stl.items()}}
    if not args.no_gn:
        line.update(gauss_newton_legs(ctx, w, grid, ring, tp, data, prec_code, args, c_start))
    if not args.no_lossy:
        line["lossy_form"] = lossy_leg(ctx, w, grid, ring, tp, c_true, prec_code, args, c_start,
                                       ms_eager)
    del data
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.serve_requests > 0:
        print("[bench] bounded serving leg", file=sys.stderr, flush=True)
        sv = serve_runs(args.serve_requests, args.rate_frac, args.prec, full=False)
        line["serving"] = {k: sv[k] for k in ("value", "unit", "p50_latency_s",
                                               "p99_latency_s", "steps", "config",
                                               "closed_loop", "alone_vs_mix_max_abs_diff")}
        line["p50_latency_s"] = sv["p50_latency_s"]
        line["p99_latency_s"] = sv["p99_latency_s"]
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


def lossy_leg(ctx, w, grid, ring, tp, c_true, prec, args, c_start, ms_lossless):
    """The same steps in the absorbing, dispersive medium (Szabo's model, y = 1.4, the
    phantom's alpha0 map of 0-1 dB MHz^-y cm^-1): data synthesised in that medium, one
    rb_frequency_step_lossy per frequency (rays traced on that frequency's map), and one step
    of a set of two frequencies (two traces) beside the lossless step of the same set."""
    import torch

    import phantoms as ph

    y = 1.4
    alpha0 = ph.absorption_for(w, y=y)
    n_total = args.warmup + args.steps
    print("[bench] lossy data", file=sys.stderr, flush=True)
    data = synthesize_data(ctx, w, grid, ring, tp, c_true, list(range(n_total)), alpha0, y)
    a_t = torch.as_tensor(alpha0, device="cuda:0")
    ms, st, _ = run_form(ctx, w, grid, ring, tp, data, prec, args.steps, args.warmup,
                         "lossy", c_start, alpha0=a_t, y=y)
    k0 = args.warmup
    oms = [2 * math.pi * w.freqs[k0], 2 * math.pi * w.freqs[k0 + 1]]
    d_om = oms[1] - oms[0]
    d2 = data[k0:k0 + 2].contiguous()
    win = w.smooth_window(k0)

    def timed(fn, reps=2):
        c = c_start.clone()
        fn(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.copy_(c_start)
            fn(c)
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - t0) / reps

    ms2 = timed(lambda c: ctx.frequency_step_lossy(grid, ring, tp, c, a_t, y, win, oms,
                                                   [d_om, d_om], d2, w.tau, prec=prec))
    ms2l = timed(lambda c: ctx.frequency_step(grid, ring, tp, c, win, oms, [d_om, d_om], d2,
                                              w.tau, prec=prec))
    print(f"[bench] lossy step {ms:.1f} ms; set of two: {ms2:.1f} ms (lossless {ms2l:.1f})",
          file=sys.stderr, flush=True)
    del data
    return {"ms_per_step": round(ms, 2), "value": round(1000.0 / ms, 4),
            "medium": "Szabo power law y = 1.4, alpha0 0-1 dB MHz^-y cm^-1 (phantom's map)",
            "cost_vs_lossless": round(ms / ms_lossless, 3),
            "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in st.items()},
            "two_frequency_set": {"lossy_ms": round(ms2, 2), "lossless_ms": round(ms2l, 2),
                                  "traces": "one per frequency (lossy), one per set (lossless)"}}


def gauss_newton_legs(ctx, w, grid, ring, tp, data, prec, args, c_start):
    """The paper's comparison methods on the same workload and set of two frequencies: one
    Hessian-based (Gauss-Newton, CG) step, one prototype Born step, and the Hessian-free step
    of the same set (the paper reports the first about ten times as costly as the last)."""
    import torch

    from paper_2211_00316_amd import _lib

    k0 = args.warmup
    oms = [2 * math.pi * w.freqs[k0], 2 * math.pi * w.freqs[k0 + 1]]
    d2 = data[k0:k0 + 2].contiguous()
    win = w.smooth_window(k0)
    d_om = oms[1] - oms[0]
    out = {}

    def timed(fn, reps=2):
        c = c_start.clone()
        fn(c)   # first call: workspaces
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.copy_(c_start)
            fn(c)
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - t0) / reps

    ms_hf = timed(lambda c: ctx.frequency_step(grid, ring, tp, c, win, oms, [d_om, d_om], d2,
                                               w.tau, prec=prec))
    print(f"[bench] Hessian-free step of 2 frequencies: {ms_hf:.1f} ms", file=sys.stderr,
          flush=True)
    for name, model in (("gauss_newton_form", _lib.RB_GREEN_RAY),
                        ("prototype_born_form", _lib.RB_GREEN_WATER)):
        ms = timed(lambda c: ctx.gauss_newton_step(grid, ring, tp, c, win, oms, d2, 1.0,
                                                   args.gn_inner, model=model, prec=prec))
        print(f"[bench] {name}: {ms:.1f} ms", file=sys.stderr, flush=True)
        out[name] = {"ms_per_step": round(ms, 2), "value": round(1000.0 / ms, 4),
                     "set": "2 frequencies", "cg_iterations": args.gn_inner,
                     "hessian_free_ms_same_set": round(ms_hf, 2),
                     "cost_vs_hessian_free": round(ms / ms_hf, 2)}
    return out


if __name__ == "__main__":
    main()
