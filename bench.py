"""Effective-field throughput on one MI355X: H_eff evaluations per second.

Workload: the 3D-periodic composite of 27 magnetic spheres in a 100 nm cell
(about 1.03 M unknowns, AIM grid 128^3, Lagrange order 3, near radius 2
boxes, element-exact radius 1 mean edge length), plain FP32 path. One step is
one full H_eff = H_ex + H_ms evaluation (all nine kernels) of a fixed
magnetisation already resident in HBM. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
                    [--precision 0|1|2] [--no-cpu-baseline] [--copy-mib MIB]
    python bench.py --config batched_films [--cells 64]
    python bench.py --llg implicit [--t-end 1e-9] [--lte-tol 1e-6] [--alpha 0.02] [--relax 5e-10]
                          [--scheme midpoint|bdf2]
    python bench.py --surrogate [--sg-pairs 2000] [--sg-steps 10000] [--sg-bf16]
"""
from __future__ import annotations

import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak of the MI355X


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(ctx, names, precision=0):
    """Algorithmic HBM bytes per launch of each named kernel (every array once).

    precision 1 stores the grid charges and potential as BF16 (2 bytes per
    grid value), precision 0 as FP32 and precision 2 as a BF16 pair (4)."""
    gb = 2.0 if precision == 1 else 4.0
    info = ctx.export("grid_info")
    N = info[0:3].astype(np.int64)
    M = info[3:6].astype(np.int64)
    n = float(ctx.n)
    nL = float(ctx.export("loc_rowptr")[-1])
    nZ = float(ctx.export("z0_rowptr")[-1])
    nP = float(ctx.export("p_rowptr")[-1])
    nbox = float(ctx.export("box_start").size)
    ng = float(np.prod(N))
    hx = float(M[0] // 2 + 1)
    s_in = float(N[2] * N[1]) * hx * 8      # half-spectrum rows y < Ny
    s_full = float(N[2] * M[1]) * hx * 8    # half-spectrum, all My rows
    khat = hx * M[1] * M[2] * 4
    fam = {
        "k_charges": n * (4 + 12 + 4) + nL * 16,
        "k_zcorr": n * (4 + 12 + 4) + nZ * 16,
        "k_anterp": n * (4 + 16) + nbox * 4 + ng * gb,
        "k_anterp_scatter": n * (4 + 16 + 4),
        "k_anterp_sum": ng * gb,
        "k_r2c_x": ng * gb + s_in,
        "k_fft_y_fwd": s_in + s_full,
        "k_fft_z_mul": 2 * s_full + khat,
        "k_fft_y_inv": s_full + s_in,
        "k_c2r_x": s_in + ng * gb,
        "k_fft_xy_fwd": ng * gb + s_full,
        "k_fft_yx_inv": s_full + ng * gb,
        "k_interp": n * (16 + 4 + 4 + 4 + 4) + ng * gb + nP * 4,
        "k_grad": n * (4 + 12 + 4 + 12) + nL * 20,
        "k_exch": n * (4 + 12 + 12) + nL * 8,
        "k_gsum": n * (4 + 4 + 12 + 12) + nL * 16,
    }
    # every form of a stage moves the same algorithmic bytes (longest prefix wins)
    return {name: next(v for k, v in sorted(fam.items(), key=lambda kv: -len(kv[0]))
                       if name.startswith(k)) for name in names}


WORKLOADS = {
    "composite_c3": "3D-periodic composite, 27 spheres r=12-18 nm in a 100 nm cell",
    "wire_c2": "1D-periodic wire, radius 10 nm, period 40 nm, two domain walls",
    "film_c1": "2D-periodic film, 20x20x2 nm cell",
}


def measured_traffic(kernel, summary="composite_c3_hbm_traffic.json", source="kernels.hip"):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_2409_13958_amd", "csrc", source)
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get(source.replace(".", "_") + "_sha256") != h:
        return None
    for name, b in rec.get("bytes_per_launch", {}).items():
        if name.split("<")[0] == kernel:
            return float(b)
    return None


def calibrate_counters(mib):
    """Plain streams of known size for the HBM counters of a profiled run, each
    one elementwise kernel (a device copy may run on a DMA engine that the
    counters do not see): a fill writes mib MiB, a negation reads and writes
    mib MiB each; the counters of the other kernels are scaled by what they
    read for these."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"counter calibration: one {mib} MiB fill, 3 negations of {mib} MiB")


def host_info():
    """CPU model and the number of hardware threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        threads = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        threads = os.cpu_count() or 1
    return model, threads


def cpu_baseline(prob, rows_sample=64, seed=7, budget_s=10.0):
    """Time the FP64 oracle on a bounded sample of the same workload.

    The oracle's operators for a sample of observer rows are built untimed
    (as the library's setup is); the timed part is one evaluation: the
    full-size steps (exchange, charges, projection, 3D FFT convolution) once,
    plus interpolation, precorrection and element correction on the ring of
    the sampled rows and the gradient at the sampled rows, extrapolated
    linearly to all N' rows. It is timed twice: with its thread pools held to
    one thread, and with every hardware thread of the host allowed; the
    threads actually used are the process CPU time over the wall time.
    """
    from oracle import model
    from threadpoolctl import threadpool_limits
    t0 = time.perf_counter()
    orc = model.Oracle(prob)
    log(f"  oracle operators built ({time.perf_counter() - t0:.0f} s)")
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(orc.n, size=rows_sample, replace=False))
    ring = orc.ops.neighbours(rows)
    m = orc.unknown_values(prob.m)
    orc.potential(m, ring, "aim")          # builds and caches the ring's P and Z0 rows
    t_setup = time.perf_counter() - t0
    log(f"  oracle ring rows built ({t_setup:.0f} s)")
    P = orc._cache[("P", tuple(ring.tolist()))]
    Z = orc.z0(ring)
    A = orc.aim

    def timed(limit):
        tt = {k: 0.0 for k in ("exchange", "charges", "grid", "ring", "grad")}
        reps = 0
        limiter = threadpool_limits(limits=limit)
        c0, w0 = time.process_time(), time.perf_counter()
        # repeat the evaluation until about budget_s of CPU work have been timed
        while reps < 200 and (reps == 0 or sum(tt.values()) < budget_s):
            t = time.perf_counter()
            orc.ops.exchange(m)
            tt["exchange"] += time.perf_counter() - t
            t = time.perf_counter()
            q = orc.ops.charges(m)
            tt["charges"] += time.perf_counter() - t
            t = time.perf_counter()
            U = A.convolve(A.project(q))
            tt["grid"] += time.perf_counter() - t
            t = time.perf_counter()
            u_ring = ((A.interpolate(U, ring) + P @ q) / (4 * np.pi)
                      + sum(Z[c] @ m[:, c] for c in range(3)))
            tt["ring"] += time.perf_counter() - t
            u = np.zeros(orc.n)
            u[ring] = u_ring
            t = time.perf_counter()
            orc.ops.gradient_field(u, rows)
            tt["grad"] += time.perf_counter() - t
            reps += 1
        used = (time.process_time() - c0) / max(time.perf_counter() - w0, 1e-9)
        limiter.restore_original_limits()
        full = (tt["exchange"] + tt["charges"] + tt["grid"] + tt["ring"] * orc.n / ring.size
                + tt["grad"] * orc.n / rows.size) / reps
        return 1.0 / full, reps, sum(tt.values()), used

    model_name, threads = host_info()
    v1, reps1, t1, used1 = timed(1)
    log(f"  one thread: {v1:.4f} evals/s ({reps1} reps, {t1:.1f} s, {used1:.2f} threads busy)")
    va, repsa, ta, useda = timed(threads)
    log(f"  {threads} threads allowed: {va:.4f} evals/s ({repsa} reps, {ta:.1f} s, "
        f"{useda:.2f} threads busy)")
    return {
        "value": v1,
        "unit": "H_eff evals/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one FP64 oracle evaluation: full-size exchange, charges and "
                   f"{'x'.join(str(g) for g in prob.grid)} FFT convolution timed once; "
                   f"interpolation+precorrection+element correction on the {ring.size}-row "
                   f"ring of {rows.size} sampled rows and their gradient, scaled to "
                   f"N'={orc.n}; {reps1} repetitions, timed {t1:.1f} s (setup "
                   f"{t_setup:.0f} s untimed)"),
        "all_threads": {"value": va, "threads_allowed": threads,
                        "threads_busy": round(useda, 2), "reps": repsa,
                        "timed_s": round(ta, 1)},
        "host": {"cpu_model": model_name, "nproc": threads},
    }


def sampled_error(ctx, prob, name, m, h):
    """Relative error of the timed run's H_eff (and of H_ex, H_ms evaluated
    alone) at the unknowns whose FP64 oracle values are stored with the tests:
    relative L2 over the samples and max-norm relative to the largest sample."""
    import torch
    from paper_2409_13958_amd import binding as B
    path = os.path.join(ROOT, "tests", "golden", "expected_fullsize.npz")
    try:
        exp = np.load(path)
    except OSError:
        return None
    if f"{name}_nodes" not in exp.files:
        return None
    _, uon, _, _ = ctx.query()
    idx = uon[exp[f"{name}_nodes"]]
    hex_, hms = torch.empty_like(h), torch.empty_like(h)
    ctx.heff(m, hex_, terms=B.TERM_EX)
    ctx.heff(m, hms, terms=B.TERM_MS)
    torch.cuda.synchronize()
    out = {"samples": int(idx.size),
           "reference": "FP64 oracle (same AIM), stored at sampled unknowns"}
    for k, v in (("h_eff", h), ("h_ex", hex_), ("h_ms", hms)):
        got = v.cpu().numpy().astype(np.float64)[idx]
        ref = exp[f"{name}_{k.replace('_eff', '').replace('_', '')}"]
        d = got - ref
        out[k] = {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                  "rel_max": float(np.abs(d).max() / np.abs(ref).max())}
    return out


def run_batched(args):
    """Independent 2D-periodic films of uneven size: one H_eff of every film per
    step, as one batch (one launch per stage for all films), beside the same
    films evaluated one after another; the same for one RK4 step."""
    import torch
    from paper_2409_13958_amd import binding as B, meshgen as mg
    t = time.perf_counter()
    probs = mg.films_c4(args.cells, extents=args.film_extents)
    log(f"{len(probs)} films, {sum(p.n_nodes for p in probs)} nodes "
        f"({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    ctxs, ms = [], []
    for p in probs:
        ctx = B.Context.from_problem(p, device=0)
        n, uon, nou, bpe = ctx.query()
        ctxs.append(ctx)
        ms.append(torch.tensor(p.m[nou], dtype=torch.float32))
    batch = B.Batch(ctxs)
    m = torch.cat(ms).cuda()
    h = torch.empty_like(m)
    off = batch.offsets
    log(f"setup: {batch.n} unknowns, model bytes per batch evaluation "
        f"{batch.bytes_per_eval / 1e9:.3f} GB ({time.perf_counter() - t:.1f} s)")

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    cells_m = [m[off[k]:off[k + 1]] for k in range(len(ctxs))]
    cells_h = [torch.empty_like(x) for x in cells_m]

    def loop_heff():
        for c, mk, hk in zip(ctxs, cells_m, cells_h):
            c.heff(mk, hk)

    dt_batch = timed(lambda: batch.heff(m, h), args.steps)
    dt_loop = timed(loop_heff, args.steps)
    torch.cuda.synchronize()
    diff = max(float((h[off[k]:off[k + 1]] - cells_h[k]).abs().max() /
                     cells_h[k].abs().max()) for k in range(len(ctxs)))
    log(f"H_eff of {len(ctxs)} films: batch {dt_batch * 1e3:.3f} ms, one after another "
        f"{dt_loop * 1e3:.3f} ms (x{dt_loop / dt_batch:.2f}); max relative difference {diff:.1e}")
    m64 = m.double()
    llg_steps = max(1, args.steps // 10)
    dt_llg = timed(lambda: batch.llg_step(m64, 1e-13, 0.5, 1), llg_steps)
    dt_graph = timed(lambda: batch.llg_step_graph(m64, 1e-13, 0.5, 1), llg_steps)
    log(f"one RK4 step of {len(ctxs)} films (batch): {dt_llg * 1e3:.3f} ms, replayed from a "
        f"captured HIP graph {dt_graph * 1e3:.3f} ms")
    achieved = batch.bytes_per_eval / dt_batch / 1e9
    result = {
        "metric": "H_eff evals/s of batched unit cells (cell evaluations)",
        "value": len(ctxs) / dt_batch,
        "unit": "cell H_eff evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{len(ctxs)} independent 2D-periodic films, node counts log-uniform "
                         f"5k-80k ({batch.n} unknowns in all), periods 20-200 nm, thickness "
                         f"2-10 nm, Ms 4e5-1.6e6 A/m, in-plane FFT extents "
                         f"{'with factors 2, 3, 5, 7' if args.film_extents == 'smooth' else 'powers of two'}"
                         f" ({sum(int(np.prod(p.grid)) for p in probs)} grid points in all), one "
                         f"H_eff of every film per step, one launch per stage for all films"),
            "name": "batched_films",
            "cells": len(ctxs),
            "film_extents": args.film_extents,
            "n_unknowns": batch.n,
            "unknown_evals_per_s": batch.n / dt_batch,
            "one_after_another_ms": dt_loop * 1e3,
            "batch_speedup": dt_loop / dt_batch,
            "rk4_step_ms": dt_llg * 1e3,
            "rk4_step_graph_ms": dt_graph * 1e3,
            "max_rel_diff_vs_per_cell": diff,
        },
        "roofline": {"kernel": "whole batch evaluation (model bytes)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    print(json.dumps(result), flush=True)


def run_implicit(args, prob):
    """A run of LLG dynamics in the manner of the paper's timing of magnetisation
    dynamics (Sec. 5: 1 ns of the 3D-periodic granular structure under a
    uniform 1 Oe drive, adaptive implicit stepping with Newton and a
    preconditioned Krylov solver): the composite from a uniform state along z,
    a 1 Oe field along x (a 5 MHz drive changes by about 3 % over 1 ns, so it
    is held constant), damping 0.02, adaptive BDF2 (or, with --scheme, the
    adaptive midpoint rule) at a local error tolerance of --lte-tol. The uniform state is not an equilibrium of
    the grains, so an untimed relaxation (damping 1, no applied field, local
    tolerance 1e-4, --relax seconds of dynamics) comes first, as the paper's
    drive starts from the structure's own state. Reports the wall time of the
    driven run and its accepted and rejected steps, Newton and Krylov
    iterations."""
    import torch
    from paper_2409_13958_amd import binding as B
    t = time.perf_counter()
    ctx = B.Context.from_problem(prob, device=0)
    n, uon, nou, bpe = ctx.query()
    log(f"setup: N'={n} ({time.perf_counter() - t:.1f} s)")
    alpha, h_app = args.alpha, [1e3 / (4 * math.pi), 0.0, 0.0]
    m0 = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    m0[:, 2] = 1.0

    def torque(mm):
        m32 = mm.float().contiguous()
        hh = torch.empty_like(m32)
        ctx.heff(m32, hh)
        torch.cuda.synchronize()
        return float(torch.cross(m32, hh, dim=1).norm(dim=1).pow(2).mean().sqrt())

    tq0 = torque(m0)
    t0 = time.perf_counter()
    rel = ctx.llg_implicit_adaptive(m0, args.relax, args.dt, 1.0, lte_tol=1e-4)
    torch.cuda.synchronize()
    tq1 = torque(m0)
    log(f"relaxation, {args.relax * 1e9:g} ns at damping 1: {time.perf_counter() - t0:.1f} s, "
        f"{rel['accepted']} steps, rms torque |m x H| {tq0:.3g} -> {tq1:.3g} A/m")
    # warm-up: the first launches of the driven run, untimed
    m = m0.clone()
    ctx.llg_implicit_adaptive(m, 10 * args.dt, args.dt, alpha, lte_tol=args.lte_tol,
                              h_applied=h_app, scheme=args.scheme)
    torch.cuda.synchronize()
    m = m0.clone()
    t0 = time.perf_counter()
    st = ctx.llg_implicit_adaptive(m, args.t_end, args.dt, alpha, lte_tol=args.lte_tol,
                                   h_applied=h_app, log_steps=100000, scheme=args.scheme)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    norm_dev = float((m.norm(dim=1) - 1).abs().max())
    mx = float(m[:, 0].mean())
    dts = st["dts"]
    log(f"adaptive {args.scheme}, {args.t_end * 1e9:g} ns: {wall:.2f} s wall, {st['accepted']} steps "
        f"({st['rejected']} rejected), {st['newton']} Newton and {st['krylov']} Krylov "
        f"iterations; steps {dts.min():.2e} .. {dts.max():.2e} s; <m_x> = {mx:.3e}; "
        f"max ||m|-1| {norm_dev:.1e}")
    result = {
        "metric": f"wall time of LLG dynamics (adaptive implicit {args.scheme}, Newton-GMRES)",
        "value": wall,
        "unit": "s",
        "n_gpus": 1,
        "steps": st["accepted"],
        "warmup": 1,
        "ms_per_step": wall * 1e3 / max(st["accepted"], 1),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FP32 fields)",
        "data": "synthetic",
        "config": {
            "workload": (f"{WORKLOADS.get(args.config, args.config)}, N'={n} unknowns, "
                         f"{args.t_end * 1e9:g} ns after {args.relax * 1e9:g} ns of relaxation "
                         f"from uniform m along z, 1 Oe along x, "
                         f"alpha = {alpha}, local error tolerance {args.lte_tol:g}, "
                         f"first step {args.dt:g} s"),
            "name": args.config,
            "relaxed_rms_torque_A_per_m": tq1,
            "accepted_steps": st["accepted"],
            "rejected_steps": st["rejected"],
            "newton_iterations": st["newton"],
            "krylov_iterations": st["krylov"],
            "min_step_s": float(dts.min()),
            "max_step_s": float(dts.max()),
            "mean_mx": mx,
            "max_norm_deviation": norm_dev,
        },
    }
    print(json.dumps(result), flush=True)


def run_surrogate(args):
    """The learned-surrogate workload: a 2D-periodic film of 512 x 512 x 8 nm
    (1 nm lattice, 2.36 M unknowns) on the AIM grid 512 x 512 x 8. Trains the
    6-layer, 32-channel convolution network on AIM pairs from random, vortex
    and domain-wall textures (--sg-pairs pairs, one Adam step each), then
    times H_eff with the surrogate in place of the FFT convolution against the
    plain path on a vortex state, the network alone against the FFT
    convolution alone (per layer, HIP events on the context's stream), and
    runs --sg-steps RK4 steps judged by the plain AIM every 50 steps with
    fallback above a field error of 1e-3."""
    import torch
    from paper_2409_13958_amd import binding as B, meshgen as mg
    t = time.perf_counter()
    prob = mg.film_c5()
    log(f"mesh film_c5: {prob.n_nodes} nodes, {prob.tets.shape[0]} tets "
        f"({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    ctx = B.Context.from_problem(prob, device=0)
    n = ctx.n
    shape = ctx._grid_shape()
    nvox = int(np.prod(shape))
    log(f"setup: N'={n}, grid {shape[::-1]} ({time.perf_counter() - t:.1f} s)")
    if args.copy_mib > 0:
        calibrate_counters(args.copy_mib)
    depth = 6
    ctx.surrogate_init(depth, seed=1, bf16_activations=args.sg_bf16)
    t = time.perf_counter()
    chunks = []
    for c0 in range(0, args.sg_pairs, 1000):
        chunks.append(ctx.surrogate_train(min(1000, args.sg_pairs - c0), lr=args.sg_lr,
                                          seed=2 + c0))
        log(f"training: {c0 + chunks[-1].size} pairs, loss of the last {chunks[-1].size}: "
            f"{chunks[-1].mean():.3e} ({time.perf_counter() - t:.1f} s)")
    losses = np.concatenate(chunks) if chunks else np.zeros(1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    k = max(1, min(50, args.sg_pairs // 10))
    log(f"training: {args.sg_pairs} pairs in {train_s:.1f} s ({train_s / max(1, args.sg_pairs) * 1e3:.1f}"
        f" ms/pair); loss first {k}: {losses[:k].mean():.3e}, last {k}: {losses[-k:].mean():.3e}")

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    m64 = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    ctx.surrogate_texture(m64, 1, seed=7)
    m32 = m64.float()
    h_plain = torch.empty_like(m32)
    h_sur = torch.empty_like(m32)
    dt_plain = timed(lambda: ctx.heff(m32, h_plain), args.steps)
    ctx.surrogate_enable(True)
    dt_sur = timed(lambda: ctx.heff(m32, h_sur), args.steps)
    ctx.surrogate_enable(False)
    ctx.heff(m32, h_plain)
    ctx.surrogate_enable(True)
    ctx.heff(m32, h_sur)
    ctx.surrogate_enable(False)
    hm_plain = torch.empty_like(m32)
    hm_sur = torch.empty_like(m32)
    ctx.heff(m32, hm_plain, terms=B.TERM_MS)
    ctx.surrogate_enable(True)
    ctx.heff(m32, hm_sur, terms=B.TERM_MS)
    ctx.surrogate_enable(False)
    torch.cuda.synchronize()
    err_heff = float(torch.linalg.norm((h_sur - h_plain).double()) /
                     torch.linalg.norm(h_plain.double()))
    err_hms = float(torch.linalg.norm((hm_sur - hm_plain).double()) /
                    torch.linalg.norm(hm_plain.double()))
    log(f"H_eff: plain {dt_plain * 1e3:.3f} ms, surrogate {dt_sur * 1e3:.3f} ms; field error of "
        f"the surrogate (vortex state): H_ms {err_hms:.3e}, H_eff {err_heff:.3e}")
    # the grid step alone: FFT convolution against the network, per layer
    qg = torch.randn(shape, device="cuda")
    ug = torch.empty_like(qg)
    dt_fft = timed(lambda: ctx.grid_convolve(qg, ug), args.steps)
    layer_ms = ctx.surrogate_profile(qg, ug, reps=max(3, args.steps // 4))
    mid_ms = float(np.mean(layer_ms[1:depth - 1]))
    flop_mid = 2.0 * 27 * 32 * 32 * nvox
    achieved = flop_mid / (mid_ms * 1e-3) / 1e12
    log(f"grid step: FFT convolution {dt_fft * 1e3:.3f} ms; network {layer_ms.sum():.3f} ms "
        f"(layers {', '.join(f'{x:.3f}' for x in layer_ms)} ms); 32->32 layer "
        f"{achieved:.1f} TFLOP/s of {MFMA_BF16_PEAK_TFLOPS:.0f}")
    # judged LLG
    m = m64.clone()
    t0 = time.perf_counter()
    rep = ctx.llg_step_judged(m, 1e-13, 0.5, args.sg_steps, check_every=50, tol=1e-3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"judged RK4: {args.sg_steps} steps in {wall:.1f} s; {rep['checks']} checks, max error "
        f"{rep['max_error']:.3e}, fallback at step {rep['fallback_step']}")
    result = {
        "metric": "H_eff evals/s with the learned surrogate in place of the FFT convolution",
        "value": 1.0 / dt_sur,
        "unit": "H_eff evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_sur * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 weights, " + ("bf16" if args.sg_bf16 else "f32 (bf16 pair)") +
                 " activations, f32 accumulation",
        "data": "synthetic",
        "config": {
            "workload": (f"2D-periodic film 512x512x8 nm, 1 nm lattice, N'={n} unknowns, AIM grid "
                         f"512x512x8; 6-layer 32-channel 3x3x3 network trained on {args.sg_pairs} "
                         f"AIM pairs (random, vortex, domain-wall textures) at lr {args.sg_lr:g}; "
                         f"H_eff of a vortex state"),
            "name": "film_c5_surrogate",
            "plain_heff_evals_per_s": 1.0 / dt_plain,
            "surrogate_field_error_hms": err_hms,
            "surrogate_field_error_heff": err_heff,
            "training_pairs": args.sg_pairs,
            "training_s": train_s,
            "training_loss_first": float(losses[:k].mean()),
            "training_loss_last": float(losses[-k:].mean()),
            "fft_convolution_ms": dt_fft * 1e3,
            "network_layer_ms": [float(x) for x in layer_ms],
            "judged_rk4_steps": args.sg_steps,
            "judged_rk4_wall_s": wall,
            "judge_checks": rep["checks"],
            "judge_max_error": rep["max_error"],
            "judge_fallback_step": rep["fallback_step"],
        },
        "roofline": {"kernel": "k_sg_mid (32->32 layer, matrix cores)", "bound": "mfma",
                     "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_BF16_PEAK_TFLOPS,
                     "traffic": (None if args.sg_bf16 else measured_traffic(
                         "k_sg_mid", "film_c5_surrogate_hbm_traffic.json", "surrogate.hip")),
                     "flop_per_launch": flop_mid,
                     "note": ("algorithmic FLOPs 2*27*32*32 per grid point; the FP32-accurate "
                              "form issues twice as many matrix-core products (BF16 high part "
                              "and remainder)" if not args.sg_bf16 else
                              "algorithmic FLOPs 2*27*32*32 per grid point")},
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="composite_c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", type=int, default=0, choices=(0, 1, 2),
                    help="grid storage: 0 FP32, 1 BF16, 2 BF16 hi + lo (one refinement step)")
    ap.add_argument("--llg", choices=("none", "implicit"), default="none",
                    help="implicit: time a run of adaptive implicit LLG dynamics instead")
    ap.add_argument("--dt", type=float, default=1e-13, help="--llg: first trial step (s)")
    ap.add_argument("--t-end", type=float, default=1e-9, help="--llg: simulated time (s)")
    ap.add_argument("--lte-tol", type=float, default=1e-6, help="--llg: local error tolerance")
    ap.add_argument("--alpha", type=float, default=0.02, help="--llg: damping")
    ap.add_argument("--scheme", choices=("midpoint", "bdf2"), default="bdf2",
                    help="--llg: the adaptive implicit scheme of the driven run")
    ap.add_argument("--relax", type=float, default=5e-10,
                    help="--llg: untimed relaxation before the driven run (s)")
    ap.add_argument("--cells", type=int, default=64,
                    help="films of the batched_films workload")
    ap.add_argument("--film-extents", choices=("smooth", "pow2"), default="smooth",
                    help="batched_films: FFT extents with factors 2, 3, 5, 7, or powers of two")
    ap.add_argument("--surrogate", action="store_true",
                    help="the learned-surrogate workload (film 512x512x8 nm)")
    ap.add_argument("--sg-pairs", type=int, default=2000, help="--surrogate: training pairs")
    ap.add_argument("--sg-lr", type=float, default=1e-3, help="--surrogate: Adam learning rate")
    ap.add_argument("--sg-steps", type=int, default=10000, help="--surrogate: judged RK4 steps")
    ap.add_argument("--sg-bf16", action="store_true",
                    help="--surrogate: BF16 activations in the 32->32 layers")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also stream this many MiB through plain kernels (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is designed but not implemented", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.config == "batched_films":
        run_batched(args)
        return
    if args.surrogate:
        run_surrogate(args)
        return

    import torch
    from paper_2409_13958_amd import binding as B, meshgen as mg

    t = time.perf_counter()
    prob = mg.CONFIGS[args.config]()
    log(f"mesh {args.config}: {prob.n_nodes} nodes, {prob.tets.shape[0]} tets "
        f"({time.perf_counter() - t:.1f} s)")
    if args.llg == "implicit":
        run_implicit(args, prob)
        return
    t = time.perf_counter()
    ctx = B.Context.from_problem(prob, device=0, precision=args.precision)
    n, uon, nou, bpe = ctx.query()
    log(f"setup: N'={n}, model bytes/eval={bpe / 1e9:.3f} GB ({time.perf_counter() - t:.1f} s)")
    m = torch.tensor(prob.m[nou], dtype=torch.float32, device="cuda")
    h = torch.empty_like(m)
    if args.copy_mib > 0:
        calibrate_counters(args.copy_mib)
    for _ in range(args.warmup):
        ctx.heff(m, h)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")
    # timed region: the evaluations alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.heff(m, h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    log(f"timed {args.steps} steps: {dt * 1e3:.4f} ms/step")
    # error of the timed run's output against the stored oracle values
    h_timed = h.clone()
    rel_err = sampled_error(ctx, prob, args.config, m, h_timed)
    if rel_err:
        log("error vs FP64 oracle at %d samples: " % rel_err["samples"]
            + " ".join(f"{k} {rel_err[k]['rel_l2']:.2e}/{rel_err[k]['rel_max']:.2e}"
                       for k in ("h_eff", "h_ex", "h_ms")) + " (rel L2 / rel max)")
    # the same number of evaluations again with a HIP event pair around every
    # kernel (on the stream it runs on): per-kernel durations for the roofline
    # (the events add gaps between kernels, so this pass is not the one timed)
    ctx.profile_begin(args.steps)
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ctx.heff(m, h)
    prof = ctx.profile_end()
    t3 = time.perf_counter()
    log(f"event pass {args.steps} steps: {(t3 - t2) / args.steps * 1e3:.4f} ms/step")
    # a plain stream of known size on the same GPU (elementwise: 512 MiB read
    # + 512 MiB written), the practical counterpart of the spec peak
    src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(10):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    stream_gbs = 2 * src.numel() * 4 / ((time.perf_counter() - t4) / 10) / 1e9
    del src, dst
    log(f"plain stream (elementwise, read + write): {stream_gbs:.0f} GB/s")
    kb = kernel_bytes(ctx, list(prof), args.precision)
    per_kernel = {k: (ms / max(c, 1), c) for k, (ms, c) in prof.items()}
    for k, (avg, c) in per_kernel.items():
        gbs = kb[k] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        log(f"  {k:14s} {avg * 1e3:9.2f} us  {kb[k] / 1e6:9.2f} MB  {gbs:8.1f} GB/s  x{c}")
    dom = max(per_kernel, key=lambda k: per_kernel[k][0])
    avg_ms = per_kernel[dom][0]
    achieved = kb[dom] / (avg_ms * 1e-3) / 1e9
    storage = {0: "fp32", 1: "bf16", 2: "bf16 hi+lo"}[args.precision]
    result = {
        "metric": ("H_eff evals/s at 1M nodes (plain FP32)" if args.precision == 0 else
                   f"H_eff evals/s at 1M nodes (FP32 arithmetic, {storage} grid storage)"),
        "value": 1.0 / dt,
        "unit": "H_eff evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{WORKLOADS.get(args.config, args.config)}, "
                         f"N'={n} unknowns, {prob.tets.shape[0]} tets, AIM grid "
                         f"{'x'.join(str(g) for g in prob.grid)}, p={prob.order_p}, "
                         f"r_b={prob.near_boxes}, kappa={prob.z0_radius:g}"),
            "name": args.config,
            "grid_storage": storage,
            "n_unknowns": n,
            "model_bytes_per_eval": bpe,
            "model_gbs": bpe / dt / 1e9,
            "kernels_us": {k: round(v[0] * 1e3, 3) for k, v in per_kernel.items()},
        },
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "stream_gbs": stream_gbs,
            "stream_frac": achieved / stream_gbs,
            "traffic": (measured_traffic(dom)
                        if args.config == "composite_c3" and args.precision == 0 else None),
        },
        "rel_err": rel_err,
    }
    if rank == 0 and not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle, bounded sample) ...")
        try:
            result["cpu_baseline"] = cpu_baseline(prob)
        except Exception as e:  # report, never hide the GPU number
            result["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
