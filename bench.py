"""Throughput benchmark: B_eff evaluations x cells per second on one MI355X.

Workload: the 1024 x 1024 x 1 film of 2 nm cells (Msat 8e5 A/m, Aex 1.3e-11
J/m, alpha 0.01, 10 mT along x) starting from a vortex with 1 % noise,
advanced by Dormand-Prince RK45 steps with MaxErr 1e-5 under device-side step
control.  One benchmark step = one RK45 attempt = 6 fused B_eff + torque
evaluations (demag FFT convolution, exchange, anisotropy, Zeeman, torque,
stage combine, error norm).  Following the paper's protocol (appendix
"Benchmark: throughput"), throughput = cells x evaluations / wall time of the
timed attempts, which run without instrumentation.  A second pass of the same
number of attempts has every field-pass launch record HIP events at its own
start and end; those durations give the per-kernel figures and the roofline
fraction of the dominant kernel.

Prints one JSON line.  --gpus N > 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Beff evals·cells/s: plain FP32 vs MFMA/surrogate at ≤1e-4 rel demag error"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1406_7635_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "film1024_rk45_hbm_traffic.txt")
DEVICE_WARMUP_S = 0.3  # untimed attempts on a scratch state before the warm-up attempts
REPEAT_WINDOWS = 5     # timed windows of the film (the first one is `value`)


# the sources the single-grid field kernels are compiled from (kernels,
# device bodies, FFT core, epilogue, argument structures)
PLAIN_KERNEL_SOURCES = ("kernels_fft.hip", "fft_passes.h", "fft_core.h", "field_epilogue.h", "mm_internal.h")


def kernel_source_digest():
    """SHA-256 over the sources of the single-grid field kernels: measured
    traffic is only reported while the kernels are the ones it was taken on."""
    h = hashlib.sha256()
    for name in PLAIN_KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, n):
    """HBM bytes per launch from a rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (lines 'source_sha256 <hex>', 'grid <n>' and 'traffic_bytes <pass> <bytes>');
    {} when absent, taken on another film size or on other kernel sources."""
    if not path or not os.path.exists(path):
        return {}
    digest, grid, out = None, None, {}
    with open(path) as fh:
        for line in fh:
            w = line.split()
            if len(w) == 2 and w[0] == "source_sha256":
                digest = w[1]
            elif len(w) == 2 and w[0] == "grid":
                grid = int(w[1])
            elif len(w) == 3 and w[0] == "traffic_bytes":
                out[w[1]] = float(w[2])
    if digest != kernel_source_digest() or grid != n:
        return {}
    return out


def column_pass_bytes(ctx):
    """Algorithmic HBM bytes of one launch of the y convolution pass (2D):
    read + write of the interleaved spectrum (3 complex64 per (y < ny, kx))
    and one read of the FP32 kernel octant (4 components per (kx, ky <= py/2))."""
    info = ctx.info()
    nx, ny, nz = ctx.grid
    spec = 3 * 8 * info["kx"] * ny * nz
    khat = 4 * info["khat_elems"]
    return 2 * spec + khat


def spectrum_bytes(ctx):
    """Half spectrum of the three components (complex64 per (kx, y, z))."""
    info = ctx.info()
    nx, ny, nz = ctx.grid
    return 3 * 8 * info["kx"] * ny * nz


def xinv_pass_bytes(ctx, k_reads):
    """x-inverse + field/torque pass of the last stage: read the spectrum, m_s,
    the region map and k_reads stage derivatives (error norm); write the torque."""
    n = int(np.prod(ctx.grid))
    return spectrum_bytes(ctx) + (12 + 1 + 12 * k_reads + 12) * n


def xfwd_pass_bytes(ctx, k_reads):
    """x-forward pass: read m0, the region map and k_reads stage derivatives,
    write m_s and the spectrum."""
    n = int(np.prod(ctx.grid))
    return (12 + 1 + 12 * k_reads + 12) * n + spectrum_bytes(ctx)


def xrow_pass_bytes(ctx, k_reads):
    """Fused x-inverse of stage s + x-forward of stage s+1: read the spectrum,
    m_s, the region map, m0 and k_reads derivatives (k_s itself stays on chip);
    write k_s, m_{s+1} and the spectrum."""
    n = int(np.prod(ctx.grid))
    return 2 * spectrum_bytes(ctx) + (12 + 1 + 12 + 12 + 12 * k_reads + 12) * n


# Dormand-Prince 5(4) per attempt: the first x-forward combines k0 only, the
# five fused passes read 1, 2, 3, 4, 4 earlier derivatives from HBM (the last
# term of each combine is the one just computed), and the error norm of the
# last stage reads 5 derivatives (e_1 = 0; e_6 multiplies the torque just
# computed).
DP45_XROW_K = (1 + 2 + 3 + 4 + 4) / 5.0


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(case, reps=5):
    """The FP64 oracle timed on this host: the median of `reps` B_eff + torque
    evaluations of the same state (after one untimed evaluation that pays
    scipy's plan setup), scipy.fft with one worker per host thread."""
    from oracle import fields as ofields

    t_init = time.perf_counter()
    prob = ofields.Problem(case["grid"], case["cell"], case["region"], case["params"], workers=-1)
    t_init = time.perf_counter() - t_init
    m = case["m0"].astype(np.float64)
    prob.torque(m)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        prob.torque(m)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    ncell = int(np.prod(case["grid"]))
    threads = os.cpu_count()
    return {"value": ncell / med, "unit": "Beff evals*cells/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "median_eval_s": med, "eval_s": times, "kernel_init_s": t_init,
            "sample": "median of %d FP64 B_eff+torque evaluations of the %dx%dx%d vortex state (scipy.fft with "
                      "%d workers); the oracle's demag tensor set-up (%.1f s) not included"
                      % (reps, case["grid"][0], case["grid"][1], case["grid"][2], threads, t_init)}


def oracle_timing(reps=5):
    """The FP64 oracle timed on this host for the three parity states: the
    32x32x4 RK4 film, the 1024x1024x1 vortex film and the 256x256x64 grains
    (median of `reps` B_eff + torque evaluations each, tensor set-up apart)."""
    from paper_1406_7635_amd import synth

    out = {"kind": "oracle", "unit": "Beff evals*cells/s", "cores": os.cpu_count(), "cpu_model": cpu_model()}
    for name, case in (("film32x32x4", synth.parity_cube(seed=1)), ("vortex1024", synth.vortex_film(seed=2, n=1024)),
                       ("grains256x256x64", synth.grains(seed=3))):
        r = cpu_baseline(case, reps)
        out[name] = {k: r[k] for k in ("value", "median_eval_s", "eval_s", "kernel_init_s")}
        print("oracle %s: %.3g cell evals/s, median %.3f s, set-up %.1f s" % (name, r["value"], r["median_eval_s"],
                                                                            r["kernel_init_s"]), flush=True)
    return out


def periodic_variant(n, steps, warmup):
    """The vortex film made periodic in x and y (one image per side): the
    periodic axes are transformed at their own length (no zero padding), so
    every transform is half as long and the spectrum a quarter of the open
    film's.  Dormand-Prince throughput from the vortex state."""
    import torch

    from paper_1406_7635_amd import mm, synth

    case = synth.vortex_film(seed=2, n=n)
    ncell = int(np.prod(case["grid"]))
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"], pbc=(1, 1, 0))
    info = ctx.info()
    m = torch.from_numpy(case["m0"]).cuda()
    opts = mm.solver_opts(max_err=1e-5)
    t, dt, _ = ctx.run(m, float("inf"), dt=1e-14, max_attempts=warmup, opts=opts)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t, dt, st = ctx.run(m, float("inf"), t=t, dt=dt, max_attempts=steps, opts=opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.close()
    return {"value": ncell * st["evals"] / wall, "unit": "Beff evals*cells/s", "ms_per_attempt": 1e3 * wall / steps,
            "attempts": steps, "accepted": st["steps"], "padded": [info["px"], info["py"], info["pz"]],
            "workload": "vortex film %dx%dx1 periodic in x and y (1 image per side), 2 nm cells; RK45 MaxErr 1e-5; "
                        "plain FP32, periodic axes unpadded" % (n, n),
            "dtype": "f32"}


def mfma_variants(ctx, m, opts, ncell, steps):
    """The same RK45 attempts with the y-convolution DFT stages on the matrix
    cores (BF16 / FP16 split precision): throughput, column-pass duration and
    the relative B_demag difference to the FP32 path at the current state (the
    error against the FP64 oracle is established by the parity tests)."""
    import torch

    res = {}
    ctx.set_conv_precision("fp32")
    _, b32 = ctx.beff(m, want_demag=True)
    b32 = b32.double()
    for prec in ("bf16", "fp16"):
        ctx.set_conv_precision(prec)
        _, bd = ctx.beff(m, want_demag=True)
        diff = float((bd.double() - b32).abs().max() / b32.abs().max())
        mm_ = m.clone()
        t, dt, _ = ctx.run(mm_, float("inf"), dt=1e-14, max_attempts=20, opts=opts)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t, dt, st = ctx.run(mm_, float("inf"), t=t, dt=dt, max_attempts=steps, opts=opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ctx.timing_enable(1)
        ctx.run(mm_, float("inf"), t=t, dt=dt, max_attempts=max(1, steps // 4), opts=opts)
        n, ms = ctx.timing_read(1)
        ctx.timing_enable(1, False)
        res["mfma_" + prec] = {"value": ncell * st["evals"] / wall, "ms_per_step": 1e3 * wall / steps,
                               "column_conv_avg_us": 1e3 * ms / max(n, 1), "demag_rel_diff_vs_fp32": diff,
                               "dtype": prec + " split (hi*hi + hi*lo + lo*hi), f32 accumulate"}
    ctx.set_conv_precision("fp32")
    return res


def copy_bandwidth(reps=20):
    """Achieved HBM bandwidth of a plain 256 MiB device-to-device copy (read +
    write bytes / time), the practical ceiling the roofline fraction is also
    stated against."""
    import torch

    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def ensemble_attempt_bytes(members):
    """Algorithmic HBM bytes of one Dormand-Prince attempt of every member of
    an ensemble (the pass model above, per member: x-forward, five fused
    x passes, x-inverse with the error norm, finalisation; six column stages:
    the y convolution in 2D, the one-pass y/z convolution of thin 3D grids,
    else y-forward + z convolution + y-inverse)."""
    def pad(n):
        return 1 if n == 1 else 1 << (2 * n - 2).bit_length()

    tot = 0.0
    for c in members:
        nx, ny, nz = c["grid"]
        px, py, pz = pad(nx), pad(ny), pad(nz)
        kx = px // 2 + 1
        n = nx * ny * nz
        spec = 3 * 8 * kx * ny * nz
        x = ((12 + 1 + 12 + 12) * n + spec) + 5 * (2 * spec + (12 + 1 + 12 + 12 + 12 * DP45_XROW_K + 12) * n) \
            + (spec + (12 + 1 + 12 * 5 + 12) * n) + 24 * n
        if pz == 1:
            col = 2 * spec + 4 * 4 * kx * (py // 2 + 1)
        elif pz in (4, 8) and py * pz <= 4096:
            # thin grid: one pass per kx column (y FFT, z convolution with the kernel
            # in z space: 4 + 6 (pz/2 - 1) floats per (kx, ky_h), inverse y FFT)
            col = 2 * spec + 4 * (4 + 6 * (pz // 2 - 1)) * kx * (py // 2 + 1)
        else:
            yf = 3 * 8 * kx * nz * (ny + py)
            zc = 2 * 3 * 8 * kx * py * nz + 4 * 6 * kx * (py // 2 + 1) * (pz // 2 + 1)
            col = 2 * yf + zc
        tot += x + 6 * col
    return tot


def ensemble_variant(steps, warmup, n=512):
    """The 512-member ensemble (nx, ny in {32..256}, nz in {1, 2}, DP45): every
    pass one persistent launch over all members, attempts replayed as a graph,
    persistent grids tuned first; also the same attempts with one workgroup per
    tile and with direct launches."""
    import torch

    from paper_1406_7635_amd import mm, synth

    members = synth.ensemble(n=n, seed=4)
    b = mm.Batch(members)
    ncell = np.array(b.ncells, dtype=np.float64)
    m = b.pack([c["m0"] for c in members])
    b.start(45, 0.0, 1e-14, members[0]["t_end"], mm.solver_opts(max_err=1e-5))

    def timed(k):
        s0 = b.stats_all()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        na, act = b.run(m, k)
        wall = time.perf_counter() - w0
        s1 = b.stats_all()
        cell_evals = float(np.sum(ncell * (s1["evals"] - s0["evals"])))
        return cell_evals / wall, wall, na, act, int(np.sum(s1["steps"] - s0["steps"])), \
            int(np.sum(s1["rejects"] - s0["rejects"]))

    b.run(m, max(1, warmup))
    untuned = timed(max(1, steps // 4))
    grids = b.autotune(m)
    tiles = {p: b.get_tile(p) for p in ("x", "conv2d")}
    b.run(m, max(1, warmup))
    val, wall, na, act, acc, rej = timed(steps)
    b.set_graph(False)
    direct = timed(max(1, steps // 4))
    b.set_graph(True)
    bytes_att = ensemble_attempt_bytes(members)
    gbs = bytes_att * na / wall / 1e9
    b.close()
    return {"value": val, "unit": "Beff evals*cells/s", "members": n, "cells": int(ncell.sum()),
            "attempts": na, "ms_per_attempt": 1e3 * wall / na, "accepted_steps": acc, "rejected_steps": rej,
            "running_after": act, "alg_bytes_per_attempt": bytes_att, "alg_GBs": gbs,
            "alg_frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "persistent_grids": grids, "tile_shapes": tiles,
            "untuned_value": untuned[0], "direct_launch_value": direct[0],
            "workload": "512 independent sims: nx, ny from {32,64,128,256}, nz from {1,2}, cubic cells "
                        "U(2,5) nm, Msat U(4e5,1.2e6), Aex U(5e-12,2e-11), alpha U(0.005,0.5), random m0, "
                        "no field; DP45 MaxErr 1e-5 towards 1 ns (timed window of %d attempts)" % steps,
            "dtype": "f32"}


def size_sweep():
    """The paper's throughput workload (n x n x 1, 4 nm cells, Msat 8e5, Aex
    13e-12, alpha 0.01, B_ext 10 mT along y, m along x, RK45) for the powers of
    two n = 16 ... 1024: cell evaluations per second against n (each point
    about 0.1 s of attempts)."""
    import torch

    from paper_1406_7635_amd import mm, synth

    out = {}
    for n in (16, 32, 64, 128, 256, 512, 1024):
        case = synth.paper_bench(n)
        ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"])
        m = torch.from_numpy(case["m0"]).cuda()
        opts = mm.solver_opts(max_err=1e-5)
        t, dt, _ = ctx.run(m, float("inf"), dt=1e-14, max_attempts=10, opts=opts)
        k = int(min(3000, max(20, 4e7 / (n * n))))
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t, dt, st = ctx.run(m, float("inf"), t=t, dt=dt, max_attempts=k, opts=opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        out[str(n)] = {"value": n * n * st["evals"] / wall, "ms_per_attempt": 1e3 * wall / k, "attempts": k}
        ctx.close()
    return {"unit": "Beff evals*cells/s", "points": out,
            "workload": "n x n x 1, 4 nm cells, Msat 8e5, Aex 13e-12, alpha 0.01, B_ext (0, 10 mT, 0), "
                        "m = x; RK45 MaxErr 1e-5; plain FP32", "dtype": "f32"}


def grains_variant(steps, warmup):
    """The 3D workload: 256 x 256 x 64 cells of 3 nm, 256 Voronoi grains
    (random m, the worst-case spectrum), Dormand-Prince with the column passes
    (y forward, z convolution, y inverse) in FP32 and with their DFT stages on
    the matrix cores (BF16 / FP16 split precision): throughput of each from the
    same state, the three-pass path's algorithmic bytes, and each matrix-core
    form's B_demag difference from the FP32 path at that state."""
    import torch

    from paper_1406_7635_amd import mm, synth

    case = synth.grains(seed=3)
    ncell = int(np.prod(case["grid"]))
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"])
    m0 = torch.from_numpy(case["m0"]).cuda()
    opts = mm.solver_opts(max_err=1e-5)
    b_att = ensemble_attempt_bytes([case])
    out = {}
    bd32 = None
    for prec in ("fp32", "bf16", "fp16"):
        ctx.set_conv_precision(prec)
        m = m0.clone()
        _, bd = ctx.beff(m, want_demag=True)
        if prec == "fp32":
            bd32 = bd
        diff = float((bd - bd32).abs().max() / bd32.abs().max())
        t, dt, _ = ctx.run(m, float("inf"), dt=1e-14, max_attempts=warmup, opts=opts)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t, dt, st = ctx.run(m, float("inf"), t=t, dt=dt, max_attempts=steps, opts=opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        gbs = b_att * steps / wall / 1e9
        out[prec] = {"value": ncell * st["evals"] / wall, "ms_per_attempt": 1e3 * wall / steps,
                     "attempts": steps, "accepted": st["steps"], "alg_GBs": gbs,
                     "alg_frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "demag_rel_diff_vs_fp32": diff}
    ctx.close()
    res = dict(out["fp32"])
    res.update({"unit": "Beff evals*cells/s", "alg_bytes_per_attempt": b_att,
                "matrix_core": {"bf16": out["bf16"], "fp16": out["fp16"]},
                "workload": "256x256x64 grains, 3 nm cells, 256 Voronoi regions (Msat U(6e5,1e6), Ku1 U(0,5e5), "
                            "S 0.9), random m; DP45 MaxErr 1e-5; column passes FP32 (value) and matrix-core "
                            "split BF16 / FP16",
                "dtype": "f32"})
    return res


# the uncoupled Heun path moves m (12 B read, 12 B written) and the region
# (1 B) once per launch of up to this many steps; the rest is arithmetic
HEUN_UNCOUPLED_BYTES_PER_CELL_PER_LAUNCH = 25
HEUN_UNCOUPLED_CHUNK = 4096


def thermal_variant(steps, warmup):
    """The paper's thermal-switching workload (figure figSwitch): 512 x 512
    uncoupled 10 nm cubes, Msat 1 MA/m, alpha 0.1, Ku1 1e4 J/m^3 along z, no
    demag, Heun at the fixed step 1e-12 s with Brown's thermal field at 90.5 K
    (KV/kT = 8).  Throughput in field evaluations x cells per second (two per
    step).  The cells do not interact, so the library runs whole chunks of
    steps per launch with each cell's state in registers: the path is bound by
    arithmetic (the generator, Box-Muller and two torques per step), not HBM."""
    import torch

    from paper_1406_7635_amd import mm, synth

    n, cell, ku = 512, 10e-9, 1e4
    params = synth.material(1e6, 0.0, alpha=0.1, ku1=ku, anis_u=(0.0, 0.0, 1.0))
    ctx = mm.Context((n, n, 1), (cell,) * 3, np.zeros((1, n, n), np.uint8), params, demag=False)
    ctx.set_temperature(ku * cell ** 3 / 8.0 / 1.380649e-23, 1)
    m = torch.zeros((3, 1, n, n), dtype=torch.float32, device="cuda:0")
    m[2] = 1.0
    dt = 1e-12
    t, _, _ = ctx.run(m, float("inf"), dt=dt, solver=12, max_attempts=warmup)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t, _, st = ctx.run(m, float("inf"), t=t, dt=dt, solver=12, max_attempts=steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    # the paper's check (Eq. eqSwitch): after 10 ns inside the wells, the
    # population difference decays as exp(-2 f t) over 0.2 us
    kt = ku * cell ** 3 / 8.0
    ctx.set_temperature(kt / 1.380649e-23, 2024)
    m.zero_()
    m[2] = 1.0
    t, _, _ = ctx.run(m, 10e-9, dt=dt, solver=12)
    mz1 = float(m[2].double().mean())
    t, _, _ = ctx.run(m, t + 0.2e-6, t=t, dt=dt, solver=12)
    mz2 = float(m[2].double().mean())
    f_meas = -math.log(mz2 / mz1) / (2 * 0.2e-6)
    alpha, msat, gamma = 0.1, 1e6, 1.7595e11
    f_th = gamma * alpha / (1 + alpha ** 2) * math.sqrt(8 * ku ** 3 * cell ** 3 / (2 * math.pi * msat ** 2 * kt)) \
        * math.exp(-ku * cell ** 3 / kt)
    ctx.close()
    ncell = n * n
    launches = -(-steps // HEUN_UNCOUPLED_CHUNK)
    gbs = HEUN_UNCOUPLED_BYTES_PER_CELL_PER_LAUNCH * ncell * launches / wall / 1e9
    return {"value": ncell * st["evals"] / wall, "unit": "Beff evals*cells/s (uncoupled cells, no demag)",
            "us_per_step": 1e6 * wall / steps,
            "comparable_to_metric": False,
            "steps": st["steps"], "cell_steps_per_s": ncell * steps / wall, "bound": "alu",
            "alg_GBs": gbs, "path": "uncoupled cells: one launch per chunk of up to %d steps" % HEUN_UNCOUPLED_CHUNK,
            "switching_rate_per_s": f_meas, "eq_switch_rate_per_s": f_th,
            "workload": "512x512 uncoupled 10 nm cubes, Msat 1e6, alpha 0.1, Ku1 1e4 (z), no demag; Heun, fixed "
                        "dt 1e-12 s, thermal field at KV/kT = 8 (90.5 K)",
            "dtype": "f32"}


def surrogate_variant(steps, warmup):
    """The surrogate workload: 256 x 256 x 1 film of 4 nm cells (Msat 8e5,
    Aex 1.3e-11, alpha 0.01), trained weights.  Reports the surrogate's
    relative B_demag error (max over cells, against the exact FP32 field) on
    held-out textures, the durations of one surrogate evaluation and of one
    exact field evaluation, the Dormand-Prince throughput with surrogate
    stages at the 1e-4 tolerance (falls back to the exact path on the first
    miss) and with the check disabled (every attempt keeps the surrogate)."""
    import torch

    from paper_1406_7635_amd import mm, sno_train, synth

    n, cell, msat = 256, 4e-9, 8e5
    ncell = n * n
    params = synth.material(msat, 1.3e-11, alpha=0.01)
    region = np.zeros((1, n, n), dtype=np.uint8)
    w = sno_train.load_weights()
    ctx = mm.Context((n, n, 1), (cell, cell, cell), region, params)
    sur = mm.Surrogate(n, n, w, 4e-7 * np.pi * msat)
    errs = []
    for m0 in synth.film_textures(24, seed=6, grid=(n, n), cell=cell):
        m = torch.from_numpy(m0).cuda()
        _, bd = ctx.beff(m, want_demag=True)
        bs = sur(m)
        errs.append(float((bs - bd).norm(dim=0).max() / bd.norm(dim=0).max()))
    m = torch.from_numpy(synth.film_textures(2, seed=7, grid=(n, n), cell=cell)[1]).cuda()  # a vortex
    out = torch.empty_like(m)

    def per_call_us(fn, reps=50):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 1e3 * e0.elapsed_time(e1) / reps

    sno_us = per_call_us(lambda: sur(m, out))
    exact_us = per_call_us(lambda: ctx.beff(m))

    def run(tol):
        ctx.set_surrogate(sur if tol is not None else None, tol if tol is not None else 1.0)
        mm_ = m.clone()
        t, dt, _ = ctx.run(mm_, float("inf"), dt=1e-14, max_attempts=warmup, opts=mm.solver_opts(max_err=1e-5))
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t, dt, st = ctx.run(mm_, float("inf"), t=t, dt=dt, max_attempts=steps, opts=mm.solver_opts(max_err=1e-5))
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        return ncell * st["evals"] / wall, ctx.surrogate_stats()

    plain, _ = run(None)
    at_tol, st_tol = run(1e-4)
    forced, st_forced = run(1e30)
    ctx.set_surrogate(None)
    ctx.close()
    sur.close()
    return {"value": forced, "unit": "Beff evals*cells/s", "qualifies": bool(max(errs) <= 1e-4),
            "surrogate_rel_err_max": max(errs), "surrogate_rel_err_median": float(np.median(errs)),
            "sno_eval_us": sno_us, "exact_field_eval_us": exact_us,
            "value_at_tol_1e-4": at_tol, "fallbacks_at_tol_1e-4": st_tol["fallbacks"],
            "plain_value_same_film": plain, "surrogate_steps_forced": st_forced["surrogate_steps"],
            "workload": "256x256x1 film, 4 nm cells, Msat 8e5, Aex 1.3e-11, alpha 0.01; vortex texture; "
                        "DP45 MaxErr 1e-5, surrogate at stages 2-6, exact last stage; errors on 24 held-out "
                        "textures", "dtype": "bf16 weights, f32 arithmetic"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1024, help="film edge in cells")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble variant")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate variant")
    ap.add_argument("--no-grains", action="store_true", help="skip the 3D grain-workload variant")
    ap.add_argument("--no-sweep", action="store_true", help="skip the n x n x 1 size sweep")
    ap.add_argument("--no-thermal", action="store_true", help="skip the thermal-switching (Heun) variant")
    ap.add_argument("--no-periodic", action="store_true", help="skip the periodic-film variant")
    ap.add_argument("--grains-only", action="store_true",
                    help="only the 3D grain-workload variant (one JSON line; for profiling)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate variant (one JSON line; for profiling)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only the FP64 oracle's host timing on the 32x32x4, 1024^2 and 256x256x64 states")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the batched-ensemble variant (one JSON line; for profiling)")
    ap.add_argument("--traffic", default=TRAFFIC_FILE,
                    help="rocprofv3 traffic summary with measured HBM bytes per launch")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy 10 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1406_7635_amd import mm, synth

    torch.cuda.init()
    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4,
                          "launches": 10}))
        return
    if args.ensemble_only:
        print(json.dumps(ensemble_variant(max(4, args.steps // 10), max(2, args.warmup // 5))))
        return
    if args.oracle_timing:
        print(json.dumps(oracle_timing()))
        return
    if args.grains_only:
        print(json.dumps(grains_variant(max(5, args.steps // 20), max(2, args.warmup // 10))))
        return
    if args.surrogate_only:
        print(json.dumps(surrogate_variant(max(10, args.steps // 4), max(2, args.warmup // 4))))
        return
    case = synth.vortex_film(seed=2, n=args.n)
    ncell = int(np.prod(case["grid"]))
    ctx = mm.Context(case["grid"], case["cell"], case["region"], case["params"])
    m = torch.from_numpy(case["m0"]).to("cuda:0")
    opts = mm.solver_opts(max_err=1e-5)
    # bring the GPU to its steady clocks first: untimed attempts on a scratch
    # copy of m for about DEVICE_WARMUP_S (the state of the run below is not
    # touched; without this a short warm-up leaves every kernel a few per cent slow)
    mw = m.clone()
    w0 = time.perf_counter()
    while time.perf_counter() - w0 < DEVICE_WARMUP_S:
        ctx.run(mw, float("inf"), dt=1e-14, max_attempts=32, opts=opts)
        torch.cuda.synchronize()
    del mw
    t, dt, _ = ctx.run(m, float("inf"), dt=1e-14, max_attempts=max(1, args.warmup), opts=opts)
    # timed region: exactly `steps` RK45 attempts, no instrumentation
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    w0 = time.perf_counter()
    t, dt, st = ctx.run(m, float("inf"), t=t, dt=dt, max_attempts=args.steps, opts=opts)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = e0.elapsed_time(e1)
    evals = st["evals"]
    value = ncell * evals / wall
    # the same number of attempts again with every field-pass launch recording a
    # HIP event pair at its own start and end (on the context stream): the
    # per-kernel durations behind the roofline figures
    names = ("x_forward", "column_conv", "x_inverse", "x_row")
    for k in range(len(names)):
        ctx.timing_enable(k)
    t, dt, st2 = ctx.run(m, float("inf"), t=t, dt=dt, max_attempts=args.steps, opts=opts)
    torch.cuda.synchronize()
    per = {}
    for k, name in enumerate(names):
        n, ms = ctx.timing_read(k)
        ctx.timing_enable(k, False)
        if n:
            per[name] = {"launches": n, "avg_us": 1e3 * ms / n, "total_ms": ms}
    dominant = max(per, key=lambda k: per[k]["total_ms"])
    # four more uninstrumented windows of `steps` attempts: the spread of the
    # timed figure (value itself is the first window)
    windows = [value]
    for _ in range(REPEAT_WINDOWS - 1):
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        t, dt, st3 = ctx.run(m, float("inf"), t=t, dt=dt, max_attempts=args.steps, opts=opts)
        torch.cuda.synchronize()
        windows.append(ncell * st3["evals"] / (time.perf_counter() - r0))
    copy_gbs = copy_bandwidth()
    bytes_per_launch = {"x_forward": xfwd_pass_bytes(ctx, 1), "column_conv": column_pass_bytes(ctx),
                        "x_inverse": xinv_pass_bytes(ctx, 5), "x_row": xrow_pass_bytes(ctx, DP45_XROW_K)}
    for k in per:
        per[k]["alg_bytes"] = bytes_per_launch[k]
        per[k]["gbs"] = bytes_per_launch[k] / (per[k]["avg_us"] * 1e-6) / 1e9
    ach = per[dominant]["gbs"]
    traffic = measured_traffic(args.traffic, args.n).get(dominant)
    # whole path: the algorithmic bytes of one attempt (x-forward, 6 column
    # passes, 5 fused passes, x-inverse with the error norm, and the
    # commit's read + write of m) over the measured time per attempt
    path_bytes = (bytes_per_launch["x_forward"] + 6 * bytes_per_launch["column_conv"] +
                  5 * bytes_per_launch["x_row"] + bytes_per_launch["x_inverse"] + 24 * ncell)
    path_gbs = path_bytes / (wall / args.steps) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "Beff evals*cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "vortex film %dx%dx1, 2 nm cells, Msat 8e5, Aex 1.3e-11, alpha 0.01, "
                               "B_ext 10 mT x; RK45 MaxErr 1e-5; plain FP32 FFT demag" % (args.n, args.n),
                   "cells": ncell, "evals": evals, "accepted": st["steps"], "rejected": st["rejects"],
                   "evals_per_step": 6, "gpu_event_ms": gpu_ms,
                   "kernel_timing": "second pass of %d attempts, dispatch-recorded HIP events" % args.steps,
                   "device_warmup": "%.1f s of untimed attempts on a scratch copy of m before the %d warm-up "
                                    "attempts" % (DEVICE_WARMUP_S, args.warmup),
                   "repeats": {"windows": REPEAT_WINDOWS, "values": windows,
                               "median": float(np.median(windows)),
                               "note": "value is the first window; the others follow the kernel-timing pass"}},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": dominant,
                     "copy_GBs": copy_gbs, "frac_of_copy": ach / copy_gbs,
                     "path": {"alg_bytes_per_step": path_bytes, "achieved": path_gbs,
                              "frac": path_gbs / HBM_PEAK_GBS, "frac_of_copy": path_gbs / copy_gbs}},
        "kernels": per,
    }
    out["variants"] = mfma_variants(ctx, m, opts, ncell, args.steps)
    ctx.close()
    if not args.no_ensemble:
        out["variants"]["ensemble"] = ensemble_variant(max(4, args.steps // 10), max(2, args.warmup // 5))
    if not args.no_surrogate:
        out["variants"]["surrogate"] = surrogate_variant(max(10, args.steps // 4), max(2, args.warmup // 4))
    if not args.no_grains:
        out["variants"]["grains"] = grains_variant(max(5, args.steps // 20), max(2, args.warmup // 10))
    if not args.no_sweep:
        out["variants"]["size_sweep"] = size_sweep()
    if not args.no_periodic:
        out["variants"]["periodic"] = periodic_variant(args.n, args.steps, args.warmup)
    if not args.no_thermal:
        out["variants"]["thermal"] = thermal_variant(max(200, args.steps * 10), max(20, args.warmup))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
