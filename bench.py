#!/usr/bin/env python3
"""Throughput of the NUFFT Radon forward + adjoint projector on one MI355X.

One step = forward projection and adjoint (back-projection) of every slice
of a stack: by default 32 slices of 2560 x 2560 random-ellipse phantoms
(20 ellipses each), 1024 angles uniform in [0, pi), 2560 detector bins,
float32 data with complex64 intermediates.  Inputs are resident in device
memory before timing starts.

Prints one JSON line: slices/s, per-stage kernel times from HIP events
recorded on the library's stream during the timed steps, the roofline of
the dominant kernel against the algorithmic byte model, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adj Radon slices/s (2560², 1024 angles) & % HBM roofline; MBIR iters/s"
HBM_PEAK_GBS = 8000.0


def stage_bytes(n: int, nd: int, na: int, tile_entries: int) -> dict:
    """Algorithmic HBM bytes of each stage for one slice.

    Each pass reads and writes its operands once at storage precision, with
    the half-plane grid of G(G/2+1) complex64 values (G = 2N) and H = N_t/2+1
    points per half-line.  The interpolation reads the inscribed disc of the
    grid (pi/4 of it), writes the half-line values and reads them back for
    the radial transforms.  The spreading also reads its 4-byte point list.
    """
    G = 2 * n
    H = nd // 2 + 1
    half = G // 2 + 1
    return {
        "fwd_rows": 4 * n * n + 8 * n * half,
        "fwd_cols": 8 * n * half + 8 * G * half,
        "fwd_interp": 8 * G * half * math.pi / 4 + 16 * na * H + 4 * na * nd,
        "adj_radial": 4 * na * nd + 8 * na * H,
        "spread": 8 * na * H + 4 * tile_entries + 8 * G * half,
        "adj_cols": 8 * G * half + 8 * n * half,
        "adj_rows": 8 * n * half + 4 * n * n,
    }


KERNEL_SOURCES = ("radon_kernels.hip", "radon_kernels.hpp", "fft.hpp", "layout.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_radon_2560x1024.md")


def kernel_source_digest() -> str:
    """sha1 of the projector's kernel sources (the counters are stale once it changes)."""
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2304_12934_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stage: str, n: int, na: int, per_launch: float) -> float | None:
    """HBM bytes of one launch of `stage` from the committed counter summary.

    The summary holds FETCH_SIZE and WRITE_SIZE per dispatch (rocprofv3
    --pmc), each scaled by what the same counter reads for a device copy of
    known size, for one workload, one number of slices per launch and one
    version of the kernel sources; None when any of them differs.
    """
    if (n, na) != (2560, 1024) or not os.path.exists(TRAFFIC_FILE):
        return None
    digest, rows, slices = None, {}, None
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if line.startswith("source digest:"):
                digest = line.split(":", 1)[1].strip().strip("`")
            if line.startswith("slices per launch:"):
                slices = float(line.split(":", 1)[1])
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) >= 5 and cells[0] in ("fwd_rows", "fwd_cols", "fwd_interp", "adj_radial", "spread",
                                                "adj_cols", "adj_rows"):
                try:
                    rows[cells[0]] = float(cells[4])
                except ValueError:
                    pass
    if digest != kernel_source_digest() or slices != per_launch:
        return None
    return rows.get(stage)


def model_bytes_per_slice(n: int, nd: int, na: int) -> float:
    """Unfused pipeline model (forward + adjoint) of one slice."""
    G = 2 * n
    H = nd // 2 + 1
    half = G // 2 + 1
    fwd = 4 * n * n + 16 * n * half + 8 * G * half * (1 + math.pi / 4) + 16 * na * H + 4 * na * nd
    adj = 4 * na * nd + 16 * na * H + 16 * G * half + 16 * n * half + 4 * n * n
    return fwd + adj


def mbir_model_bytes(n: int, nd: int, na: int, nz: int) -> float:
    """Algorithmic bytes of one MBIR iteration over nz slices: the forward +
    adjoint model of every slice, the data b read once and five volumes
    streamed by the prior and the update (4 B each)."""
    return nz * (model_bytes_per_slice(n, nd, na) + 4 * na * nd + 20 * n * n)


def cpu_model() -> str | None:
    """The host CPU's model name (first "model name" line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(f64_slice, angles, n_det: int, n_angles_total: int, sample_angles: int) -> dict:
    """FP64 oracle on the host: forward + adjoint of one slice on a subset of angles."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import radon as ora
    idx = np.linspace(0, len(angles) - 1, sample_angles).round().astype(int)
    sub = angles[idx]
    t0 = time.perf_counter()
    s = ora.radon_fwd(f64_slice, sub, n_det)
    ora.radon_adj(s, sub, f64_slice.shape[0])
    dt = time.perf_counter() - t0
    per_slice = dt * n_angles_total / sample_angles
    blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
    threads = max([p.get("num_threads", 1) for p in blas] or [1])
    return {
        "value": 1.0 / per_slice,
        "unit": "slices/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"1 slice {f64_slice.shape[0]}^2, forward+adjoint on {sample_angles} of {n_angles_total} "
                   f"angles in {dt:.1f} s, extrapolated linearly in the angle count (cost exactly linear in it)"),
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
        "blas": ", ".join(sorted({f"{p.get('internal_api')} {p.get('version')}" for p in blas})) or None,
        "blas_threads": int(threads),
    }


MBIR_TUNING = {"batch_mb": 80, "streams": 3}


def mbir_leg(dev, n: int, nz: int, na: int, iters: int, timed: int) -> dict:
    """MBIR iterations/s on a 3D ellipsoid volume with Poisson data: the plain
    per-iteration entry (mbir_step) against the autograd path (DataFidelityFn +
    QGGMRFFn backward, then the update kernel), and the reconstruction error of
    each after `iters` iterations (relative L2 inside the inscribed cylinder)."""
    import numpy as np
    import torch

    import synth
    from paper_2304_12934_amd import MBIR, Plan, Prior, power_lipschitz

    vol = synth.ellipsoid_volume(4, n, nz, 20, device=dev).to(torch.float32).contiguous()
    # one 1280^2 slice per batch on three streams: 181 it/s against 175 with
    # the library's default (three 1280^2 slices per batch, two streams)
    plan = Plan.uniform_stack(n, n, synth.uniform_angles(na), nz, device=dev, tuning=MBIR_TUNING)
    b_true = plan.fwd(vol)
    scale = 2.0 / float(b_true.max())          # largest attenuation 2 (transmission ~13.5%)
    vol *= scale
    b_true *= scale
    b = torch.as_tensor(synth.poisson_log_data(b_true, synth.rng_for(4, 1), 1.0e4), dtype=torch.float32,
                        device=dev).contiguous()
    prior = Prior(lam=1.0)
    L_data = power_lipschitz(plan, 30)
    x_ = (torch.arange(n, device=dev, dtype=torch.float32) - n // 2)
    mask = ((x_[None, :] ** 2 + x_[:, None] ** 2) <= (n / 2) ** 2).to(torch.float32)

    def err(x):
        d = (x - vol) * mask
        return float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(vol * mask))

    out = {"volume": f"{nz} x {n}^2 random ellipsoids (20)", "n_angles": na, "data": "Poisson, 1e4 photons/bin",
           "iterations": iters, "prior": "qGGMRF p=1.2 sigma=1/0.7 c=1e-4 lambda=1, 26 neighbours",
           "tuning": MBIR_TUNING}
    gb = mbir_model_bytes(n, n, na, nz) / 1e9
    out["model_GB_per_iter"] = round(gb, 3)
    for name, fn in (("plain", "step"), ("autograd", "step_autograd"), ("graph", None)):
        # same iterations from the same start on every path; the graph path
        # replays a capture of `timed` plain steps
        m = MBIR(plan, b, prior, L_data=L_data)
        if fn is None:
            graph = m.capture(timed)
            step, per = graph.launch, timed
        else:
            step, per = getattr(m, fn), 1
        for _ in range(max(1, 2 // per)):         # warm-up (iterates restart below)
            step()
        m = MBIR(plan, b, prior, L_data=L_data)
        if fn is None:
            graph.close()
            graph = m.capture(timed)
            step = graph.launch
        else:
            step = getattr(m, fn)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(timed // per):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        for _ in range((iters - timed) // per):
            step()
        torch.cuda.synchronize()
        if fn is None:
            graph.close()
        ips = timed / dt
        out[f"iters_per_s_{name}"] = round(ips, 2)
        out[f"frac_of_hbm_peak_{name}"] = round(gb * ips / HBM_PEAK_GBS, 4)
        out[f"recon_rel_err_{name}"] = round(err(m.x), 5)
        out[f"restarts_{name}"] = m.restarts
    plan.close()
    out["prior_alone"] = prior_alone(dev, vol, prior)
    torch.cuda.synchronize()
    return out


# The prior gradient is bound by arithmetic: per voxel 13 neighbour pairs
# (plus 8 % of pairs recomputed at strip edges), each 9.3 full-rate VALU
# instructions and 3 transcendental ones (exp2, log2, reciprocal) that cost
# about 1.9 full-rate issue slots each; the VALU issues one instruction per
# lane per cycle on 256 CUs x 64 lanes at 2.4 GHz.
QG_SLOTS_PER_VOXEL = 13 * 1.08 * (9.3 + 3 * 1.9)
VALU_LANE_SLOTS_PER_S = 256 * 64 * 2.4e9


def prior_alone(dev, vol, prior, calls: int = 10) -> dict:
    """The qGGMRF gradient alone on an MBIR volume, timed with HIP events on
    the launch stream, against its ALU bound."""
    import torch

    from paper_2304_12934_amd import qggmrf_grad

    grad = torch.zeros_like(vol)
    for _ in range(2):
        qggmrf_grad(vol, prior, 1.0, grad)
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(calls):
        qggmrf_grad(vol, prior, 1.0, grad)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    vox = vol.numel()
    bound_ms = vox * QG_SLOTS_PER_VOXEL / VALU_LANE_SLOTS_PER_S * 1e3
    del grad
    return {"ms_per_call": round(ms, 4), "bound": "alu", "alu_bound_ms": round(bound_ms, 4),
            "frac_of_alu_bound": round(bound_ms / ms, 4), "hbm_GB_per_s": round(12 * vox / ms / 1e6, 1),
            "hbm_frac": round(12 * vox / ms / 1e6 / HBM_PEAK_GBS, 4)}


# Full sparse-view MBIR: 128 slices of 2560^2, 361 angles, 30 ellipsoids with
# 12 blurred cracks, Gaussian noise of 1 % of the largest datum, 100
# iterations over the resident stack (the prior couples adjacent slices).
CONFIG5_LAMBDA = 300.0   # the reconstruction error falls through the 100 iterations


def config5_leg(dev, iters: int = 100) -> dict:
    import torch

    import synth
    from paper_2304_12934_amd import MBIR, Plan, Prior, power_lipschitz

    n, nz, na = 2560, 128, 361
    vol64 = synth.ellipsoid_volume(5, n, nz, 30, device=dev)
    vol = synth.add_cracks(vol64, synth.rng_for(5, 1), 12).to(torch.float32).contiguous()
    del vol64
    torch.cuda.empty_cache()
    plan = Plan.uniform_stack(n, n, synth.uniform_angles(na), nz, device=dev)
    b = torch.as_tensor(synth.gaussian_noise(plan.fwd(vol), synth.rng_for(5, 2), 0.01), dtype=torch.float32,
                        device=dev).contiguous()
    prior = Prior(lam=CONFIG5_LAMBDA)
    L_data = power_lipschitz(plan, 30)
    x_ = torch.arange(n, device=dev, dtype=torch.float32) - n // 2
    mask = ((x_[None, :] ** 2 + x_[:, None] ** 2) <= (n / 2) ** 2).to(torch.float32)

    def err(x):
        return float(torch.linalg.vector_norm((x - vol) * mask) / torch.linalg.vector_norm(vol * mask))

    m = MBIR(plan, b, prior, L_data=L_data)
    m.step()                                      # warm-up, then restart from zero
    m = MBIR(plan, b, prior, L_data=L_data)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.run(10)
    torch.cuda.synchronize()
    e10 = err(m.x)
    t1 = time.perf_counter()
    m.run(iters - 10)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) + (t1 - t0)
    gb = mbir_model_bytes(n, n, na, nz) / 1e9
    ips = iters / dt
    out = {"volume": f"{nz} x {n}^2, 30 ellipsoids + 12 cracks", "n_angles": na, "data": "Gaussian noise 1% of max",
           "iterations": iters, "lambda": CONFIG5_LAMBDA, "iters_per_s": round(ips, 2),
           "model_GB_per_iter": round(gb, 2), "frac_of_hbm_peak": round(gb * ips / HBM_PEAK_GBS, 4),
           "recon_rel_err_10": round(e10, 4), "recon_rel_err_final": round(err(m.x), 4), "restarts": m.restarts}
    del m
    torch.cuda.empty_cache()
    out["host_resident"] = host_mbir_leg(dev, plan, b, prior, L_data, n, nz, na)
    plan.close()
    del vol, b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def host_mbir_leg(dev, plan, b, prior, L_data: float, n: int, nz: int, na: int, chunk: int = 16,
                  iters: int = 3) -> dict:
    """The sparse-view workload with its iterates in host memory (pinned):
    mbir_stream_iterate streams chunks of `chunk` slices through the device
    each iteration.  Timed over `iters` iterations from zero, against the
    device-resident iterates after the same number of steps, and against the
    PCIe copy rates measured here."""
    import torch

    import synth
    from paper_2304_12934_amd import MBIR, HostMBIR, Plan

    plan_c = Plan.uniform_stack(n, n, synth.uniform_angles(na), chunk, device=dev)
    b_host = b.cpu().reshape(-1).pin_memory()
    m = HostMBIR(plan_c, b_host, nz // chunk, prior, L_data=L_data)
    m.step()                                      # warm-up, then restart from zero
    m.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.run(iters)
    dt = time.perf_counter() - t0
    ref = MBIR(plan, b, prior, L_data=L_data)
    ref.run(iters)
    torch.cuda.synchronize()
    x_ref = ref.x.cpu()
    diff = float(torch.linalg.vector_norm(m.x - x_ref) / torch.linalg.vector_norm(x_ref))
    del ref, x_ref
    # bytes over PCIe per iteration: x_k and x_{k-1} with their halo slices and
    # the data in, x_{k+1} out
    chunks = nz // chunk
    slices_in = 2 * (nz + 2 * (chunks - 1))
    gb_in = (slices_in * n * n + nz * na * n) * 4 / 1e9
    gb_out = nz * n * n * 4 / 1e9
    src = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32).pin_memory()
    dst = torch.empty(src.numel(), dtype=torch.float32, device=dev)
    rates = []
    for a, c in ((src, dst), (dst, src)):
        c.copy_(a, non_blocking=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            c.copy_(a, non_blocking=True)
        torch.cuda.synchronize()
        rates.append(3 * src.numel() * 4 / (time.perf_counter() - t) / 1e9)
    bound = 1.0 / max(gb_in / rates[0], gb_out / rates[1])
    out = {"chunk_slices": chunk, "chunks": chunks, "iterations": iters, "iters_per_s": round(iters / dt, 3),
           "GB_in_per_iter": round(gb_in, 2), "GB_out_per_iter": round(gb_out, 2),
           "h2d_GB_per_s": round(rates[0], 1), "d2h_GB_per_s": round(rates[1], 1),
           "pcie_bound_iters_per_s": round(bound, 3), "rel_diff_vs_resident": float(f"{diff:.3g}"),
           "restarts": m.restarts}
    plan_c.close()
    del m, b_host, src, dst
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# The paper's end-to-end timings (Sec. 5, Table "tab:runtimes": tomoCAM MBIR,
# 100 iterations, one machine with 4x Tesla P100 and 2x Xeon E5-2620 v4, data
# streamed from host memory) for the shapes that this projector supports; the
# 2448-wide dataset needs radix-17 transforms and is left out.
PAPER_SHAPES = (
    ("foam phantom", 2048, 16, 128, 93.0),
    ("TB-25", 2048, 128, 400, 862.0),
)


def paper_shapes_leg(dev, iters: int = 100) -> list:
    """100 plain MBIR iterations at the paper's dataset shapes (slices x N^2,
    angles), on synthetic ellipsoid volumes with Poisson data standing in for
    the paper's data, with the volume resident in HBM.  Context beside the
    paper's timings, not a target: different hardware, data and stopping."""
    import torch

    import synth
    from paper_2304_12934_amd import MBIR, Plan, Prior, power_lipschitz

    out = []
    for name, n, nz, na, paper_s in PAPER_SHAPES:
        vol = synth.ellipsoid_volume(6, n, nz, 20, device=dev).to(torch.float32).contiguous()
        plan = Plan.uniform_stack(n, n, synth.uniform_angles(na), nz, device=dev)
        b_true = plan.fwd(vol)
        scale = 2.0 / float(b_true.max())
        b_true *= scale
        b = torch.as_tensor(synth.poisson_log_data(b_true, synth.rng_for(6, nz), 1.0e4), dtype=torch.float32,
                            device=dev).contiguous()
        del vol, b_true
        prior = Prior(lam=1.0)
        L_data = power_lipschitz(plan, 30)
        m = MBIR(plan, b, prior, L_data=L_data)
        m.step()
        m = MBIR(plan, b, prior, L_data=L_data)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.run(iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.append({"dataset_shape": name, "slices": nz, "n": n, "n_angles": na, "iterations": iters,
                    "seconds": round(dt, 3), "slice_iters_per_s": round(nz * iters / dt, 1),
                    "paper_seconds": paper_s, "paper_hardware": "4x Tesla P100, 2x Xeon E5-2620 v4"})
        plan.close()
        del m, plan, b
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def batched_leg(dev, count: int, reps: int) -> dict:
    """Uneven stack: `count` slices with N in {512, 1024, 2048}, angle counts
    U[128, 1500] (half sparse with a random offset, half limited-view), N_t = N.
    Forward + adjoint of the whole stack as one HIP-graph launch of the batched
    plan, against per-slice launches (one slice per batch, no graph)."""
    import numpy as np
    import torch

    import synth
    from paper_2304_12934_amd import Plan, SliceGeometry

    geoms = [SliceGeometry(n, n, ang) for n, ang in synth.uneven_stack(synth.rng_for(3, 0), count)]
    from paper_2304_12934_amd.autotune import autotune
    tuning = autotune(geoms, device=dev, use_cache=False)
    plan = Plan(geoms, device=dev, tuning=tuning)
    per = Plan(geoms, device=dev, tuning={"batch": 1})
    vol = torch.empty(plan.vol_numel, dtype=torch.float32, device=dev)
    for i, g in enumerate(geoms):
        o = plan.vol_offsets[i]
        vol[o:o + g.n * g.n] = synth.ellipse_phantom(3, i, g.n, 20, device=dev).to(torch.float32).reshape(-1)
    sino = torch.empty(plan.sino_numel, dtype=torch.float32, device=dev)
    back = torch.empty(plan.vol_numel, dtype=torch.float32, device=dev)
    graph = plan.capture("fwd+adj", vol, sino, back)

    def t(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_graph = t(graph.launch)
    t_per = t(lambda: (per.fwd(vol, sino), per.adj(sino, back)))
    info = plan.info()
    graph.close()
    per.close()
    # the same pass with each batch as one persistent kernel over per-XCD work
    # queues (built for the 64x32 spreading tile), with the tuned batches and
    # with the whole stack as one batch (one launch)
    persistent = {}
    for label, extra in (("tuned_batches", {}), ("one_batch", {"batch_mb": 1 << 20, "streams": 1})):
        with Plan(geoms, device=dev, tuning={**tuning, "tile_w": 64, "tile_h": 32, "persistent": 1, **extra}) as pp:
            g2 = pp.capture("fwd+adj", vol, sino, back)
            t_p = t(g2.launch)
            pp.check()
            g2.close()
            persistent[label] = {"graph_slices_per_s": round(count / t_p, 1), "batches": pp.info()["batches"],
                                 "launches_per_pass": pp.info()["launches"]}
    plan.close()
    torch.cuda.synchronize()
    sizes = {n: sum(1 for g in geoms if g.n == n) for n in (512, 1024, 2048)}
    gb = sum(model_bytes_per_slice(g.n, g.n_det, len(g.angles)) for g in geoms) / 1e9
    def frac(seconds):   # model bytes of one pass over its time, against the HBM peak
        return round(gb / seconds / HBM_PEAK_GBS, 4)

    for v in persistent.values():
        v["frac_of_hbm_peak"] = frac(count / v["graph_slices_per_s"])
    return {"slices": count, "sizes": sizes, "angles_total": int(sum(len(g.angles) for g in geoms)),
            "model_GB_per_pass": round(gb, 3),
            "batched_graph_slices_per_s": round(count / t_graph, 1),
            "batched_graph_frac_of_hbm_peak": frac(t_graph),
            "per_slice_slices_per_s": round(count / t_per, 1),
            "per_slice_frac_of_hbm_peak": frac(t_per),
            "speedup": round(t_per / t_graph, 3), "tuning": tuning, "batches": info["batches"], "slots": info["slots"],
            "launches_per_pass": info["launches"], "persistent": persistent}


def device_copy_gbs(dev, stream, mib: int = 2048, reps: int = 5) -> float:
    """Bytes read plus written per second by a plain device-to-device copy of
    `mib` MiB (torch's copy kernel), timed with HIP events: the attainable
    HBM rate that the dominant kernel is also compared against."""
    import torch

    src = torch.ones(mib * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def ensure_built() -> None:
    """Build the library only when none is there (bench loads what is built)."""
    from paper_2304_12934_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2304_12934_amd import build
        build.build(verbose=False)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--slices", type=int, default=32)
    ap.add_argument("--n", type=int, default=2560)
    ap.add_argument("--angles", type=int, default=1024)
    ap.add_argument("--ellipses", type=int, default=20)
    ap.add_argument("--cpu-angles", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-stage events")
    ap.add_argument("--no-mbir", action="store_true", help="skip the MBIR iterations/s leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven-stack leg")
    ap.add_argument("--no-config5", action="store_true", help="skip the 128 x 2560^2 sparse-view MBIR leg")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the 100-iteration MBIR runs at the paper's dataset shapes")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the filtered back-projection and rotation-axis offset timings")
    ap.add_argument("--batched-slices", type=int, default=96)
    ap.add_argument("--mbir-n", type=int, default=1280)
    ap.add_argument("--mbir-slices", type=int, default=64)
    ap.add_argument("--mbir-angles", type=int, default=256)
    ap.add_argument("--mbir-iters", type=int, default=50)
    ap.add_argument("--tile-w", type=int, default=None, help="spreading tile width (plan tuning)")
    ap.add_argument("--tile-h", type=int, default=None, help="spreading tile height (plan tuning)")
    ap.add_argument("--chunk", type=int, default=None, help="points per spreading/interpolation item")
    ap.add_argument("--streams", type=int, default=None, help="concurrent streams of the plan (plan tuning)")
    ap.add_argument("--batch-mb", type=int, default=1400,
                    help="scratch budget of one batch in MiB (plan tuning; 1400: eight 2560^2 slices per launch)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run one device-to-device copy of MIB MiB before timing (a counter reference)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the projector shards along z with no exchange, see the design notes", file=sys.stderr)
        return 2

    ensure_built()
    import numpy as np
    import torch

    import synth
    from paper_2304_12934_amd import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, nd, na, S = args.n, args.n, args.angles, args.slices
    angles = synth.uniform_angles(na)

    t_gen = time.perf_counter()
    vol = torch.empty((S, n, n), dtype=torch.float32, device=dev)
    for z in range(S):
        vol[z] = synth.ellipse_phantom(2, z, n, args.ellipses, device=dev).to(torch.float32)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] phantoms {S} x {n}^2 in {t_gen:.1f} s", file=sys.stderr, flush=True)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.calibrate_copy} MiB", file=sys.stderr, flush=True)
        del src, dst

    tuning = {k: v for k, v in (("tile_w", args.tile_w), ("tile_h", args.tile_h), ("chunk", args.chunk),
                                ("streams", args.streams), ("batch_mb", args.batch_mb)) if v is not None}
    plan = Plan.uniform_stack(n, nd, angles, S, device=dev, tuning=tuning or None)
    info = plan.info(0)
    sino = torch.empty(plan.sino_shape(), dtype=torch.float32, device=dev)
    back = torch.empty(plan.vol_shape(), dtype=torch.float32, device=dev)

    def step():
        plan.normal(vol, None, sino, back)   # sino = R vol, back = R^T sino

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warm-up done", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream(dev)

    def timed_steps(k: int) -> float:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # the throughput: K plain steps
    w0 = time.perf_counter()
    ms_total = timed_steps(args.steps)
    wall = time.perf_counter() - w0
    ms_per_step = ms_total / args.steps
    value = S * args.steps / (ms_total / 1e3)
    print(f"[bench] {args.steps} steps in {ms_total:.1f} ms (wall {wall:.2f} s)", file=sys.stderr, flush=True)
    # the per-stage times: K more steps with HIP events around every stage launch
    stages = {}
    if not args.no_profile:
        plan.profile(True)
        ms_prof = timed_steps(args.steps)
        stages = plan.profile_read()
        plan.profile(False)
        print(f"[bench] {args.steps} profiled steps in {ms_prof:.1f} ms", file=sys.stderr, flush=True)

    sb = stage_bytes(n, nd, na, info["tile_entries"])
    per_launch_slices = S / max(1, info["batches"])      # slices covered by one stage launch
    stage_report = {}
    for name, (ms, launches) in stages.items():
        per_slice = ms / (args.steps * S)
        gbs = sb[name] / (per_slice * 1e-3) / 1e9 if name in sb else None
        stage_report[name] = {"ms_per_launch": round(ms / launches, 5), "ms_per_slice": round(per_slice, 5),
                              "launches": launches, "GB_per_s": round(gbs, 1) if gbs else None}
    roofline = None
    if stages:
        dom = max((k for k in stages if k in sb), key=lambda k: stages[k][0])
        # one stage launch covers one batch (the spreading stage is two kernels: clear + spread)
        per_ms = stages[dom][0] / (args.steps * max(1, info["batches"]))
        bytes_launch = sb[dom] * per_launch_slices
        achieved = bytes_launch / (per_ms * 1e-3) / 1e9
        tb = measured_traffic(dom, n, na, per_launch_slices)
        traffic = int(tb) if tb is not None else None
        copy_gbs = device_copy_gbs(dev, stream)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "bytes_per_launch": int(bytes_launch), "ms_per_launch": round(per_ms, 5),
                    "slices_per_launch": per_launch_slices,
                    "measured_copy_GB_per_s": round(copy_gbs, 1),
                    "frac_of_measured_copy": round(achieved / copy_gbs, 4)}

    mb = model_bytes_per_slice(n, nd, na)
    step_gbs = mb * S / (ms_per_step * 1e-3) / 1e9

    # the operators beside the metric, on the same stack: the plain adjoint,
    # filtered back-projection (adjoint with the ramp x Butterworth weight) and
    # forward + adjoint with the rotation axis 3.25 bins off centre
    extensions = None
    if not args.no_extensions:
        def rate(fn, k):
            for _ in range(2):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(k):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return round(S * k / (e0.elapsed_time(e1) / 1e3), 2)

        extensions = {"adj_slices_per_s": rate(lambda: plan.adj(sino, back), args.steps),
                      "fbp_butterworth_slices_per_s": rate(lambda: plan.fbp(sino, back, filter="butterworth"),
                                                           args.steps)}
        plan_c = Plan.uniform_stack(n, nd, angles, S, center=3.25, device=dev, tuning=tuning or None)
        extensions["fwd_adj_axis_offset_slices_per_s"] = rate(lambda: plan_c.normal(vol, None, sino, back),
                                                               args.steps)
        plan_c.close()
        del plan_c
        # a host-resident stack three times the device stack (the same slices
        # repeated), streamed through the GPU 8 slices per chunk, against the
        # PCIe copy rates that bound it (pinned host memory; the copies
        # overlap the computation)
        chunk = 8 if S % 8 == 0 else 1
        SH = 3 * S
        h_vol = vol.cpu().repeat(3, 1, 1).pin_memory()
        h_sino = torch.empty(3 * plan.sino_numel, dtype=torch.float32, pin_memory=True)
        # the chunk plan keeps the library's batch budget: one batch per slice,
        # so its two streams overlap within a chunk
        plan_s = Plan.uniform_stack(n, nd, angles, chunk, device=dev,
                                    tuning={k: v for k, v in tuning.items() if k != "batch_mb"} or None)

        def host_rate(fn, k=2):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                fn()
            torch.cuda.synchronize()
            return SH * k / (time.perf_counter() - t0)

        def copy_gbs(src, dst, k=3):
            dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
            return src.numel() * 4 * k / (time.perf_counter() - t0) / 1e9

        h2d = copy_gbs(h_vol[:S], vol)
        d2h = copy_gbs(sino.view(-1), h_sino[:plan.sino_numel])
        fwd_rate = host_rate(lambda: plan_s.stream("fwd", h_vol.view(-1), h_sino, sync=False))
        h_back = torch.empty(3 * plan.vol_numel, dtype=torch.float32, pin_memory=True)
        adj_rate = host_rate(lambda: plan_s.stream("adj", h_sino, h_back, sync=False))
        in_b, out_b = 4 * n * n, 4 * na * nd
        extensions["host_stream"] = {
            "slices": SH, "chunk": chunk, "h2d_GB_per_s": round(h2d, 1), "d2h_GB_per_s": round(d2h, 1),
            "fwd_slices_per_s": round(fwd_rate, 1), "adj_slices_per_s": round(adj_rate, 1),
            "fwd_pcie_bound_slices_per_s": round(min(h2d * 1e9 / in_b, d2h * 1e9 / out_b), 1),
            "adj_pcie_bound_slices_per_s": round(min(h2d * 1e9 / out_b, d2h * 1e9 / in_b), 1)}
        torch.cuda.synchronize()
        plan_s.close()
        del plan_s, h_vol, h_sino, h_back
        print(f"[bench] extensions {extensions}", file=sys.stderr, flush=True)

    # the main stack's plan is closed here, while the runtime is alive
    torch.cuda.synchronize()
    plan.close()
    mbir = None
    if not args.no_mbir:
        del vol, sino, back, plan
        torch.cuda.empty_cache()
        print("[bench] MBIR leg ...", file=sys.stderr, flush=True)
        mbir = mbir_leg(dev, args.mbir_n, args.mbir_slices, args.mbir_angles, args.mbir_iters, 10)
        print(f"[bench] MBIR {mbir}", file=sys.stderr, flush=True)

    config5 = None
    if not args.no_config5:
        torch.cuda.empty_cache()
        print("[bench] sparse-view MBIR leg (128 x 2560^2) ...", file=sys.stderr, flush=True)
        config5 = config5_leg(dev)
        print(f"[bench] sparse-view MBIR {config5}", file=sys.stderr, flush=True)

    paper = None
    if not args.no_paper_shapes:
        torch.cuda.empty_cache()
        print("[bench] paper-shape MBIR leg ...", file=sys.stderr, flush=True)
        paper = paper_shapes_leg(dev)
        print(f"[bench] paper shapes {paper}", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        torch.cuda.empty_cache()
        print("[bench] uneven-stack leg ...", file=sys.stderr, flush=True)
        batched = batched_leg(dev, args.batched_slices, 3)
        print(f"[bench] uneven {batched}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline ...", file=sys.stderr, flush=True)
        f64 = synth.ellipse_phantom(2, 0, n, args.ellipses).numpy()
        cpu = cpu_baseline(f64, angles, nd, na, args.cpu_angles)

    try:
        sha = subprocess.run(["git", "rev-parse", "--short", "HEAD"], cwd=ROOT, capture_output=True,
                             text=True).stdout.strip() or None
    except Exception:
        sha = None
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{S} slices {n}x{n} random ellipses ({args.ellipses} each), {na} angles in [0,pi), "
                               f"{nd} bins, forward+adjoint per slice",
                   "slices": S, "n": n, "n_angles": na, "n_det": nd, "kernel_width": 7, "oversampling": 2,
                   "parallelism": "none (1 GPU)", **({"tuning": tuning} if tuning else {})},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "model_bytes_per_slice": int(mb),
        "step_GB_per_s_vs_model": round(step_gbs, 1),
        "step_frac_of_hbm_peak": round(step_gbs / HBM_PEAK_GBS, 4),
        "stages": stage_report,
        "mbir": mbir,
        "mbir_sparse_view_2560": config5,
        "uneven_stack": batched,
        "paper_shapes_mbir": paper,
        "extensions": extensions,
        "wall_s": round(wall, 3),
        "git": sha,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
