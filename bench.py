#!/usr/bin/env python3
"""Forward + inverse shearlet filter-bank throughput on one MI355X.

Workload: batch 16 of 512x512 synthetic cartoon images plus N(0, 30^2)
noise, 4-scale system with shear levels (1, 1, 2, 2) -> 49 filters, FP32.
One step = shear_forward then shear_inverse of the whole batch (every step
of the hot path), inputs resident in HBM before the timed region.

Prints ONE JSON line: the throughput in Mpix*filters/s (B*N*M*K per step),
the roofline of the dominant kernel (per-launch hipEvents over the timed
region, on the stream the kernels run on), the whole-path roofline, and the
FP64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+inv shearlet Mpix·filters/s @512²×49 FP32; % of HBM roofline"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
B, N, M, J = 16, 512, 512, 4
SHEAR_LEVELS = [1, 1, 2, 2]
CONFIG_ID = 2  # seeds of the synthetic images (synth.cartoon_batch config)
SIGMA = 30.0
WORKLOAD = "fwd+inv, 16 x 512x512 cartoon+N(0,30^2) images, 4 scales (shear levels 1,1,2,2) = 49 filters, FP32"
METRIC_DENOISE = "denoise (fwd + hard threshold + inv) shearlet Mpix·filters/s @512²×49 FP32"
METRIC_LAYER = "layer fwd+bwd (shear_forward + shear_adjoint) shearlet Mpix·filters/s @256²×33 FP32"
WORKLOAD_LAYER = ("differentiable layer, forward and backward (upstream gradient N(0,1)), 32 x 1 x 256x256 "
                  "cartoon images, 3 scales (shear levels 1,1,2) = 33 filters, FP32")
WORKLOAD_DENOISE = ("hard-threshold denoising (threshold 3 x sigma x RMS_k on every plane), "
                    "16 x 512x512 cartoon+N(0,30^2) images, 49 filters, FP32")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_algorithmic_bytes(kind: str, K: int, real_filters: bool, plane_fwd: bool = False) -> float:
    """Algorithmic bytes per transform call of each kernel kind at this workload (a call with chunked
    launches splits these bytes evenly over its launches).

    The method must read x and the filter bank and write the coefficients in the
    forward transform, and read the coefficients and the filter bank and write
    the images in the inverse. Each of these compulsory transfers is attributed
    to the kernel that performs it; exchange intermediates count as overhead.
    With the whole-plane forward (plane_fwd), its plane kernel reads the filters and
    writes the coefficients, and the forward's column pass only forms the images'
    column spectra.
    """
    img = B * N * M * 4
    coef = B * K * N * M * 4
    filt = K * N * (M // 2 + 1) * (4 if real_filters else 8)
    return {
        "rows_r2c_images": img,
        "cols_fwd": 0 if plane_fwd else filt,
        "rows_c2r_coeffs": coef,
        "rows_r2c_coeffs": coef,
        "cols_inv": filt,
        "rows_c2r_images": img,
        "rows_thresh": 0,
        "plane_fwd": coef + filt,
    }[kind]


def exchange_bytes(kind: str, K: int, plane_fwd: bool = False) -> float:
    """Bytes of the packed exchange planes a kernel kind reads and writes per transform call
    (the intermediates between the row and column stages)."""
    plane = N * (M // 2) * 8
    return {
        "rows_r2c_images": B * plane,
        "cols_fwd": 2 * B * plane if plane_fwd else B * plane + B * K * plane,
        "rows_c2r_coeffs": B * K * plane,
        "rows_r2c_coeffs": B * K * plane,
        "cols_inv": B * K * plane + B * plane,
        "rows_c2r_images": B * plane,
        "rows_thresh": 2 * B * K * plane,
        "plane_fwd": B * plane,  # the images' column spectra
    }.get(kind, 0.0)


def path_algorithmic_bytes(K: int, real_filters: bool) -> float:
    """Whole fwd+inv step: x in, c out, c in, y out, filter bank read once per direction."""
    filt = K * N * (M // 2 + 1) * (4 if real_filters else 8)
    return B * (8 * N * M + 8 * K * N * M) + 2 * filt


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2006_04591_amd", "csrc", f) for f in ("kernels.hip", "fft_core.h")]
VALU_ISSUE_PEAK = 256 * 2.4e9  # wave64 VALU instructions per second: 256 CUs x 2.4 GHz x 1 per CU per clock


def source_digest(src=None) -> str:
    """sha256 over the transform kernels' sources (kernels.hip and fft_core.h), or over `src`."""
    h = hashlib.sha256()
    for path in ([src] if isinstance(src, str) and src else (src or KERNEL_SOURCES)):
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


COUNTER_WORKLOAD = "16x512x512x49"  # batch x rows x cols x filters the stored counters were taken on


def counters_from_profiles(kind: str, path: str = "", src=None, workload: str = COUNTER_WORKLOAD):
    """Counter figures per launch of a kernel kind measured with rocprofv3 (profiles/counters.json:
    calibrated HBM bytes, VALU instructions), if they were taken on this workload (batch x rows x
    cols x filters: the record's own, or one under "other_workloads") and the kernel sources have
    not changed since; else None."""
    path = path or os.path.join(ROOT, "profiles", "counters.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("kernel_sources_sha256") != source_digest(src):
            return None
        if rec.get("workload") == workload:
            return rec["kernels"].get(kind)
        return rec.get("other_workloads", {}).get(workload, {}).get("kernels", {}).get(kind)
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def traffic_from_profiles(kind: str, per_launch_units: float = 1.0, path: str = "", src=None,
                          workload: str = COUNTER_WORKLOAD):
    """Calibrated HBM bytes per launch (FETCH_SIZE + WRITE_SIZE) of a kernel kind, or None."""
    ent = counters_from_profiles(kind, path, src, workload)
    return None if ent is None else float(ent["bytes_per_launch"]) * per_launch_units


def valu_bound(kind: str, avg_ms: float, path: str = "", src=None, workload: str = COUNTER_WORKLOAD):
    """The compute side of the roofline: the kernel's VALU wave instructions per launch (rocprofv3
    SQ_INSTS_VALU) against the issue peak, i.e. the share of its duration the VALU would need at
    full issue; None without current counters."""
    ent = counters_from_profiles(kind, path, src, workload)
    if ent is None or ent.get("valu_wave_instructions") is None:
        return None
    n = float(ent["valu_wave_instructions"])
    min_ms = n / VALU_ISSUE_PEAK * 1e3
    return {"bound": "valu", "wave_instructions_per_launch": n, "peak_per_s": VALU_ISSUE_PEAK,
            "min_ms": min_ms, "frac": min_ms / avg_ms}


def device_copy_gbs(mib: int = 512, reps: int = 5) -> float:
    """Bytes read plus written per second by a device-to-device copy of `mib` MiB: the practical
    bandwidth ceiling beside the 8 TB/s specification."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * n * 4 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_host, min_seconds: float, max_images: int, workload: str = "fwdinv") -> dict:
    """The FP64 oracle (numpy, as it stands) on a bounded sample of the same workload:
    fwd+inv (or denoising) of the batch images in order (cycling), until min_seconds have elapsed."""
    import numpy as np

    from oracle import apps as OA
    from oracle import filters as OF
    from oracle import transform as OT

    log(f"cpu baseline: oracle system build {N}x{M} J={J}")
    ref = OF.build_system(N, M, J)
    thr = OA.thresholds(ref.idx, ref.rms, SIGMA, factors=[3.0] * J)
    t0 = time.perf_counter()
    n = 0
    while n < max_images:
        xi = x_host[n % B].astype(np.float64)
        if workload == "denoise":
            OA.denoise(xi, ref.spectra, ref.W, thr)
        elif workload == "layer":
            c = OT.forward_plain(xi, ref.spectra)
            OT.adjoint_plain(c, ref.spectra)
        else:
            c = OT.forward_plain(xi, ref.spectra)
            OT.inverse_plain(c, ref.spectra, ref.W)
        n += 1
        dt = time.perf_counter() - t0
        if n % 4 == 0:
            log(f"cpu baseline: {n} images, {dt:.1f} s")
        if dt >= min_seconds:
            break
    dt = time.perf_counter() - t0
    units = n * N * M * ref.K / 1e6
    res = {
        "value": units / dt,
        "unit": "Mpix·filters/s",
        "cores": 1,
        "cpu": cpu_model(),
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": f"numpy FP64 oracle, {dict(denoise='denoising', layer='forward+adjoint').get(workload, 'fwd+inv')} "
                  f"of {n} images of the {N}x{M}, {ref.K}-filter batch (cycling through the {B}), {dt:.1f} s; "
                  f"numpy.fft runs single-threaded",
    }
    if workload == "fwdinv":
        # second leg: the same shift-free forms with scipy.fft's threaded FFTs on every core this
        # process may use (the CPU share of the machine, capped by OMP_NUM_THREADS where it is set)
        workers = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            workers = max(1, min(workers, int(os.environ["OMP_NUM_THREADS"])))
        t0 = time.perf_counter()
        n2 = 0
        while n2 < max_images:
            xi = x_host[n2 % B].astype(np.float64)
            c = OT.forward_plain_threaded(xi, ref.spectra, workers)
            OT.inverse_plain_threaded(c, ref.spectra, ref.W, workers)
            n2 += 1
            if time.perf_counter() - t0 >= min_seconds / 2:
                break
        dt2 = time.perf_counter() - t0
        log(f"cpu baseline, {workers} threads: {n2} images, {dt2:.1f} s")
        res["all_cores"] = {"value": n2 * N * M * ref.K / 1e6 / dt2, "unit": "Mpix·filters/s", "cores": workers,
                            "kind": "oracle (scipy.fft threaded forms)",
                            "sample": f"scipy.fft FP64 shift-free forms with workers={workers}, fwd+inv of {n2} "
                                      f"images of the batch, {dt2:.1f} s"}
    return res


METRIC_INPAINT = "uneven inpainting (Algorithm 3) shearlet Mpix·filters·iterations/s, 8 images of 256²/512²/1024²"


def bench_inpaint(args) -> int:
    """Batched uneven inpainting: 8 cartoon images of sizes drawn (seeded) from {256, 512, 1024} squared,
    50% random-pixel masks, 33 filters up to 256x256 else 49, 100 iterations of Algorithm 3 with
    thresholds delta_i RMS_k decaying linearly to 0 from the largest RMS-normalised coefficient of the
    masked image. One step = the whole batch through all iterations (one captured graph per size group,
    groups on their own streams)."""
    import numpy as np
    import torch

    import synth
    from paper_2006_04591_amd import UnevenInpainter, delta_schedule

    iters = 100
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(3)
    sizes = [int(v) for v in rng.choice([256, 512, 1024], size=8)]
    inp = UnevenInpainter()
    fms, ms, scheds, cleans = [], [], [], []
    units = 0.0
    for i, n in enumerate(sizes):
        f = synth.cartoon(n, n, seed=3000 + i)
        m = synth.random_mask(n, n, 0.5, seed=3500 + i)
        fm = (f * m).astype(np.float32)
        s = inp.system(n, n)
        c = s.forward(torch.from_numpy(fm[None]).to(dev))
        d0 = float((c[0].abs().amax(dim=(1, 2)).cpu().numpy() / s.rms).max())
        fms.append(torch.from_numpy(fm).to(dev))
        ms.append(torch.from_numpy(m).to(dev))
        scheds.append(delta_schedule("linear", d0, iters))
        cleans.append((f, m, fm))
        units += n * n * s.K * iters / 1e6
    log(f"bench inpaint: sizes {sizes}")
    for _ in range(args.warmup):
        out = inp.run(fms, ms, scheds)
    torch.cuda.synchronize()
    steps = args.steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        out = inp.run(fms, ms, scheds)
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps

    def psnr(a, b):
        d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
        return float(20.0 * np.log10(255.0 * np.sqrt(d.size) / np.linalg.norm(d)))

    p_out = [psnr(cleans[i][0], out[i].cpu().numpy()) for i in range(8)]
    p_in = [psnr(cleans[i][0], cleans[i][2]) for i in range(8)]
    if not min(np.array(p_out) - np.array(p_in)) > 0:
        print("bench.py: inpainting did not improve the PSNR", file=sys.stderr)
        return 1
    # per-launch timing: one more pass with the launches issued directly (timing switches capture off)
    for s in inp._systems.values():
        s.profile(True)
    inp.run(fms, ms, scheds)
    torch.cuda.synchronize()
    kernels = {}
    for (n, _), s in inp._systems.items():
        rec = s.profile_read()
        s.profile(False)
        nb = sizes.count(n)
        plane = n * (n // 2) * 8
        xbytes = {"rows_r2c_images": 3 * nb * n * n * 4, "cols_fwd": nb * plane * (1 + s.K),
                  "rows_thresh": 2 * nb * s.K * plane, "cols_inv": nb * plane * (1 + s.K),
                  "rows_c2r_images": nb * n * n * 4}
        for kind, (cnt, tot) in rec.items():
            if cnt == 0:
                continue
            avg = tot / cnt
            per = xbytes.get(kind, 0) * iters / cnt
            kernels[f"{kind}@{n}"] = {"launches": cnt, "avg_ms": avg, "bytes_per_launch": per,
                                      "GBs": per / (avg / 1e3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dk = kernels[dom]
    # algorithmic bytes of the whole step: per iteration and image, f_masked, the mask and f read and
    # f written (4 B per pixel each); per iteration and size group, the two real filter sets read
    alg = 0.0
    for (n, _), s in inp._systems.items():
        nb = sizes.count(n)
        alg += iters * (nb * 16.0 * n * n + 2.0 * s.K * n * (n // 2 + 1) * 4)
    ach = alg / (ms_step / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None, "kernel": "whole step", "avg_launch_ms": ms_step, "bytes_per_launch": alg,
                "bytes_basis": "algorithmic (per iteration: f_masked, mask, f in, f out; two filter sets per size)",
                "dominant_kernel": {"kernel": dom, "avg_launch_ms": dk["avg_ms"],
                                    "exchange_bytes_per_launch": dk["bytes_per_launch"], "exchange_GBs": dk["GBs"],
                                    "exchange_frac": dk["GBs"] / HBM_PEAK_GBS}}
    res = {
        "metric": METRIC_INPAINT, "value": units / (ms_step / 1e3), "unit": "Mpix·filters·iterations/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched uneven inpainting, 8 cartoon images, 50% random-pixel masks, 100 iterations, "
                               "linear decay to 0, 33/49 filters", "sizes": sizes, "iterations": iters},
        "roofline": roofline, "kernels": kernels,
        "column_schedules": {f"{k[0]}x{k[1]}": list(v) for k, v in inp.schedules.items()},
        "psnr_masked_mean_db": float(np.mean(p_in)), "psnr_inpainted_mean_db": float(np.mean(p_out)),
    }
    inp.close()
    print(json.dumps(res))
    return 0


METRIC_SHRINK = "learned-shrinkage denoising (fwd + bf16-MFMA shrink network + inv) Mpix·filters/s @512²×49"


def bench_shrink(args) -> int:
    """Learned shrinkage: a 3-layer 3x3 network (49 -> 32 -> 32 -> 49, bf16 matrix-core kernels, FP32
    accumulate) is trained on generated (image, noise) pairs: a seeded pool of 32 clean 512x512 cartoons, each
    step draws 16 of them with noise levels sigma ~ U[10, 50] and fresh noise (seeded), 1250 steps = 20k pairs.
    It is then judged on 16 held-out noisy images against plain hard thresholding (3 sigma RMS_k), by PSNR.
    One timed step = forward transform + shrink network + inverse transform of the 16 held-out images."""
    import numpy as np
    import torch

    import synth
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    dev = torch.device("cuda:0")
    shs = ShearletSystem.build(N, M, J)
    K = shs.K
    shs.reserve(B)
    schedule = shs.autotune(B)
    pool = torch.from_numpy(np.stack([synth.cartoon(N, M, seed=5000 + i) for i in range(32)])).to(dev)
    rng = np.random.default_rng(5)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    # initial parameters: small random weights, output bias giving tau = 3 (hard thresholding at 3 sigma)
    r0 = np.random.default_rng(6)

    def he(co, ci):
        return (r0.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci))).astype(np.float32)

    params = {"W1": he(32, K), "b1": np.zeros(32, np.float32), "W2": he(32, 32), "b2": np.zeros(32, np.float32),
              "W3": 0.1 * he(K, 32), "b3": np.full(K, np.log(np.expm1(3.0)), np.float32)}
    net = ShrinkNet(shs, params)
    cn = torch.empty((B, K, N, M), dtype=torch.float32, device=dev)
    cc = torch.empty_like(cn)
    steps_train = int(args.train_steps)
    t0 = time.perf_counter()
    losses = []
    for it in range(steps_train):
        idx = torch.from_numpy(rng.integers(0, 32, size=B)).to(dev)
        sig = torch.from_numpy(rng.uniform(10.0, 50.0, size=B).astype(np.float32)).to(dev)
        clean = pool[idx]
        noisy = clean + sig[:, None, None] * torch.randn((B, N, M), generator=gen, device=dev)
        shs.forward(noisy, out=cn)
        shs.forward(clean, out=cc)
        lr = 2e-3 if it < steps_train // 2 else 5e-4
        loss = net.train_step(cn, cc, sig, lr=lr, temperature=0.5)
        if it % 250 == 0 or it == steps_train - 1:
            losses.append((it, float(loss)))
            log(f"bench shrink: step {it} loss {losses[-1][1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # held-out test set (its own seeds: independent of the number of training steps)
    sig_t = np.random.default_rng(7).uniform(10.0, 50.0, size=B).astype(np.float32)
    clean_t = np.stack([synth.cartoon(N, M, seed=5500 + i) for i in range(B)])
    noisy_t = np.stack([clean_t[i] + synth.gaussian_noise(N, M, float(sig_t[i]), seed=6000 + i) for i in range(B)])
    x = torch.from_numpy(noisy_t).to(dev)
    sg = torch.from_numpy(sig_t).to(dev)
    c = torch.empty((B, K, N, M), dtype=torch.float32, device=dev)
    cs = torch.empty_like(c)
    y = torch.empty((B, N, M), dtype=torch.float32, device=dev)

    def step():
        shs.forward(x, out=c)
        net.apply(c, sg, out=cs)
        shs.inverse(cs, out=y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    # the transform's launches timed one by one in a second pass (its timing events add to the step)
    shs.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    rec = shs.profile_read()
    shs.profile(False)
    # the network's kernels are timed apart, same stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        net.apply(c, sg, out=cs)
    e1.record()
    torch.cuda.synchronize()
    ms_net = e0.elapsed_time(e1) / args.steps
    yl = y.cpu().numpy()
    thr = torch.from_numpy(np.stack([shs.paper_thresholds(float(sig_t[i]), factors=[3.0] * J) for i in range(B)])).to(dev)
    yh = shs.denoise(x, thr).cpu().numpy()

    def psnr(a, b):
        d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
        return float(20.0 * np.log10(255.0 * np.sqrt(d.size) / np.linalg.norm(d)))

    p_learned = [psnr(clean_t[i], yl[i]) for i in range(B)]
    p_hard = [psnr(clean_t[i], yh[i]) for i in range(B)]
    p_noisy = [psnr(clean_t[i], noisy_t[i]) for i in range(B)]
    flops = 2.0 * B * N * M * 9 * (32 * K + 32 * 32 + K * 32)  # the three layers, real channels
    net_tflops = flops / (ms_net / 1e3) / 1e12
    # algorithmic bytes of the network: the coefficients in (FP32) and the shrunk coefficients out;
    # the hidden activations (bf16, 2 x 2 x 32 channels per pixel written and read) are intermediates
    alg = 2.0 * B * K * N * M * 4
    hidden = 4.0 * B * 32 * N * M * 2
    net_gbs = alg / (ms_net / 1e3) / 1e9
    units = B * N * M * K / 1e6
    res = {
        "metric": METRIC_SHRINK, "value": units / (ms_step / 1e3), "unit": "Mpix·filters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (network) / f32 (transform)", "data": "synthetic",
        "config": {"workload": "learned shrinkage, 16 held-out 512x512 cartoons, sigma ~ U[10,50], 49 filters; "
                               "network 49-32-32-49, 3x3, trained on 20k generated pairs",
                   "batch": B, "rows": N, "cols": M, "filters": K, "train_steps": steps_train,
                   "train_pairs": steps_train * B, "column_schedule": list(schedule)},
        # arithmetic intensity flops / (alg + hidden) ~ 90 flop/B, below the bf16 matrix ridge of 2500 / 8 = 312
        # flop/B: the network is bound by HBM, and its matrix-core rate is reported beside
        "roofline": {"bound": "hbm", "achieved": net_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": net_gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "shrink network (3 layers)",
                     "avg_launch_ms": ms_net, "bytes_per_launch": alg,
                     "bytes_basis": "algorithmic (coefficients in and out, FP32)",
                     "intermediate_bytes_per_launch": hidden,
                     "intensity_flop_per_byte": flops / (alg + hidden),
                     "mfma": {"achieved_tflops": net_tflops, "peak_tflops": 2500.0, "frac": net_tflops / 2500.0,
                              "flops_per_launch": flops}},
        "kernels": {k: {"launches": n, "avg_ms": t / n} for k, (n, t) in rec.items() if n},
        "train_seconds": train_s, "train_losses": losses,
        "psnr_noisy_mean_db": float(np.mean(p_noisy)), "psnr_hard_mean_db": float(np.mean(p_hard)),
        "psnr_learned_mean_db": float(np.mean(p_learned)),
        "learned_beats_hard": bool(np.mean(p_learned) > np.mean(p_hard)),
    }
    shs.close()
    print(json.dumps(res))
    return 0


def copy_calibration(mib: int) -> int:
    """Device-to-device copies of a known size, to calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.arange(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}))
    return 0


def traffic_summary(fetch_csv: str, write_csv: str, cal_fetch_csv: str, cal_write_csv: str, cal_bytes: int,
                    out_path: str = "", src=None, valu_csv: str = "", workload: str = COUNTER_WORKLOAD) -> int:
    """Writes profiles/counters.json: per-kernel HBM bytes per launch from rocprofv3 counter CSVs
    (FETCH_SIZE and WRITE_SIZE in KiB per dispatch), each scaled by the factor that makes the
    same counter read cal_bytes for the calibration copy kernel, and (valu_csv) the VALU, LDS and
    vector-memory instruction counts per launch (SQ_INSTS_*, summed over the counter's instances).
    The headline workload's figures form the record; another workload's ("BxNxMxK", its kernels
    identified by their row length M) go under "other_workloads" of an existing record taken on the
    same kernel sources, which they require."""
    import csv
    import statistics

    def per_kernel(path, counter):
        unit = 1024.0 if counter in ("FETCH_SIZE", "WRITE_SIZE") else 1.0  # KiB -> bytes
        sums = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Kernel_Name"], r["Dispatch_Id"])
            sums[key] = sums.get(key, 0.0) + float(r["Counter_Value"]) * unit
        by = {}
        for (name, _), v in sums.items():
            by.setdefault(name, []).append(v)
        return {k: statistics.mean(v) for k, v in by.items()}

    def copy_factor(path, counter):
        vals = [v for k, v in per_kernel(path, counter).items() if "shear" not in k and v > cal_bytes / 8]
        return cal_bytes / statistics.median(vals)

    ff = copy_factor(cal_fetch_csv, "FETCH_SIZE")
    fw = copy_factor(cal_write_csv, "WRITE_SIZE")
    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    insts = {c: per_kernel(valu_csv, c) for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
                                                 "SQ_INSTS_VMEM_WR")} if valu_csv else {}
    mcols = int(workload.split("x")[2])
    kinds = {f"k_rows_r2c<{mcols}, 0": "rows_r2c_images", "k_cols_fwd<": "cols_fwd", "k_cols_spec<": "cols_fwd",
             f"k_rows_c2r<{mcols}, 1": "rows_c2r_coeffs", f"k_rows_r2c<{mcols}, 1": "rows_r2c_coeffs",
             "k_cols_inv<": "cols_inv", f"k_rows_c2r<{mcols}, 0": "rows_c2r_images", "k_plane_fwd<": "plane_fwd"}
    out = {}
    for name in fetch:
        kind = next((v for k, v in kinds.items() if k in name), None)
        if kind is None:
            continue
        f = fetch[name] * ff
        w = write.get(name, 0.0) * fw
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        out[kind] = {"kernel": short, "fetch_bytes": f, "write_bytes": w, "bytes_per_launch": f + w}
        for c, vals in insts.items():
            key = {"SQ_INSTS_VALU": "valu_wave_instructions"}.get(c, c.lower().replace("sq_insts_", "") +
                                                                   "_wave_instructions")
            out[kind][key] = vals.get(name)
    path = out_path or os.path.join(ROOT, "profiles", "counters.json")
    digest = source_digest(src)
    if workload == COUNTER_WORKLOAD:
        rec = {"kernel_sources_sha256": digest, "workload": COUNTER_WORKLOAD, "fetch_scale": ff, "write_scale": fw,
               "calibration_bytes": cal_bytes, "kernels": out}
    else:
        try:
            with open(path) as fh:
                rec = json.load(fh)
        except (OSError, ValueError):
            rec = None
        if not rec or rec.get("kernel_sources_sha256") != digest:
            print(f"bench.py: no counter record of the current kernel sources in {path} to add {workload} to",
                  file=sys.stderr)
            return 1
        rec.setdefault("other_workloads", {})[workload] = {"fetch_scale": ff, "write_scale": fw, "kernels": out}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))
    return 0


def main() -> int:
    if len(sys.argv) > 1 and sys.argv[1] == "--copy-calibration":
        return copy_calibration(int(sys.argv[2]))
    if len(sys.argv) > 1 and sys.argv[1] == "--counter-summary":
        # fetch.csv write.csv cal_fetch.csv cal_write.csv cal_bytes [valu.csv [BxNxMxK]]
        a = sys.argv[2:]
        return traffic_summary(a[0], a[1], a[2], a[3], int(a[4]), valu_csv=a[5] if len(a) > 5 else "",
                               workload=a[6] if len(a) > 6 else COUNTER_WORKLOAD)
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle baseline sample length (0 = skip)")
    ap.add_argument("--chunk-images", type=int, default=0,
                    help="images per chunk of the K-expanded intermediate (0 = whole batch)")
    ap.add_argument("--train-steps", type=int, default=1250, help="shrink: training steps (16 pairs each)")
    ap.add_argument("--schedule", default="",
                    help="fwdinv/denoise/layer: fixed column-pass schedule 'pw_fwd,pw_inv,kg_fwd,kg_inv[,pc_fwd,pc_inv]' instead of "
                         "the autotuner (counter runs use it so that one kernel variant runs)")
    ap.add_argument("--workload", default="fwdinv", choices=("fwdinv", "denoise", "layer", "inpaint", "shrink"),
                    help="fwdinv: shear_forward + shear_inverse (the headline); denoise: shear_denoise with the "
                         "paper's thresholds (Section 4.2); layer: the autograd layer's forward and backward at "
                         "32 x 256x256, 33 filters; inpaint: Algorithm 3 on 8 images of uneven sizes; shrink: train and run "
                         "the learned shrinkage network")
    args = ap.parse_args()
    denoise = args.workload == "denoise"
    layer = args.workload == "layer"
    if args.workload in ("inpaint", "shrink"):
        import torch

        if not torch.cuda.is_available():
            print("bench.py: no GPU visible", file=sys.stderr)
            return 2
        return bench_inpaint(args) if args.workload == "inpaint" else bench_shrink(args)
    global B, N, M, J, SHEAR_LEVELS, CONFIG_ID
    if layer:
        B, N, M, J, SHEAR_LEVELS, CONFIG_ID = 32, 256, 256, 3, [1, 1, 2], 4
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (got --gpus {args.gpus}); run with --gpus 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_2006_04591_amd import ShearletSystem

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    log(f"bench: building system {N}x{M} J={J}")
    t0 = time.perf_counter()
    cap = 0
    if args.chunk_images > 0:
        pb = N * (M // 2) * 8
        cap = B * pb + args.chunk_images * 49 * pb
    shs = ShearletSystem.build(N, M, J, max_workspace_bytes=cap)
    build_s = time.perf_counter() - t0
    K = shs.K
    S, _ = shs.export_spectra()
    real_filters = bool(np.all(S.imag == 0))
    log(f"bench: K={K}, build {build_s:.2f} s, real filters={real_filters}")
    x_host = synth.cartoon_batch(B, N, M, config=CONFIG_ID, sigma=0.0 if layer else SIGMA)
    x = torch.from_numpy(x_host).to(dev)
    c = torch.empty((B, K, N, M), dtype=torch.float32, device=dev)
    y = torch.empty((B, N, M), dtype=torch.float32, device=dev)
    shs.reserve(B)
    if args.schedule:
        schedule = tuple(int(v) for v in args.schedule.split(","))
        if len(schedule) not in (4, 6):
            print("bench.py: --schedule needs pw_fwd,pw_inv,kg_fwd,kg_inv[,pc_fwd,pc_inv]", file=sys.stderr)
            return 2
        shs.set_schedule(*schedule)
        log(f"bench: fixed column-pass schedule (pw_fwd, pw_inv, kg_fwd, kg_inv[, pc_fwd, pc_inv]): {schedule}")
    else:
        schedule = shs.autotune(B)
        log(f"bench: autotuned column-pass schedule (pw_fwd, pw_inv, kg_fwd, kg_inv, pc_fwd, pc_inv): {schedule}")
    # denoising workload: hard threshold 3 sigma RMS_k on every plane (the listing of Section 4.2)
    thr = torch.from_numpy(np.tile(shs.paper_thresholds(SIGMA, factors=[3.0] * J), (B, 1))).to(dev)
    if layer:
        from paper_2006_04591_amd import ShearletLayer

        net = ShearletLayer(N, M, J, system=shs)
        xg = x[:, None].clone().requires_grad_(True)
        gen = torch.Generator(device=dev)
        gen.manual_seed(4)
        g = torch.randn((B, K, N, M), generator=gen, device=dev, dtype=torch.float32)

    def step():
        if denoise:
            shs.denoise(x, thr, out=y)
        elif layer:
            xg.grad = None
            net(xg).backward(g)
        else:
            shs.forward(x, out=c)
            shs.inverse(c, out=y)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: {args.warmup} warmup steps done")

    stream = torch.cuda.current_stream()
    # timed region: K steps bracketed by events on the stream the library launches on
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    log(f"bench: {args.steps} timed steps, {ms_step:.3f} ms/step")
    # profiled region: the same K steps again, every launch bracketed by the library's timing events
    # (same stream) and every step by a torch event; the events themselves add a few percent to the
    # step, so the step time above comes from the region without them
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    shs.profile(True)
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    ms_total = evs[0].elapsed_time(evs[-1])
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    rec = shs.profile_read()
    shs.profile(False)
    log(f"bench: {args.steps} profiled steps, {ms_total / args.steps:.3f} ms/step")

    quality = {}
    err = None
    if layer:
        # the timed gradient is the adjoint of the upstream gradient (same kernels, so bitwise)
        ref_grad = shs.adjoint(g)
        torch.cuda.synchronize()
        if not torch.equal(xg.grad[:, 0], ref_grad):
            print("bench.py: layer gradient differs from shear_adjoint of the upstream gradient", file=sys.stderr)
            return 1
    elif denoise:
        # the timed output against the clean images: PSNR = 20 log10(255 sqrt(pixels) / ||f - g||) (Section 4.2)
        def psnr(f, g):
            d = np.asarray(f, dtype=np.float64) - np.asarray(g, dtype=np.float64)
            return float(20.0 * np.log10(255.0 * np.sqrt(d.size) / np.linalg.norm(d)))

        clean = synth.cartoon_batch(B, N, M, config=CONFIG_ID, sigma=0.0)
        yh = y.cpu().numpy()
        p_out = [psnr(clean[b], yh[b]) for b in range(B)]
        p_in = [psnr(clean[b], x_host[b]) for b in range(B)]
        quality = {"psnr_denoised_mean_db": float(np.mean(p_out)), "psnr_noisy_mean_db": float(np.mean(p_in))}
        if not np.all(np.isfinite(yh)) or quality["psnr_denoised_mean_db"] <= quality["psnr_noisy_mean_db"]:
            print(f"bench.py: denoising did not improve the PSNR: {quality}", file=sys.stderr)
            return 1
        err = None
    else:
        # correctness guard on the timed output: reconstruction of the inputs
        err = float(torch.linalg.vector_norm(y - x) / torch.linalg.vector_norm(x))
        if not err <= 1e-5:
            print(f"bench.py: reconstruction error {err:.3e} exceeds 1e-5", file=sys.stderr)
            return 1

    units = B * N * M * K / 1e6
    value = units / (ms_step / 1e3)
    kernels = {}
    plane_fwd = rec.get("plane_fwd", (0, 0.0))[0] > 0
    for kind, (n, tot) in rec.items():
        if n == 0:
            continue
        avg = tot / n
        ab = kernel_algorithmic_bytes(kind, K, real_filters, plane_fwd) * args.steps / n  # per launch
        xb = exchange_bytes(kind, K, plane_fwd) * args.steps / n
        kernels[kind] = {"launches": n, "avg_ms": avg, "share": tot / ms_total, "algorithmic_bytes_per_launch": ab,
                         "algorithmic_GBs": ab / (avg / 1e3) / 1e9, "exchange_bytes_per_launch": xb,
                         "exchange_GBs": xb / (avg / 1e3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dk = kernels[dom]
    pb = path_algorithmic_bytes(K, real_filters)
    if denoise:
        pb = 2 * B * N * M * 4 + 2 * K * N * (M // 2 + 1) * (4 if real_filters else 8)  # x, y, two filter sets
    path = {"bound": "hbm", "achieved": pb / (ms_step / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": pb / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_step": pb}
    wl = f"{B}x{N}x{M}x{K}"  # stored counters apply only to the workload they were taken on
    if dk["algorithmic_bytes_per_launch"] > 0:
        ab = dk["algorithmic_bytes_per_launch"]
        achieved = ab / (dk["avg_ms"] / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(dom, workload=wl),
                    "kernel": dom, "avg_launch_ms": dk["avg_ms"], "bytes_per_launch": ab, "bytes_basis": "algorithmic",
                    "valu": valu_bound(dom, dk["avg_ms"], workload=wl)}
    else:
        # the fused threshold kernel moves none of the method's inputs or outputs (every byte it
        # reads and writes is an exchange plane), so the roofline is the whole step's: its
        # algorithmic bytes (x, y, the two filter sets) over the step time; the dominant kernel's
        # exchange traffic is reported beside it
        roofline = dict(path, traffic=None, kernel="whole step", avg_launch_ms=ms_step, bytes_per_launch=pb,
                        bytes_basis="algorithmic (x, y, two filter sets) per step",
                        dominant_kernel={"kernel": dom, "avg_launch_ms": dk["avg_ms"],
                                         "exchange_bytes_per_launch": dk["exchange_bytes_per_launch"],
                                         "exchange_GBs": dk["exchange_GBs"],
                                         "exchange_frac": dk["exchange_GBs"] / HBM_PEAK_GBS})

    out = {
        "metric": METRIC_DENOISE if denoise else (METRIC_LAYER if layer else METRIC),
        "value": value,
        "unit": "Mpix·filters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DENOISE if denoise else (WORKLOAD_LAYER if layer else WORKLOAD), "batch": B,
                   "rows": N, "cols": M, "filters": K, "shear_levels": SHEAR_LEVELS},
        "roofline": roofline,
        "path_roofline": path,
        "kernels": kernels,
        "system_build_s": build_s,
    }
    out["config"]["column_schedule"] = list(schedule)
    out["ms_per_step_profiled"] = ms_total / args.steps
    out["ms_per_step_profiled_p10_p50_p90"] = [float(v) for v in np.percentile(per_step, [10, 50, 90])]
    out["device_copy_GBs"] = device_copy_gbs()
    if denoise:
        out.update(quality)
        out["config"]["path"] = "separate (fused row threshold kernel)"
    elif not layer:
        out["reconstruction_rel_err"] = err
    if args.chunk_images > 0:
        out["config"]["chunk_images"] = args.chunk_images
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(x_host, args.cpu_seconds, 64, args.workload)
    shs.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
