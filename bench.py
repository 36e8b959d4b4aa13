#!/usr/bin/env python3
"""Projector-pair benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one forward projection plus one back projection (a "pair") of the
paper-scale workload: 128x128x80 volume at 4.8 mm, 128 views over 360
degrees, 37x37 depth/view-dependent Gaussian PSFs (sigma 1 -> 6 voxels), an
ellipsoidal body phantom with hot lesions and a tissue/lung/bone attenuation
map (synthetic, seeded).  The PSF convolution runs as FP32 FFTs (the
paper's method); the PSFs are checked on the host to be symmetric in x and
z, which the plan is told, so it keeps real spectra.  Inputs are resident in
HBM before the timed region.  Prints ONE JSON line with pairs/s, the per-pair
latency distribution, EM reconstruction latency, the roofline of the
dominant kernel (timed live with HIP events on the launch stream), the same
pair with the direct convolution and other plan variants beside it, and the
FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3          # MI355X published FP32 matrix (MFMA) peak, dense
LP_PEAK_TFLOPS = 2500.0           # MI355X published dense BF16 / FP16 matrix peak
HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak without packed FP32 instructions (which this build
# disables): 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz = 78.6 TFLOP/s
# (the published 157.3 TFLOP/s counts packed FP32, two FMAs per lane and cycle)
FP32_VALU_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="fft", choices=["fft", "direct"],
                    help="PSF convolution of the timed pair: FP32 FFTs (the paper's method, "
                         "SPECT_CONV_FFT) or the direct sum on the FP32 matrix cores")
    ap.add_argument("--direct-steps", type=int, default=10,
                    help="timed pairs of the other FP32 convolution method (0: skip)")
    ap.add_argument("--cache-mubar", type=int, default=1,
                    help="1: keep the Eq. (1) attenuation factor of all views in HBM (plan flag)")
    ap.add_argument("--em-recons", type=int, default=5, help="EM reconstructions timed for latency")
    ap.add_argument("--em-iters", type=int, default=8, help="EM iterations per reconstruction")
    ap.add_argument("--cpu-views", type=int, default=128,
                    help="views in the bounded oracle sample (0 disables the CPU baseline)")
    ap.add_argument("--grad-iters", type=int, default=10,
                    help="unrolled EM iterations differentiated end to end (0 disables)")
    ap.add_argument("--precision-steps", type=int, default=10,
                    help="pairs timed for each reduced-precision (BF16, FP16) convolution plan (0 disables)")
    ap.add_argument("--all-taps-steps", type=int, default=10,
                    help="timed pairs with mirror-image tap pairing switched off (0: skip)")
    ap.add_argument("--bilinear-steps", type=int, default=10,
                    help="timed pairs of the FP32 pair with 2-D bilinear rotation (0: skip)")
    ap.add_argument("--separable-steps", type=int, default=10,
                    help="timed pairs with the PSFs given as their 1-D factors (0: skip)")
    ap.add_argument("--large-steps", type=int, default=3,
                    help="pairs timed per precision on the 256x256x160 precision workload (0 disables)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests in the continuous-batching serving trace (0 disables)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=4, help="concurrent requests at most")
    ap.add_argument("--serve-precisions", default="fp32,bf16",
                    help="comma-separated convolution precisions of the served reconstructions "
                         "(one serving run per precision, on the same trace)")
    ap.add_argument("--uncached-steps", type=int, default=10,
                    help="timed pairs with the attenuation factor recomputed per call "
                         "(no SPECT_CACHE_MUBAR), the paper's memory-saving order (0: skip)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device-to-device: a plain "
                         "copy kernel of known size that calibrates HBM byte counters")
    return ap.parse_args()


def note(stage):
    """One progress line per bench stage, on stderr (the JSON line is stdout)."""
    print(f"bench: {stage}", file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def source_sha(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel calibration),
    or None if absent or taken on different kernel sources (every file the
    record names -- the kernel's source and the headers it includes -- must
    still hash to the recorded SHA-256)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
        if not rec:
            return None
        for src, sha in rec["sources"].items():
            if source_sha(os.path.join(ROOT, src)) != sha:
                return None
        return rec["hbm_bytes_per_launch"]
    except Exception:
        return None


def fft_flop_per_plane(Lx, Lz, mac, real=False):
    """Algorithmic work of one plane of the FFT convolution: the real
    two-dimensional transform of Lx x Lz points counted as 2.5 N log2 N
    (N = Lx Lz), plus the spectral product over the Lz (Lx/2 + 1) bins of the
    half spectrum: a complex product (6 FLOP, 8 with the accumulation of the
    depth sum) or, with the real spectra of symmetric PSFs, a real one (2,
    or 4 with the accumulation)."""
    import math
    n = Lx * Lz
    per_bin = (4.0 if mac else 2.0) if real else (8.0 if mac else 6.0)
    return 2.5 * n * math.log2(n) + per_bin * Lz * (Lx // 2 + 1)


def conv_roofline(kern_name, avg_ms, sel, nview, ny, op_flops, conv_flops, mirror):
    """Roofline of a convolution kernel: FP32 matrix cores for the direct sum,
    the FP32 vector ALUs (no packed FP32) for the FFT form."""
    if kern_name in ("conv_fwd_fft", "conv_back_fft"):
        Lx, Lz = (int(t) for t in sel["fft_size"].split("x"))
        flops = nview * ny * fft_flop_per_plane(Lx, Lz, kern_name == "conv_fwd_fft",
                                                sel.get("fft_real") == "1")
        a = flops / (avg_ms * 1e-3) / 1e12
        return {"kernel": kern_name, "bound": "alu", "achieved": a, "peak": FP32_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": a / FP32_VALU_TFLOPS, "traffic": traffic_for(kern_name),
                "algorithmic_per_launch": flops, "avg_launch_ms": avg_ms,
                "form": f"FFT {Lx}x{Lz} per plane (2.5 N log2 N + spectral product)"}
    a = conv_flops / (avg_ms * 1e-3) / 1e12
    return {"kernel": kern_name, "bound": "mfma", "achieved": a, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": a / FP32_PEAK_TFLOPS, "traffic": traffic_for(kern_name),
            "algorithmic_per_launch": conv_flops, "avg_launch_ms": avg_ms,
            "form": "mirror-paired taps" if mirror else "all taps",
            "operator_flop_per_launch": op_flops}


def time_pairs(torch, pl, xd, steps, warmup, vd_shape):
    """ms per pair and per-kernel ms per launch of `steps` forward + back pairs."""
    v2 = torch.empty(vd_shape, dtype=torch.float32, device=xd.device)
    b2 = torch.empty_like(xd)
    for _ in range(warmup):
        pl.forward(xd, out=v2)
        pl.back(v2, out=b2)
    torch.cuda.synchronize()
    pl.profile_start(max_launches=64 * steps + 64)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        pl.forward(xd, out=v2)
        pl.back(v2, out=b2)
    b.record()
    torch.cuda.synchronize()
    kt = pl.profile_stop()
    return a.elapsed_time(b) / steps, {k: v["total_ms"] / v["launches"] for k, v in kt.items()}


def cpu_baseline(x, mu, psf, dy, nviews_sample, seed):
    """The FP64 oracle as it stands (FFT convolution path), forward + back of
    `nviews_sample` views over a process pool of views on the host cores this
    process may use (its CPU affinity, at most 16: the host share of one GPU
    on the benchmark machines), scaled to whole pairs."""
    import numpy as np
    from oracle.pool import OraclePool, host_cores
    from oracle.projector import Geometry

    cores = host_cores(cap=16)
    nz, ny, nx = x.shape
    nview, _, pz, px = psf.shape
    step = max(1, nview // nviews_sample)
    views = list(range(0, nview, step))[:nviews_sample]
    g = Geometry(nx, ny, nz, len(views), px, pz, dy,
                 angles=[2 * np.pi * l / nview for l in views])
    y = np.random.default_rng(seed + 7).uniform(0.5, 1.5, size=(len(views), nz, nx))
    with OraclePool(mu, psf[views], g, workers=cores, conv="fft") as pool:
        pool.forward(np.zeros_like(x))          # workers started and warm
        t0 = time.perf_counter()
        pool.forward(x)
        pool.back(y)
        dt = time.perf_counter() - t0
        workers = pool.workers
    sec_per_pair = dt * nview / len(views)
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / sec_per_pair, "unit": "pairs/s", "cores": workers, "kind": "oracle",
            "sample": f"FP64 oracle (numpy + scipy.fft, FFT convolution) forward+back of "
                      f"{len(views)} of {nview} views at {nx}x{ny}x{nz}, {px}x{pz} PSF, "
                      f"{workers} worker processes over views, {dt:.1f} s"
                      + (", scaled to a full pair" if len(views) < nview else ""),
            "seconds_per_pair": sec_per_pair, "cpu_model": model,
            "os_cpu_count": os.cpu_count(), "affinity_cores": host_cores(cap=1 << 20)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this projector build runs on one GPU only (no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2301_09710_amd import spect, synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    spect.load()

    cfg = synth.CONFIGS["paper"]
    x, mu, psf, dy = synth.config_inputs("paper", seed=args.seed)
    nx, ny, nz, nview, px, pz = cfg["nx"], cfg["ny"], cfg["nz"], cfg["nview"], cfg["px"], cfg["pz"]
    xd = torch.from_numpy(x).to(dev)
    mud = torch.from_numpy(mu).to(dev)
    psfd = torch.from_numpy(psf).to(dev)
    # The Gaussian PSFs are symmetric in x and in z (checked here on the host,
    # exactly): the plan is told so (SPECT_PSF_SYMMETRIC_X | _Z), which pairs
    # mirror-image taps on the direct path and keeps real spectra on the FFT path.
    sym_x = bool(np.array_equal(psf, psf[..., ::-1]))
    sym_z = bool(np.array_equal(psf, psf[..., ::-1, :]))
    sym_kw = dict(mirror="assume" if sym_x else "auto", symmetric_z=sym_z)
    plan = spect.Plan(mud, psfd, dy, cache_mubar=bool(args.cache_mubar), method=args.method,
                      **sym_kw)
    sel = plan.describe()            # kernels chosen
    vd = torch.empty(plan.proj_shape, dtype=torch.float32, device=dev)
    bd = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def pair():
        plan.forward(xd, out=vd)
        plan.back(vd, out=bd)

    for _ in range(args.warmup):
        pair()
    torch.cuda.synchronize()

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    plan.profile_start(max_launches=64 * K + 64)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for s in range(K):
        ev[s][0].record()
        pair()
        ev[s][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    kern = plan.profile_stop()
    step_ms = [a.elapsed_time(b) for a, b in ev]
    total_ms = ev[0][0].elapsed_time(ev[-1][1])
    ms_per_step = total_ms / K
    value = 1000.0 / ms_per_step

    # dominant kernel and its roofline (algorithmic work per launch / average duration)
    N = nx * ny * nz
    views_per_launch = plan.nview  # one launch covers all views (view_batch = all)
    # the direct operator's products: 2 px pz FLOP per voxel per view; with
    # mirror-image tap pairing the matrix cores take 2 (px + 1) / 2 pz (the
    # pre-adds of the two input columns run on the vector ALUs)
    op_flops = 2.0 * px * pz * N * views_per_launch
    paired_flops = 2.0 * ((px + 1) // 2) * pz * N * views_per_launch
    mirror = sel.get("mirror") == "1"
    conv_flops = paired_flops if mirror else op_flops
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    avg_ms = {k: v["total_ms"] / v["launches"] for k, v in kern.items()}
    if dom in ("conv_fwd", "conv_back", "conv_fwd_fft", "conv_back_fft"):
        roof = conv_roofline(dom, avg_ms[dom], sel, nview, ny, op_flops, conv_flops, mirror)
    else:
        byts = 3.0 * 4 * N * views_per_launch
        achieved = byts / (avg_ms[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom),
                "algorithmic_per_launch": byts, "avg_launch_ms": avg_ms[dom]}

    # EM reconstruction latency (not part of `value`)
    em = None
    note("em_recons")
    if args.em_recons > 0:
        ones = torch.ones(plan.proj_shape, dtype=torch.float32, device=dev)
        sens = plan.back(ones)
        # the FFT convolution leaves rounding-level negatives where the exact
        # projection is zero; a Poisson rate must be nonnegative
        yd = torch.poisson(vd.clamp_min(0.0))
        rd = torch.full_like(yd, 0.05 * float(yd.mean()))
        lat = []
        for _ in range(args.em_recons):
            xe = torch.ones(plan.vol_shape, dtype=torch.float32, device=dev)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.em_iters):
                plan.em_step(xe, yd, sens, rd)
            b.record()
            torch.cuda.synchronize()
            lat.append(a.elapsed_time(b))
        em = {"iters": args.em_iters, "recons": args.em_recons, "p50_ms": pct(lat, 50),
              "p99_ms": pct(lat, 99)}
        # method variants on the same data: one regularised EM step (Eq. (7)-(8),
        # beta > 0, target u), and OSEM with 4 subsets x 16 iterations (the
        # comparison reconstruction's setting), each timed from its first launch
        ud = torch.ones(plan.vol_shape, dtype=torch.float32, device=dev)
        xe = torch.ones(plan.vol_shape, dtype=torch.float32, device=dev)
        plan.reg_em_step(xe, yd, sens, ud, 0.01, rd)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.em_iters):
            plan.reg_em_step(xe, yd, sens, ud, 0.01, rd)
        b.record()
        torch.cuda.synchronize()
        em["reg_em_step_ms"] = a.elapsed_time(b) / args.em_iters
        from paper_2301_09710_amd.osem import OSEM
        os_ = OSEM(mud, psfd, dy, 4, cache_mubar=bool(args.cache_mubar))
        os_.sensitivities()
        xo = torch.ones(plan.vol_shape, dtype=torch.float32, device=dev)
        os_.run(xo, yd, rd, iters=1)
        torch.cuda.synchronize()
        xo.fill_(1.0)
        a.record()
        os_.run(xo, yd, rd, iters=16)
        b.record()
        torch.cuda.synchronize()
        em["osem_4x16_ms"] = a.elapsed_time(b)
        os_.close()
        del os_

    # The other FP32 convolution method on the same pair (not part of `value`):
    # the direct sum on the matrix cores (mirror-paired taps for these
    # symmetric PSFs) when the headline runs the FFTs, and the other way round.
    other = None
    note("direct_steps")
    if args.direct_steps > 0:
        om = "direct" if args.method == "fft" else "fft"
        pl = spect.Plan(mud, psfd, dy, cache_mubar=bool(args.cache_mubar), method=om, **sym_kw)
        osel = pl.describe()
        ms, kav = time_pairs(torch, pl, xd, args.direct_steps, args.warmup, vd.shape)
        v2 = pl.forward(xd)
        b2 = pl.back(vd)
        torch.cuda.synchronize()
        odom = max((k for k in kav if k.startswith("conv_")), key=lambda k: kav[k])
        other = {"method": om, "pairs_per_s": 1000.0 / ms, "ms_per_pair": ms, "plan": osel,
                 "rel_l2_forward_vs_headline": float((v2.double() - vd.double()).norm() / vd.double().norm()),
                 "rel_l2_back_vs_headline": float((b2.double() - bd.double()).norm() / bd.double().norm()),
                 "kernels_ms_per_launch": kav,
                 "conv_roofline": conv_roofline(odom, kav[odom], osel, nview, ny, op_flops,
                                                paired_flops if osel.get("mirror") == "1" else op_flops,
                                                osel.get("mirror") == "1")}
        pl.close()
        del pl, v2, b2

    # The direct pair with every PSF tap taken separately (SPECT_PSF_ALL_TAPS):
    # the direct path for PSFs that are not symmetric in x (not part of `value`).
    all_taps = None
    note("all_taps_steps")
    if args.all_taps_steps > 0 and sym_x:
        pl = spect.Plan(mud, psfd, dy, cache_mubar=bool(args.cache_mubar), mirror="off")
        v2 = torch.empty_like(vd)
        b2 = torch.empty_like(bd)
        for _ in range(args.warmup):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        torch.cuda.synchronize()
        pl.profile_start(max_launches=64 * args.all_taps_steps + 64)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.all_taps_steps):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        b.record()
        torch.cuda.synchronize()
        kt = pl.profile_stop()
        ms = a.elapsed_time(b) / args.all_taps_steps
        pl.forward(xd, out=v2)
        pl.back(vd, out=b2)
        torch.cuda.synchronize()
        kav = {k: v["total_ms"] / v["launches"] for k, v in kt.items()}
        all_taps = {"pairs_per_s": 1000.0 / ms, "ms_per_pair": ms, "plan": pl.describe(),
                    "rel_l2_forward_vs_headline": float((v2.double() - vd.double()).norm() / vd.double().norm()),
                    "rel_l2_back_vs_headline": float((b2.double() - bd.double()).norm() / bd.double().norm()),
                    "kernels_ms_per_launch": kav,
                    "conv_fwd_tflops": op_flops / (kav["conv_fwd"] * 1e-3) / 1e12,
                    "conv_back_tflops": op_flops / (kav["conv_back"] * 1e-3) / 1e12}
        pl.close()
        del pl, v2, b2

    # The same pair without the attenuation cache (not part of `value`): the
    # Eq. (1) factor is recomputed from mu for every view in every call, as in
    # the paper's memory-saving design, and the workspace shrinks by the cache.
    uncached = None
    note("uncached_steps")
    if args.uncached_steps > 0:
        pl = spect.Plan(mud, psfd, dy, cache_mubar=False, method=args.method, **sym_kw)
        v2 = torch.empty_like(vd)
        b2 = torch.empty_like(bd)
        for _ in range(args.warmup):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        torch.cuda.synchronize()
        pl.profile_start(max_launches=64 * args.uncached_steps + 64)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.uncached_steps):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        b.record()
        torch.cuda.synchronize()
        kt = pl.profile_stop()
        ms = a.elapsed_time(b) / args.uncached_steps
        pl.forward(xd, out=v2)
        torch.cuda.synchronize()
        uncached = {"pairs_per_s": 1000.0 / ms, "ms_per_pair": ms, "workspace_bytes": pl.ws_bytes,
                    "forward_bitwise_equal_to_cached": bool(torch.equal(v2, vd)),
                    "kernels_ms_per_launch": {k: v["total_ms"] / v["launches"] for k, v in kt.items()}}
        pl.close()
        del pl, v2, b2

    # Reduced-precision convolution (not part of `value`): the same pair with
    # BF16 / FP16 matrix-core operands, and with split-BF16 operands (three
    # BF16 products per FP32 product), their speed and distance from the FP32
    # path (itself within 1e-5 of the FP64 oracle).
    lp = None
    note("precision_steps")
    if args.precision_steps > 0:
        lp = {}
        ref_v = vd.double()
        ref_b = bd.double()
        for prec in ("bf16", "fp16", "bf16x3"):
            pl = spect.Plan(mud, psfd, dy, cache_mubar=bool(args.cache_mubar), precision=prec)
            v2 = torch.empty_like(vd)
            b2 = torch.empty_like(bd)
            for _ in range(args.warmup):
                pl.forward(xd, out=v2)
                pl.back(vd, out=b2)
            torch.cuda.synchronize()
            pl.profile_start(max_launches=64 * args.precision_steps + 64)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.precision_steps):
                pl.forward(xd, out=v2)
                pl.back(v2, out=b2)
            b.record()
            torch.cuda.synchronize()
            kt = pl.profile_stop()
            ms = a.elapsed_time(b) / args.precision_steps
            pl.back(vd, out=b2)          # adjoint of the same input as the FP32 reference
            pl.forward(xd, out=v2)
            torch.cuda.synchronize()
            kav = {k: v["total_ms"] / v["launches"] for k, v in kt.items()}
            # the LP kernels take every tap (no mirror pairing); split BF16
            # issues three BF16 products per FP32 product
            lp_flops = op_flops * (3 if prec == "bf16x3" else 1)

            def lp_roof(ms_, flops_=lp_flops):
                if not ms_:
                    return None
                a_ = flops_ / (ms_ * 1e-3) / 1e12
                return {"bound": "mfma", "achieved": a_, "peak": LP_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": a_ / LP_PEAK_TFLOPS, "algorithmic_per_launch": flops_,
                        "avg_launch_ms": ms_}
            lp[prec] = {
                "pairs_per_s": 1000.0 / ms, "ms_per_pair": ms,
                "rel_l2_forward_vs_fp32": float((v2.double() - ref_v).norm() / ref_v.norm()),
                "rel_l2_back_vs_fp32": float((b2.double() - ref_b).norm() / ref_b.norm()),
                "kernels_ms_per_launch": kav,
                "conv_fwd_roofline": lp_roof(kav.get("conv_fwd_lp")),
                "conv_back_roofline": lp_roof(kav.get("conv_back_lp")),
            }
            pl.close()
            del pl, v2, b2

    # The same FP32 pair with 2-D bilinear rotation (SPECT_ROT_BILINEAR), the
    # alternative rotation the paper implements and times (not part of
    # `value`; a different operator, so its distance from the 3-pass pair is
    # the difference between the two interpolations, not an error).
    bil = None
    note("bilinear_steps")
    if args.bilinear_steps > 0:
        pl = spect.Plan(mud, psfd, dy, cache_mubar=bool(args.cache_mubar), rotation="bilinear",
                        method=args.method, **sym_kw)
        v2 = torch.empty_like(vd)
        b2 = torch.empty_like(bd)
        for _ in range(args.warmup):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        torch.cuda.synchronize()
        pl.profile_start(max_launches=64 * args.bilinear_steps + 64)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.bilinear_steps):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        b.record()
        torch.cuda.synchronize()
        kt = pl.profile_stop()
        ms = a.elapsed_time(b) / args.bilinear_steps
        pl.forward(xd, out=v2)
        torch.cuda.synchronize()
        bil = {"pairs_per_s": 1000.0 / ms, "ms_per_pair": ms,
               "rel_l2_forward_vs_3pass": float((v2.double() - vd.double()).norm() / vd.double().norm()),
               "kernels_ms_per_launch": {k: v["total_ms"] / v["launches"] for k, v in kt.items()}}
        pl.close()
        del pl, v2, b2

    # The same pair with the Gaussian PSFs given as their 1-D factors
    # (SPECT_PSF_SEPARABLE): the same operator up to the rounding of the
    # factors, two 1-D passes per plane (not part of `value`).
    sep = None
    note("separable_steps")
    if args.separable_steps > 0:
        cfg = synth.CONFIGS["paper"]
        fz, fx = synth.gaussian_psf_factors(px, pz, ny, nview, *cfg["sigma"])
        pl = spect.Plan(mud, (torch.from_numpy(fz).to(dev), torch.from_numpy(fx).to(dev)), dy,
                        cache_mubar=bool(args.cache_mubar))
        v2 = torch.empty_like(vd)
        b2 = torch.empty_like(bd)
        for _ in range(args.warmup):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        torch.cuda.synchronize()
        pl.profile_start(max_launches=64 * args.separable_steps + 64)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.separable_steps):
            pl.forward(xd, out=v2)
            pl.back(v2, out=b2)
        b.record()
        torch.cuda.synchronize()
        kt = pl.profile_stop()
        ms = a.elapsed_time(b) / args.separable_steps
        pl.forward(xd, out=v2)
        pl.back(vd, out=b2)
        torch.cuda.synchronize()
        kav = {k: v["total_ms"] / v["launches"] for k, v in kt.items()}
        sep_flops = 2.0 * (px + pz) * nx * ny * nz * nview
        sep = {"pairs_per_s": 1000.0 / ms, "ms_per_pair": ms,
               "rel_l2_forward_vs_2d": float((v2.double() - vd.double()).norm() / vd.double().norm()),
               "rel_l2_back_vs_2d": float((b2.double() - bd.double()).norm() / bd.double().norm()),
               "kernels_ms_per_launch": kav,
               "conv_fwd_roofline": {"bound": "alu", "achieved": sep_flops / (kav["conv_fwd"] * 1e-3) / 1e12,
                                     "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                                     "frac": sep_flops / (kav["conv_fwd"] * 1e-3) / 1e12 / FP32_VALU_TFLOPS}}
        pl.close()
        del pl, v2, b2

    # The precision workload: 256x256x160, 128 views, 37x37 PSFs, the pair and
    # a 10-iteration EM image in FP32, BF16 and FP16 (not part of `value`).
    # Distances are to the FP32 results, which the tests hold within 1e-5 of
    # the FP64 oracle at this size.
    large = None
    note("large_steps")
    if args.large_steps > 0:
        xl, mul, psfl, dyl = synth.config_inputs("large", seed=args.seed)
        xld, muld, psfld = (torch.from_numpy(a).to(dev) for a in (xl, mul, psfl))
        large = {"workload": "256x256x160 (2.4 mm), 128 views, 37x37 PSF", "precisions": {}}
        ref = None
        for prec in ("fp32", "bf16", "fp16", "bf16x3"):
            pl = spect.Plan(muld, psfld, dyl, cache_mubar=True, precision=prec)
            v2 = pl.forward(xld)
            b2 = pl.back(v2)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.large_steps):
                pl.forward(xld, out=v2)
                pl.back(v2, out=b2)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.large_steps
            yl = v2.clone() if ref is None else ref["v"]          # noiseless data from FP32
            sens = pl.back(torch.ones_like(yl))
            xe = torch.ones_like(xld)
            for _ in range(10):
                pl.em_step(xe, yl, sens)
            torch.cuda.synchronize()
            rec = {"ms_per_pair": ms, "pairs_per_s": 1000.0 / ms}
            if ref is None:
                ref = {"v": v2.clone(), "b": b2.clone(), "x": xe.clone()}
            else:
                rel = lambda p_, q_: float((p_.double() - q_.double()).norm() / q_.double().norm())
                rec.update({"rel_l2_forward_vs_fp32": rel(v2, ref["v"]),
                            "rel_l2_back_vs_fp32": rel(pl.back(ref["v"]), ref["b"]),
                            "rel_l2_em10_vs_fp32": rel(xe, ref["x"])})
            large["precisions"][prec] = rec
            pl.close()
            del pl, v2, b2, sens, xe
        del ref, xld, muld, psfld
        torch.cuda.empty_cache()

    # Differentiation through unrolled EM (not part of `value`): MSE against the
    # phantom backpropagated to x0 and y through `grad_iters` EM updates.
    grad = None
    note("grad_iters")
    if args.grad_iters > 0:
        from paper_2301_09710_amd import autograd as sag
        ones = torch.ones(plan.proj_shape, dtype=torch.float32, device=dev)
        sens = plan.back(ones)
        yc = plan.forward(xd)
        rg = torch.full_like(yc, 0.05 * float(yc.mean()))
        yg = torch.poisson((yc + rg).clamp_min(0.0))
        x0 = torch.full_like(xd, float(xd.mean()))
        # one untimed pass so that the timed one sees warm allocator pools
        xw = x0.clone().requires_grad_(True)
        ((sag.unrolled_mlem(plan, xw, yg, sens, rg, iters=1) - xd) ** 2).mean().backward()
        del xw
        torch.cuda.synchronize()
        base_mem = torch.cuda.memory_allocated(dev)
        torch.cuda.reset_peak_memory_stats(dev)
        a, m, b = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        x0g = x0.clone().requires_grad_(True)
        ygg = yg.clone().requires_grad_(True)
        a.record()
        xk = sag.unrolled_mlem(plan, x0g, ygg, sens, rg, iters=args.grad_iters)
        loss = ((xk - xd) ** 2).mean()
        m.record()
        loss.backward()
        b.record()
        torch.cuda.synchronize()
        grad = {"iters": args.grad_iters, "forward_ms": a.elapsed_time(m),
                "backward_ms": m.elapsed_time(b), "total_ms": a.elapsed_time(b),
                "projector_directions": 6 * args.grad_iters,
                "peak_extra_mb": (torch.cuda.max_memory_allocated(dev) - base_mem) / 2 ** 20}
        del x0g, ygg, xk, loss

    # Continuous-batching EM service (not part of `value`): Poisson arrivals of
    # reconstructions of three sizes, 8 EM iterations each.
    serving = None
    precs = [p_ for p_ in args.serve_precisions.split(",") if p_]
    note("serve_requests")
    if args.serve_requests > 0 and precs:
        from paper_2301_09710_amd import serve as sv
        trace0 = sv.poisson_trace(args.serve_requests, args.serve_rate, seed=args.seed + 1)
        # FP32 requests use the headline's convolution method; BF16 / FP16 the direct one
        t_gen = time.perf_counter()
        data = {r.rid: sv.RequestData(r, dev) for r in trace0}
        t_gen = time.perf_counter() - t_gen
        serving = {}
        for prec in precs:
            trace = sv.poisson_trace(args.serve_requests, args.serve_rate, seed=args.seed + 1,
                                     precision=prec,
                                     method=args.method if prec == "fp32" else "direct")
            budget = int(0.5 * torch.cuda.get_device_properties(dev).total_memory)
            sched = sv.Scheduler(budget, args.serve_slots,
                                 lambda r: sv.request_bytes(r.size, r.precision, method=r.method))
            ex = sv.GpuExecutor(dev, data, max_slots=args.serve_slots, keep_results=False)
            torch.cuda.synchronize()
            base = torch.cuda.memory_allocated(dev)
            torch.cuda.reset_peak_memory_stats(dev)
            t_s = time.perf_counter()
            done = sv.serve(trace, sched, ex)
            torch.cuda.synchronize()
            wall_s = time.perf_counter() - t_s
            rec = sv.summarize(done, wall_s)
            rec.update({"rate_req_s": args.serve_rate, "slots": args.serve_slots,
                        "precision": prec, "method": trace[0].method, "iters": trace[0].iters,
                        "budget_gb": budget / 1e9, "peak_admitted_gb": sched.peak / 1e9,
                        "peak_measured_gb": (torch.cuda.max_memory_allocated(dev) - base) / 1e9,
                        "wall_s": wall_s, "trace_s": trace[-1].arrival,
                        "data_generation_s (untimed)": t_gen})
            serving[prec] = rec
            del ex, sched
        del data

    if args.copy_mb > 0:
        nbytes = args.copy_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dstb = torch.empty_like(src)
        torch.cuda.synchronize()
        dstb.copy_(src)
        torch.cuda.synchronize()
        del src, dstb

    cpu = None
    note("cpu_views")
    if args.cpu_views > 0:
        cpu = cpu_baseline(x, mu, psf, dy, args.cpu_views, args.seed)

    out = {
        "metric": "fwd+back projector pairs/s at 128x128x80, 128 views; p50/p99 recon latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale FP32 projector pair: 128x128x80 volume (4.8 mm), "
                               "128 views over 360 deg, 37x37 depth/view-dependent Gaussian PSF",
                   "method": args.method,
                   "nx": nx, "ny": ny, "nz": nz, "nview": nview, "px": px, "pz": pz,
                   "cache_mubar": bool(args.cache_mubar), "plan": sel,
                   "psf_symmetry_stated": ("x" if sym_x else "") + ("z" if sym_z else ""),
                   "workspace_bytes": plan.ws_bytes,
                   "mubar_cache_bytes": (nview * nx * ny * nz * 4) if args.cache_mubar else 0},
        "uncached_mubar": uncached,
        "other_method": other,
        "pair_latency_ms": {"p50": pct(step_ms, 50), "p99": pct(step_ms, 99),
                            "p10": pct(step_ms, 10), "p90": pct(step_ms, 90)},
        "wall_s_timed": wall,
        "em_recon_latency": em,
        "unrolled_em_grad": grad,
        "reduced_precision": lp,
        "all_taps": all_taps,
        "bilinear_rotation": bil,
        "separable_psf": sep,
        "large_precision": large,
        "serving": serving,
        "kernels_ms_per_launch": avg_ms,
        "roofline": roof,
        # the direct sum's products per pair (forward and back convolution,
        # 2 px pz FLOP per voxel per view each) over the measured pair time: the
        # rate a direct all-taps implementation would need to match this pair
        # (above the FP32 matrix-core peak when the FFTs run the convolution)
        "direct_sum_equivalent": {"flop_per_pair": 2 * op_flops,
                                  "tflops": 2 * op_flops / (ms_per_step * 1e-3) / 1e12,
                                  "fp32_mfma_peak_tflops": FP32_PEAK_TFLOPS},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
