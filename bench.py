"""Throughput of the 2D HA-NsDLCT on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one forward NsDLCT (all five fused passes) of a 1024 x 1024
complex64 image (i.i.d. N(0,1) real and imaginary parts), ABCD drawn by the
seeded symplectic generator (seed 1, first draw with |det B| >= 1e-3 and a
CM-CC-CM-CC decomposition), spacing sqrt(2 pi / 1024).  Inputs live in HBM
before timing starts: a ring of distinct input/output image pairs larger than
the 256 MB last-level cache, one pair per step in turn.

Prints one JSON line: transforms/s (whole job), the roofline of the dominant
pass kernel (algorithmic bytes / average launch time from HIP events on the
launch stream) and the FP64 oracle timed on the host as the CPU baseline.
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

METRIC = "NsLCT/s @1024² c64 + %HBM peak; split-prec vs FP32 plain at relL2≤1e-4"
HBM_PEAK_GBPS = 8000.0
# HBM bytes per launch of the two 1024-long pass kernels: rocprofv3
# FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel calibration, read from the
# kept profile, which records a hash of the kernel sources it was taken with;
# when the sources have changed since, the traffic is unknown (None).
PROFILE = os.path.join(ROOT, "profiles", "nslct_pass_1024_c64_forward.md")
KERNEL_SOURCES = ("fft_engine.hpp", "pass_kernels.hpp", "nslct.hip")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1707_03688_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile() -> dict:
    """{"rows": bytes, "cols": bytes} from the profile's traffic line, or
    {} when the profile is missing or was taken with other kernel sources."""
    import re
    try:
        with open(PROFILE) as f:
            text = f.read()
    except OSError:
        return {}
    m = re.search(r"traffic-per-launch: rows=(\d+) cols=(\d+) sources=([0-9a-f]+)", text)
    if not m or m.group(3) != kernel_source_hash():
        return {}
    return {"rows": int(m.group(1)), "cols": int(m.group(2))}


KERNEL_NAMES = {"rows": "nslct_pass<float, 1024, false, 4, false, 0, true> (passes 0, 2, 4: row lines)",
                "cols": "nslct_pass<float, 1024, true, 4, false, 0, true> (passes 1, 3: column lines)"}


def draw_matrix(seed: int, N: int, d: float, nl):
    import numpy as np
    import synth
    for i, M in enumerate(synth.symplectic_candidates(seed)):
        if abs(np.linalg.det(M[:2, 2:])) < 1e-3:
            continue
        try:
            return i, M, nl.Plan(M, N, N, d, d)
        except nl.NslctError:
            continue
    raise RuntimeError("no acceptable draw")


def host_info() -> dict:
    """CPU model, logical CPU count and the affinity set of this process."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    try:
        aff = sorted(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        aff = list(range(os.cpu_count() or 1))
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity": len(aff),
            "affinity_set": _ranges(aff)}


def _ranges(xs) -> str:
    out, start, prev = [], None, None
    for x in xs:
        if start is None:
            start = prev = x
        elif x == prev + 1:
            prev = x
        else:
            out.append(f"{start}-{prev}" if prev > start else f"{start}")
            start = prev = x
    if start is not None:
        out.append(f"{start}-{prev}" if prev > start else f"{start}")
    return ",".join(out)


def cpu_baseline(M_plan_stages, g, budget_s: float = 20.0, threads=None):
    """The FP64 oracle (dense-DFT chain) on the host, same image and stages,
    with the BLAS pool limited to `threads` (None: as configured)."""
    from oracle import chain, plan as oplan
    typ, mats, N, d = M_plan_stages
    po = oplan.plan_from_stages(typ, mats, N, N, d, d)
    from threadpoolctl import threadpool_info, threadpool_limits
    with threadpool_limits(limits=threads):
        used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        runs, t_total, out = 0, 0.0, None
        while runs < 1 or (t_total < budget_s and runs < 5):
            t0 = time.perf_counter()
            out = chain.forward(po, g)
            t_total += time.perf_counter() - t0
            runs += 1
    return runs / t_total, used, runs, out


def cpu_fft_chain(st, g, N, d, budget_s: float = 10.0):
    """Same-algorithm CPU baseline: the unitary five-slot chain of the plan's
    stage matrices with pocketfft (scipy.fft, complex128, all host threads)."""
    import numpy as np
    import scipy.fft as sf
    typ, P = st["type"], st["mats"]
    Z = np.zeros((2, 2))
    slots = {1: [Z, -P[3], P[2], -P[1], P[0]], 2: [P[3], -P[2], P[1], -P[0], Z]}[typ]
    m = np.arange(N) - N // 2
    dw = 2 * np.pi / (N * d)

    def cm(x, S, du):
        ph = 0.5 * S[0, 0] * du * du * (m[:, None] ** 2) + S[0, 1] * du * du * np.outer(m, m) \
            + 0.5 * S[1, 1] * du * du * (m[None, :] ** 2)
        return x * np.exp(1j * ph)

    def U(x, inv):
        f = sf.ifft2 if inv else sf.fft2
        return sf.fftshift(f(sf.ifftshift(x), norm="ortho", workers=-1))

    def run():
        x = cm(g.astype(np.complex128), slots[0], d)
        x = U(cm(U(x, False), slots[1], dw), True)
        x = cm(x, slots[2], d)
        x = U(cm(U(x, False), slots[3], dw), True)
        return cm(x, slots[4], d)

    runs, t_total, out = 0, 0.0, None
    while runs < 1 or (t_total < budget_s and runs < 20):
        t0 = time.perf_counter()
        out = run()
        t_total += time.perf_counter() - t0
        runs += 1
    return runs / t_total, runs, out


def bench_batched(nl, torch, synth, np, count=256, seed=2):
    """Ragged batch: `count` images, sides uniform over 128..1024 (two of them
    3 * 2^k), each with its own seeded symplectic ABCD; one graph replay per
    batch against the per-image loop of launches."""
    sizes = synth.batch_sizes(count, seed)
    cands = synth.symplectic_candidates(seed)
    plans = []
    for s in sizes:
        d = (2 * np.pi / s) ** 0.5
        while True:
            M = next(cands)
            if abs(np.linalg.det(M[:2, 2:])) < 1e-3:
                continue
            try:
                plans.append(nl.Plan(M, s, s, d, d))
                break
            except nl.NslctError:
                continue
    b = nl.Batch(plans)
    x = torch.randn(b.total, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    def timed(mode, reps):
        for _ in range(2):
            b.run(x, y, 0, mode)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.run(x, y, 0, mode)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_graph = timed(0, 20)
    t_loop = timed(2, 5)
    px = b.total
    return {"images": count, "samples": px, "batch_per_s": 1 / t_graph, "images_per_s": count / t_graph,
            "ms_per_batch": t_graph * 1e3, "loop_ms_per_batch": t_loop * 1e3,
            "speedup_vs_loop": t_loop / t_graph,
            "hbm_effective_GBps": 80.0 * px / t_graph / 1e9,
            "pct_hbm_peak": 80.0 * px / t_graph / 1e9 / HBM_PEAK_GBPS * 100,
            "schedule": {f"{'cols' if c else 'rows'} {N}": f"{v['lines']} lines x "
                         + (f"{v['mult']}/CU" if v["mult"] else "1 WG/item")
                         + (", alternative line plan" if v["plan"] else "")
                         for (c, N), v in b.schedules().items()}}


def bench_split(nl, torch, synth, np, count=8, N=4096, reps=3):
    """`count` images of N x N, each with its own seeded ABCD (seed 3): the
    FP32 path against the split FP16 / BF16 matrix-core paths, time per
    batch and the worst per-image relative L2 error against the complex128
    path on the same input."""
    d = math.sqrt(2 * math.pi / N)
    cands = synth.symplectic_candidates(3)
    precs = ["c64", "c64_split_f16", "c64_split_bf16"]
    out = {p: {"s": 0.0, "worst_rel_l2": 0.0} for p in precs}
    y = torch.empty((N, N), dtype=torch.complex64, device="cuda")
    for b in range(count):
        M = next(cands)
        p64 = nl.Plan(M, N, N, d, d, precision="c128")
        st = p64.stages()
        x = torch.from_numpy(synth.complex_normal((N, N), seed=100 + b)).cuda()
        ref = p64.forward(x)
        xc = x.to(torch.complex64)
        del x
        for prec in precs:
            p = nl.Plan.from_stages(st["type"], st["mats"], N, N, d, d, prec)
            p.forward(xc, out=y)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(torch.cuda.current_stream())
            for _ in range(reps):
                p.forward(xc, out=y)
            e1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            out[prec]["s"] += e0.elapsed_time(e1) * 1e-3 / reps
            err = (torch.linalg.vector_norm(y.to(torch.complex128) - ref)
                   / torch.linalg.vector_norm(ref)).item()
            out[prec]["worst_rel_l2"] = max(out[prec]["worst_rel_l2"], err)
        del ref, xc
    res = {"images": count, "N": N}
    for prec in precs:
        res[prec] = {"ms_per_batch": out[prec]["s"] * 1e3, "NsLCT_per_s": count / out[prec]["s"],
                     "worst_rel_l2_vs_c128": out[prec]["worst_rel_l2"]}
    for prec in precs[1:]:
        res[prec]["speedup_vs_c64"] = out["c64"]["s"] / out[prec]["s"]
    return res


def bench_reduced(nl, torch, M, N, d, ins, outs, K):
    """Three-pass schedules at the headline size: LC-NsDLCT (rank-one gauge,
    orientation by the eq. HA24 objective) of the headline matrix, and
    CM-CC-CM of a gyrator (symmetric B).  48 B per sample per transform."""
    import numpy as np
    R = len(ins)
    phi = 0.7
    S = np.array([[0.0, 1.0], [1.0, 0.0]])
    gyr = np.block([[np.cos(phi) * np.eye(2), np.sin(phi) * S], [-np.sin(phi) * S, np.cos(phi) * np.eye(2)]])
    out = {}
    for name, MM, typ in (("lc_headline_matrix", M, 6), ("cmccm_gyrator_0.7", gyr, 3)):
        p = nl.Plan(MM, N, N, d, d, type_override=typ)
        for i in range(5):
            p.forward(ins[i % R], out=outs[i % R])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(K):
            p.forward(ins[i % R], out=outs[i % R])
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / K
        out[name] = {"stage_type": p.stages()["type"], "passes": p.passes(), "us_per_transform": sec * 1e6,
                     "NsLCT_per_s": 1 / sec, "hbm_effective_GBps": 48.0 * N * N / sec / 1e9,
                     "pct_hbm_peak": 48.0 * N * N / sec / 1e9 / HBM_PEAK_GBPS * 100}
    return out


def bench_general_sizes(nl, torch, synth, draw_matrix, K=200):
    """One image per call at side lengths without a native line FFT (the
    paper's 100 x 100 and 165 x 165 grids, and a prime 257): Bluestein line
    DFTs, complex64."""
    out = {}
    for N in (100, 165, 257):
        d = math.sqrt(2 * math.pi / N)
        _, M, p = draw_matrix(1, N, d, nl)
        x = torch.randn(N, N, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            p.forward(x, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            p.forward(x, out=y)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / K
        out[f"{N}x{N}"] = {"us_per_transform": sec * 1e6, "NsLCT_per_s": 1 / sec}
    return out


def bench_backward(nl, torch, synth, np, count=32, N=512, reps=10):
    """One training step of loss = ||NsDLCT_M(theta)(x) - y||^2 on `count`
    images of N x N (y: the transform under a perturbed matrix): forward,
    loss, backward through the adjoint kernel.  Reports the device time of
    forward + adjoint kernels (HIP events) and the whole step including the
    host-side planning (gauge re-solve for M(theta) and its Jacobian)."""
    from paper_1707_03688_amd import autograd as ag
    d = math.sqrt(2 * math.pi / N)
    M0 = next(synth.symplectic_candidates(4))
    rng = np.random.default_rng(4)
    theta_star = rng.normal(0.0, 0.05, size=10)
    x = torch.from_numpy(synth.complex_normal((count, N, N), seed=4)).to(torch.complex64).cuda()
    pstar = nl.Plan.lie(M0, theta_star, N, N, d, d, symplectic_tol=1e-8)
    y = pstar.forward(x)
    p0 = nl.Plan.lie(M0, np.zeros(10), N, N, d, d, symplectic_tol=1e-8)
    G = p0.forward(x)
    gout = 2 * (G - y)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        p0.forward(x, out=G)
        ag.backward_sums(p0, G, gout)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        p0.forward(x, out=G)
        ag.backward_sums(p0, G, gout)
    e1.record(stream)
    torch.cuda.synchronize()
    dev_s = e0.elapsed_time(e1) * 1e-3 / reps

    def step():
        xg = x.clone().requires_grad_(True)
        theta = torch.zeros(10, dtype=torch.float64, requires_grad=True)
        loss = (ag.nsdlct(xg, theta, M0, d, d) - y).abs().pow(2).sum()
        loss.backward()
        return loss

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    full_s = (time.perf_counter() - t0) / 2
    return {"images": count, "N": N, "device_fwd_bwd_ms": dev_s * 1e3, "device_steps_per_s": 1 / dev_s,
            "device_pct_hbm_peak": 240.0 * count * N * N / dev_s / 1e9 / HBM_PEAK_GBPS * 100,
            "full_step_ms": full_s * 1e3,
            "note": "device = forward (5 passes) + paired adjoint sweep (5 passes, two signals); "
                    "bytes 80 + 160 B/px; full step adds torch loss ops and host planning"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ring", type=int, default=48, help="distinct in/out image pairs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--batched", type=int, default=1, help="also time the ragged batched workload")
    ap.add_argument("--split", type=int, default=1, help="also time the split-precision 8 x 4096^2 leg")
    ap.add_argument("--conc", type=int, default=1, help="also time 8 transforms per launch")
    ap.add_argument("--backward", type=int, default=1, help="also time the 32 x 512^2 fwd+bwd step")
    ap.add_argument("--reduced", type=int, default=1, help="also time the three-pass LC / CM-CC-CM schedules")
    ap.add_argument("--general", type=int, default=1, help="also time 100^2 / 165^2 / 257^2 (Bluestein lines)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched and "
              "single-image transforms shard by image, see the design notes.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1707_03688_amd as nl
    import synth

    torch.cuda.set_device(0)
    N = 1024
    d = math.sqrt(2 * math.pi / N)
    draw, M, plan = draw_matrix(1, N, d, nl)
    st = plan.stages()
    g = synth.complex_normal((N, N), seed=1)
    x0 = torch.from_numpy(g).to(torch.complex64).cuda()
    R = max(1, args.ring)
    ins = [x0.clone() for _ in range(R)]
    outs = [torch.empty_like(x0) for _ in range(R)]
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        plan.forward(ins[i % R], out=outs[i % R])
    torch.cuda.synchronize()

    # Timed region: K whole transforms back to back (host clock for the
    # value, HIP events on the launch stream for the kernel attribution).
    K = args.steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(K):
        plan.forward(ins[i % R], out=outs[i % R])
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    value = K / sec
    chain_ms = ev0.elapsed_time(ev1) / K

    # Per-kernel durations: each pass launched K times back to back (HIP
    # events on the launch stream around the K launches).  Pass 0 reads the
    # input ring from HBM as in the chain; passes 1-4 cycle over 8 image
    # buffers (64 MiB: beyond the XCDs' L2, inside the 256 MB MALL), the
    # residency their inputs have in the chain, where they were just written
    # by the previous pass.  Passes 0, 2, 4 run the row kernel and passes 1, 3
    # the column kernel; a kernel's average launch duration is the mean over
    # its passes.
    pass_ms = []
    for p in range(5):
        Rp = R if p == 0 else min(R, 8)
        for i in range(3):
            plan.launch_pass(0, p, ins[i % Rp] if p == 0 else outs[i % Rp], outs[i % Rp])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(K):
            plan.launch_pass(0, p, ins[i % Rp] if p == 0 else outs[i % Rp], outs[i % Rp])
        e1.record(stream)
        torch.cuda.synchronize()
        pass_ms.append(e0.elapsed_time(e1) / K)
    # The passes run slower inside the chain than back to back (each starts
    # on data another XCD just wrote, with the other kernel's code in the
    # instruction caches): the per-pass times are scaled so that they add up
    # to the chain time measured over the timed region.
    loop_ms = list(pass_ms)
    pass_ms = [v * chain_ms / sum(loop_ms) for v in loop_ms]
    kernels = {"rows": [0, 2, 4], "cols": [1, 3]}
    kern_ms = {k: float(np.mean([pass_ms[p] for p in ps])) for k, ps in kernels.items()}
    dom = max(kernels, key=lambda k: kern_ms[k] * len(kernels[k]))
    px = N * N
    bytes_per_launch = 16.0 * px  # one read + one write of complex64
    achieved = bytes_per_launch / (kern_ms[dom] * 1e-3) / 1e9

    # Copy-kernel reference bandwidth on the same buffers.
    src = torch.empty(256 * 1024 * 1024 // 8, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        nl.device_copy(src, dst)
    torch.cuda.synchronize()
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record(stream)
    for _ in range(10):
        nl.device_copy(src, dst)
    ce1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 2 * src.numel() * 8 * 10 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del src, dst

    # Independent single-image transforms processed 8 per launch (same kernels,
    # grid.y = 8): the throughput regime, reported beside the sequential value.
    conc = None
    if args.conc:
        x8 = torch.stack(ins[:8]).contiguous()
        y8 = torch.empty_like(x8)
        for _ in range(3):
            plan.forward(x8, out=y8)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(10, K // 8)
        c0.record(stream)
        for _ in range(reps):
            plan.forward(x8, out=y8)
        c1.record(stream)
        torch.cuda.synchronize()
        conc = 8 * reps / (c0.elapsed_time(c1) * 1e-3)
        del x8, y8

    reduced = bench_reduced(nl, torch, M, N, d, ins, outs, K) if args.reduced else None
    general = bench_general_sizes(nl, torch, synth, draw_matrix) if args.general else None
    batched = bench_batched(nl, torch, synth, np) if args.batched else None
    split = bench_split(nl, torch, synth, np) if args.split else None
    bwd = bench_backward(nl, torch, synth, np) if args.backward else None

    plan.forward(ins[0], out=outs[0])
    G = outs[0].cpu().numpy()
    back = plan.inverse(outs[0])
    recon = (torch.linalg.vector_norm(back - ins[0]) / torch.linalg.vector_norm(ins[0])).item()

    # The small case: one 64 x 64 complex128 image per call (latency-bound).
    N0 = 64
    _, M0, _ = draw_matrix(0, N0, 1.0, nl)
    p0 = nl.Plan(M0, N0, N0, 1.0, 1.0, precision="c128")
    x0s = torch.from_numpy(synth.complex_normal((N0, N0), seed=0)).cuda()
    y0s = torch.empty_like(x0s)
    for _ in range(10):
        p0.forward(x0s, out=y0s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        p0.forward(x0s, out=y0s)
    torch.cuda.synchronize()
    c0_us = (time.perf_counter() - t0) / K * 1e6
    # Many small images per call: 256 of 64 x 64 (complex64 and complex128),
    # the whole chain per image in one launch from LDS.
    many = {}
    for prec in ("c64", "c128"):
        pm = nl.Plan(M0, N0, N0, 1.0, 1.0, precision=prec)
        xm = torch.from_numpy(synth.complex_normal((256, N0, N0), seed=1)).to(
            torch.complex64 if prec == "c64" else torch.complex128).cuda()
        ym = torch.empty_like(xm)
        for _ in range(5):
            pm.forward(xm, out=ym)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            pm.forward(xm, out=ym)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / 50 * 1e6
        many[prec] = {"us_per_call": us, "us_per_image": us / 256, "NsLCT_per_s": 256e6 / us}
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "NsLCT/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": sec / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "NsDLCT forward, 1024x1024 complex64, i.i.d. N(0,1) image, "
                               "seeded symplectic ABCD (seed 1), spacing sqrt(2pi/1024)",
                   "Nx": N, "Ny": N, "precision": "c64", "type": st["type"], "draw": draw,
                   "ring_pairs": R, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_from_profile().get(dom),
                     "kernel": KERNEL_NAMES[dom], "avg_launch_us": kern_ms[dom] * 1e3,
                     "launches_per_transform": len(kernels[dom]),
                     "other_kernel": {k: {"kernel": KERNEL_NAMES[k], "avg_launch_us": kern_ms[k] * 1e3,
                                          "achieved": bytes_per_launch / (kern_ms[k] * 1e-3) / 1e9,
                                          "frac": bytes_per_launch / (kern_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                          "traffic": traffic_from_profile().get(k)}
                                      for k in kernels if k != dom}},
        "pass_us": [round(v * 1e3, 3) for v in pass_ms],
        "pass_us_back_to_back": [round(v * 1e3, 3) for v in loop_ms],
        "chain_us_events": chain_ms * 1e3,
        "hbm_effective_GBps": 80.0 * px * value / 1e9,
        "pct_hbm_peak": 80.0 * px * value / 1e9 / HBM_PEAK_GBPS * 100,
        "copy_kernel_GBps": copy_gbps,
        "forward_inverse_rel_l2": recon,
        "small_64_c128": {"us_per_transform": c0_us, "NsLCT_per_s": 1e6 / c0_us,
                          "note": "64 x 64 complex128, unit spacing, one image per call"},
        "small_64_many": {**many, "note": "256 images of 64 x 64 per call (one launch, images held in LDS)"},
    }
    if conc:
        result["concurrent8"] = {"value": conc, "unit": "NsLCT/s",
                                 "pct_hbm_peak": 80.0 * px * conc / 1e9 / HBM_PEAK_GBPS * 100,
                                 "note": "8 independent 1024x1024 transforms per launch (grid.y = 8)"}
    if reduced:
        result["reduced_schedules_1024"] = reduced
    if general:
        result["general_sizes_c64"] = general
    if batched:
        result["batched_ragged"] = batched
    if split:
        result["split_precision_4096"] = split
    if bwd:
        result["fwd_bwd_512"] = bwd
    if not args.no_cpu:
        rate, threads, runs, ref = cpu_baseline((st["type"], st["mats"], N, d), g)
        rate1, _, runs1, _ = cpu_baseline((st["type"], st["mats"], N, d), g, budget_s=5.0, threads=1)
        from oracle import chain
        result["cpu_baseline"] = {"value": rate, "unit": "NsLCT/s", "cores": threads, "kind": "oracle",
                                  "sample": f"{runs} forward transform(s) of the same 1024x1024 image "
                                            "by the FP64 dense-DFT oracle chain",
                                  "one_core": {"value": rate1, "runs": runs1}, **host_info()}
        result["rel_l2_vs_fp64_oracle"] = chain.rel_l2(G, ref)
        frate, fruns, fout = cpu_fft_chain(st, g, N, d)
        result["cpu_fft_chain"] = {"value": frate, "unit": "NsLCT/s", "threads": os.cpu_count(),
                                   "sample": f"{fruns} forward transform(s), scipy.fft complex128",
                                   "rel_l2_gpu_vs_it": float(np.linalg.norm(G - fout) / np.linalg.norm(fout))}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
