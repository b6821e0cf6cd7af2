#!/usr/bin/env python3
"""Benchmark of the projected GEMM / cross-correlation on one MI355X.

Headline workload (recognition-shaped projected GEMM): 1024 query images x
8192 database images, each a 64 x 64 Gaussian-smoothed noise image with values
0..255 (K = 4096); the database is stored as 8192 rows of 4096 (B^T).  L = 64
DCT-II, FP32 operands and accumulation, r = 16.  One step = the whole hot path
on inputs already resident in HBM: one launch that projects and packs A and B,
then the reduced MFMA contraction over r * K / L projected indices (paper
Sec. III-B), with the library's default tile.  The steps cycle through 4
copies of the inputs (604 MB, more than the 256 MB last-level cache), so every
step reads its inputs from HBM; the rate with one copy (inputs cache-warm) is
reported next to it.

Prints ONE JSON line.  `value` is exact-equivalent TFLOP/s (2 M K W flops per
step, whatever r).  Extra sections are compact tables ({"cols": [...],
"rows": [[...], ...]}); --detail PATH writes the same object, indented.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("PROJGEMM_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "projgemm_tune_bench.json"))

M, K, W, L = 1024, 4096, 8192, 64
HEADLINE_R = 16
NCOPY = 4                                    # rotated input copies (4 x 151 MB)
SWEEP = [1, 2, 4, 8, 12, 16, 24, 32, 48, 64]
PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0, "bf16x3": 2500.0, "f16x3": 2500.0,
        "fp8": 5000.0, "fp8x2": 5000.0}      # dense MFMA TFLOP/s of the operand format
MFMA_PER_PRODUCT = {"bf16x3": 3, "f16x3": 3, "fp8x2": 3}
PEAK_HBM = 8000.0                            # GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f32_recognition_traffic.md")
SECTIONS = ["sweep", "precisions", "plain", "cfg1", "static_database", "klt", "pca2d", "conv", "batched", "mlp"]
PROFILE_CASES = ["gemm", "gemm-bf16", "gemm-fp8", "batched", "conv", "mlp"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_ms(fn, reps: int, warmup: int, warm_s: float = 0.1) -> float:
    """Mean milliseconds per call over reps calls after a warm-up of at least
    `warmup` calls and warm_s seconds (the extra sections follow host-only
    work, after which the GPU clocks ramp up again only under load)."""
    import torch
    t_end = time.perf_counter() + warm_s
    n = 0
    while n < warmup or time.perf_counter() < t_end:
        fn()
        n += 1
        if n % 10 == 0:
            torch.cuda.synchronize()
    from paper_1411_2860_amd import autotune
    return autotune._time_ms(fn, reps, warmup=0)


def graph_us(fn, out, calls=20, replays=20):
    """GPU microseconds per call with host submission out of the way: `calls`
    calls captured in one HIP graph and replayed.  Every checking replay starts
    from a cleared output (eager work and a synchronisation between replays)
    and must reproduce the eager result bit for bit; None if not."""
    import torch
    fn()
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(calls):
            fn()
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            return None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    if not torch.equal(out, ref):
        return None
    return e0.elapsed_time(e1) * 1e3 / (calls * replays)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in ("gemm.hip", "pack.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_1411_2860_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(A, Bt, r):
    """The FP64 oracle as it stands on a bounded sample: the first `rows` query
    rows against all 8192 database columns (the B projection is included in
    full), sized from a short calibration to about 12 s of host time on all
    threads; then the same on one thread with fewer rows (about 8 s)."""
    import oracle
    C, D = oracle.basis("dct2", L)
    cols = np.arange(W)
    Bk = np.ascontiguousarray(Bt.T)

    def run(n):
        t0 = time.perf_counter()
        oracle.gemm_proj_block(A, Bk, C, D, r, np.arange(n), cols)
        return time.perf_counter() - t0

    def measure(budget):
        t8, t40 = run(16), run(144)      # the B projection is a fixed cost: two sizes separate it
        per_row = max((t40 - t8) / 128.0, 1e-4)
        rows = int((budget - t8) / per_row) + 16 if t8 < budget else 16
        rows = min(M, max(8, rows // 8 * 8))
        return rows, run(rows)

    nthreads = oracle.threads()
    rows, t = measure(12.0)
    oracle.set_threads(1)
    rows1, t1 = measure(8.0)
    oracle.set_threads(nthreads)
    return {"value": round(2.0 * rows * K * W / t / 1e12, 6), "unit": "exact-equivalent TFLOP/s",
            "cores": nthreads, "kind": "oracle",
            "sample": f"{rows} of {M} query rows x all {W} database columns, r={r}, L={L}, "
                      f"FP64 pipeline (project A, project B, accumulate); {t:.1f} s",
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "value_1core": round(2.0 * rows1 * K * W / t1 / 1e12, 6),
            "sample_1core": f"{rows1} query rows, one thread; {t1:.1f} s"}


def profile_case(case, dev, iters=5):
    """A few iterations of one workload, for kernel traces and counters."""
    import torch
    from paper_1411_2860_amd import inputs, projgemm as pg
    done = []
    if case in ("gemm-bf16", "gemm-fp8"):
        A = torch.from_numpy(inputs.image_rows(M, seed_base=inputs.SEED_IMG_BASE).astype(np.float32)).to(dev)
        Bt = torch.from_numpy(inputs.image_rows(W, seed_base=inputs.SEED_IMG_BASE, first=M).astype(np.float32)).to(dev)
        basis = pg.Basis("dct2", L)
        plan = [("bf16", 16), ("bf16", 64), ("bf16x3", 16)] if case == "gemm-bf16" else [("fp8", 8), ("fp8x2", 8)]
        for prec, r in plan:
            cfg = -1           # the library's default tile (no tuning inside a traced run)
            Ap, Bp = pg.pack_ab(A, Bt, r, basis, prec=prec, transB=True)
            R = torch.empty((M, W), dtype=torch.float32, device=dev)
            torch.cuda.synchronize()
            for _ in range(iters):
                pg.pack_ab(A, Bt, r, basis, prec=prec, transB=True, out_a=Ap, out_b=Bp)
                pg.gemm_packed(Ap, Bp, r, M, W, K, L, r, r, prec=prec, out=R, tile_cfg=cfg)
            torch.cuda.synchronize()
            done.append([prec, r, cfg])
    elif case == "batched":
        shapes = inputs.batched_shapes()
        As = [torch.from_numpy(inputs.smoothed_rows(m, k, sigma=4.0, seed=6400 + i).astype(np.float32)).to(dev)
              for i, (m, w, k) in enumerate(shapes)]
        Bs = [torch.from_numpy(inputs.gaussian_matrix(k, w, seed=64000 + i).astype(np.float32)).to(dev)
              for i, (m, w, k) in enumerate(shapes)]
        bb = pg.Basis("dct2", 16)
        for prec, r in [("bf16x3", 4), ("bf16", 16)]:
            cfg = 16           # the tile the autotuner picks for both in the timed run (no tuning when traced)
            outs = pg.gemm_batched(As, Bs, r, bb, prec=prec, tile_cfg=cfg)
            ws = torch.empty(pg.gemm_batched_workspace_bytes(pg._descs(As, Bs, outs), 16, r, prec, cfg),
                             dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            for _ in range(iters):
                pg.gemm_batched(As, Bs, r, bb, prec=prec, outs=outs, tile_cfg=cfg, workspace=ws)
            torch.cuda.synchronize()
            done.append([prec, r, cfg])
    elif case == "conv":
        Wc = 1 << 22
        s = inputs.ar2_signal(Wc, seed=inputs.SEED_AR2)
        sd = torch.from_numpy(s.astype(np.float32)).to(dev)
        plan = [(16384, "dct2", 256, 16, "block"), (16384, "dct2", 256, 256, "block"), (16384, "dct2", 256, 1, "full"),
                (16384, "dct2", 256, 16, "full"), (16384, "dct2", 256, 256, "full"), (600, "haar", 2, 1, "block"),
                (600, "haar", 2, 1, "full")]
        for N, kind, Lc, r, rate in plan:
            k, _ = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
            kd = torch.from_numpy(k.astype(np.float32)).to(dev)
            b = pg.Basis(kind, Lc)
            y = torch.empty(Wc - N + 1, dtype=torch.float32, device=dev)
            ws = torch.empty(pg.conv1d_workspace_bytes(Wc, N, Lc, r, rate=rate), dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            for _ in range(iters):
                pg.conv1d(sd, kd, r, b, out=y, workspace=ws, rate=rate)
            torch.cuda.synchronize()
            done.append([N, kind, Lc, r, rate])
    elif case == "mlp":
        from paper_1411_2860_amd.autograd import proj_matmul
        X = torch.from_numpy((inputs.image_rows(4096, seed_base=8000) / 255.0).astype(np.float32)).to(dev)
        W1 = torch.from_numpy(inputs.gaussian_matrix(4096, 4096, seed=5, scale=1 / 64.0).astype(np.float32)).to(dev)
        W2 = torch.from_numpy(inputs.gaussian_matrix(4096, 1024, seed=6, scale=1 / 64.0).astype(np.float32)).to(dev)
        T = torch.from_numpy(inputs.gaussian_matrix(4096, 1024, seed=8).astype(np.float32)).to(dev)
        W1.requires_grad_()
        W2.requires_grad_()
        bm = pg.Basis("dct2", L)
        for _ in range(iters):
            W1.grad = W2.grad = None
            H = torch.nn.functional.gelu(proj_matmul(X, W1, 8, bm, "bf16"), approximate="tanh")
            loss = 0.5 * torch.mean((proj_matmul(H, W2, 16, bm, "bf16") - T) ** 2)
            loss.backward()
        torch.cuda.synchronize()
        done.append(["mlp", 8, 16])
    print(json.dumps({"profile": case, "iterations": iters, "cases": done}), flush=True)


def f3(x):
    return float(f"{x:.3e}")


def table(cols, rows):
    return {"cols": cols, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--r", type=int, default=HEADLINE_R)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma list of extra sections (" + ",".join(SECTIONS) + ") or 'none'")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--detail", default=None, help="also write the result object, indented, to this file")
    ap.add_argument("--profile", nargs="?", const="gemm", default=None, choices=PROFILE_CASES,
                    help="gemm: headline only, few steps, no CPU leg, plus a plain copy of known size "
                         "(for the HBM byte counters); the other cases run a few iterations of one "
                         "workload for a kernel trace and print a short JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path (sharding over the "
              "database columns is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_2860_amd import autotune, inputs, projgemm as pg
    import oracle

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    pg.lib()
    dev = torch.device("cuda:0")
    if args.profile not in (None, "gemm"):
        profile_case(args.profile, dev)
        return
    sections = [] if args.sections == "none" else [s for s in args.sections.split(",") if s]
    if args.profile:
        sections, args.no_cpu = [], True
        args.steps, args.warmup = min(args.steps, 5), min(args.warmup, 2)

    log("generating inputs")
    A = inputs.image_rows(M, seed_base=inputs.SEED_IMG_BASE)
    Bt = inputs.image_rows(W, seed_base=inputs.SEED_IMG_BASE, first=M)
    A32 = torch.from_numpy(A.astype(np.float32))
    B32 = torch.from_numpy(Bt.astype(np.float32))
    ncopy = 1 if args.profile else NCOPY
    Ads = [A32.to(dev) for _ in range(ncopy)]
    Bds = [B32.to(dev) for _ in range(ncopy)]
    Ad, Bd = Ads[0], Bds[0]
    basis = pg.Basis("dct2", L)
    C, D = oracle.basis("dct2", L)       # the oracle's own matrices for its references

    if args.profile:
        # plain copies of known size (256 MiB read + 256 MiB written), for
        # scaling the HBM byte counters: the runtime's device-to-device copy
        # and an elementwise FP32 kernel
        src = torch.ones(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        srcf = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dstf = torch.empty_like(srcf)
        torch.add(srcf, 1.0, out=dstf)
        torch.cuda.synchronize()
        del src, dst, srcf, dstf

    def timed(r, prec, steps, warmup, b=basis, Lb=L, warm_s=0.0, copies=1, tile_cfg=None):
        """steps timed steps after `warmup` untimed ones, cycling through the
        first `copies` input copies; with warm_s > 0 the warm-up also runs
        until that much wall time has passed.  Returns the wall-clock ms per
        step and the mean pack and contraction ms from HIP events recorded
        around each launch on the launching (current) stream.  tile_cfg None:
        the autotuner's choice; -1: the library's default for the shape."""
        cfg = autotune.tune_gemm(M, W, K, Lb, r, prec, reps=3, basis=b) if tile_cfg is None else tile_cfg
        Ap = torch.empty(pg.packed_bytes(M, K, Lb, r, prec), dtype=torch.uint8, device=dev)
        Bp = torch.empty(pg.packed_bytes(W, K, Lb, r, prec), dtype=torch.uint8, device=dev)
        R = torch.empty((M, W), dtype=torch.float32, device=dev)

        def step(i, ev=None):
            if ev is not None:
                ev[0].record()
            pg.pack_ab(Ads[i % copies], Bds[i % copies], r, b, prec=prec, transB=True, out_a=Ap, out_b=Bp)
            if ev is not None:
                ev[1].record()
            pg.gemm_packed(Ap, Bp, r, M, W, K, Lb, r, r, prec=prec, out=R, tile_cfg=cfg)
            if ev is not None:
                ev[2].record()
        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() + warm_s
        while time.perf_counter() < t_warm:
            for i in range(10):
                step(i)
            torch.cuda.synchronize()
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(i, evs[i])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        pms = float(np.mean([a.elapsed_time(b_) for a, b_, _ in evs]))
        kms = float(np.mean([b_.elapsed_time(c) for _, b_, c in evs]))
        return ms, pms, kms, R, cfg

    rng_s = np.random.default_rng(1234)
    srows = np.sort(rng_s.choice(M, 64, replace=False))
    scols = np.sort(rng_s.choice(W, 64, replace=False))
    exact_block = A[srows] @ Bt[scols].T
    proj_cache = {}

    def sampled_errors(r, R):
        got = R[torch.from_numpy(srows).to(dev)][:, torch.from_numpy(scols).to(dev)].double().cpu().numpy()
        if r not in proj_cache:
            proj_cache[r] = oracle.gemm_proj_block(A, np.ascontiguousarray(Bt.T), C, D, r, srows, scols)
        proj = proj_cache[r]
        return oracle.rel_fro(got, exact_block), oracle.rel_fro(got, proj), oracle.rel_fro(proj, exact_block)

    exact_flops = 2.0 * M * K * W
    r = args.r
    log(f"headline r={r}")
    # the W untimed warm-up steps are extended to at least 0.5 s of wall time:
    # after the host-side input generation the GPU clock starts from idle,
    # and the first milliseconds of matrix work run up to 15 % slower
    warm_s = 0.5
    # the headline runs the library's default tile (a fixed choice, so the
    # counters recorded for it in profiles/ stay attached to the same kernel)
    ms, pms, kms, R, cfg = timed(r, "f32", args.steps, args.warmup, copies=ncopy, warm_s=warm_s, tile_cfg=-1)
    ms_w, pms_w, kms_w, _, _ = timed(r, "f32", args.steps, args.warmup, copies=1, warm_s=warm_s, tile_cfg=-1)
    value = exact_flops / (ms * 1e-3) / 1e12
    G = K // L
    gemm_flops = 2.0 * M * W * r * G
    achieved = gemm_flops / (kms * 1e-3) / 1e12
    pack_bytes = 4.0 * (M + W) * K + 4.0 * (M + W) * r * G      # read A and B, write both packs (FP32)

    traffic = None
    mfma_util = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
        if tr.get("sources_hash") == kernel_sources_hash() and tr.get("r") == r and tr.get("tile_cfg") == cfg:
            traffic = tr.get("gemm_bytes_per_launch")
            mfma_util = tr.get("gemm_mfma_busy_frac")

    out = {
        "metric": "exact-equivalent TFLOP/s and rel. error vs FP64 per projection count r",
        "value": round(value, 3),
        "unit": "TFLOP/s (exact-equivalent, 2*M*K*W per step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded smoothed 64x64 images, 0..255)",
        "config": {"workload": f"recognition-shaped projected GEMM: {M} queries x {W} database images "
                               f"of 64x64 (K={K}), database stored {W}x{K}, L={L} DCT-II, r={r}, FP32; "
                               f"steps cycle through {ncopy} input copies (inputs read from HBM)",
                   "M": M, "K": K, "W": W, "L": L, "r": r, "basis": "dct2", "prec": "f32", "tile_cfg": cfg,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f32"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["f32"], 4), "traffic": traffic,
                     "kernel": "gemm_kernel (reduced contraction, FP32)",
                     "kernel_ms": round(kms, 5), "algorithmic_flops_per_launch": gemm_flops,
                     "mfma_busy_frac": mfma_util},
        "warm": {"ms_per_step": round(ms_w, 5), "value": round(exact_flops / (ms_w * 1e-3) / 1e12, 3),
                 "kernel_ms": round(kms_w, 5), "note": "one input copy: inputs stay in the 256 MB cache"},
        "pack": {"bytes": pack_bytes, "ms_cold": round(pms, 5), "ms_warm": round(pms_w, 5),
                 "gbs_cold": round(pack_bytes / (pms * 1e-3) / 1e9, 1),
                 "gbs_warm": round(pack_bytes / (pms_w * 1e-3) / 1e9, 1), "peak_gbs": PEAK_HBM},
    }
    e_exact, e_proj, _ = sampled_errors(r, R)
    out["rel_err_vs_fp64_exact"] = f3(e_exact)
    out["rel_err_vs_fp64_projected"] = f3(e_proj)
    del R
    del Ads[1:], Bds[1:]

    def section(name, fn):
        if name not in sections:
            return
        log(f"section {name}")
        t0 = time.perf_counter()
        try:
            out[name] = fn()
        except Exception as ex:   # a failing section is reported, the headline still prints
            out[name] = {"error": f"{type(ex).__name__}: {ex}"}
        log(f"section {name} done in {time.perf_counter() - t0:.1f} s")

    def sec_sweep():
        rows = []
        for rr in SWEEP:
            ms_r, _, kms_r, R_r, cfg_r = timed(rr, "f32", 10, 3, warm_s=0.1)
            e1, e2, e3 = sampled_errors(rr, R_r)
            rows.append([rr, round(ms_r, 4), round(kms_r, 4), cfg_r, round(exact_flops / (ms_r * 1e-3) / 1e12, 1),
                         round(2.0 * M * W * rr * G / (kms_r * 1e-3) / 1e12 / PEAK["f32"], 3), f3(e1), f3(e2), f3(e3)])
            del R_r
        return table(["r", "ms", "gemm_ms", "cfg", "tflops_eq", "gemm_frac", "err_exact", "err_proj", "err_method"],
                     rows)

    def sec_precisions():
        rows = []
        plan = [(p, rr) for p in ("bf16", "f16", "bf16x3", "f16x3") for rr in (1, 4, 16, 64)]
        plan += [(p, rr) for p in ("fp8", "fp8x2") for rr in (1, 2, 4, 8)]
        for prec, rr in plan:
            ms_p, _, kms_p, R_p, cfg_p = timed(rr, prec, 10, 3, warm_s=0.05)
            e1, e2, _ = sampled_errors(rr, R_p)
            mfma_flops = 2.0 * M * W * rr * G * MFMA_PER_PRODUCT.get(prec, 1)
            rows.append([prec, rr, round(ms_p, 4), round(kms_p, 4), cfg_p,
                         round(exact_flops / (ms_p * 1e-3) / 1e12, 1),
                         round(mfma_flops / (kms_p * 1e-3) / 1e12 / PEAK[prec], 3), f3(e1), f3(e2)])
            del R_p
        return table(["prec", "r", "ms", "gemm_ms", "cfg", "tflops_eq", "gemm_frac_own_peak", "err_exact",
                      "err_proj"], rows)

    def sec_plain():
        # plain (unprojected) FP32 GEMM through the same kernels: the identity
        # basis with all projections kept only permutes the contraction index
        plain = pg.Basis("identity", 4)
        ms_p, _, kms_p, R_p, cfg_p = timed(4, "f32", 10, 3, b=plain, Lb=4)
        got = R_p[torch.from_numpy(srows).to(dev)][:, torch.from_numpy(scols).to(dev)].double().cpu().numpy()
        return {"ms": round(ms_p, 5), "gemm_ms": round(kms_p, 5), "cfg": cfg_p,
                "tflops": round(exact_flops / (ms_p * 1e-3) / 1e12, 1),
                "gemm_frac": round(exact_flops / (kms_p * 1e-3) / 1e12 / PEAK["f32"], 4),
                "err_exact": f3(oracle.rel_fro(got, exact_block)), "speedup_of_headline_r": round(ms_p / ms, 3),
                "speedup_of_headline_r_warm": round(ms_p / ms_w, 3)}

    def sec_cfg1():
        # the parity configuration: FP64, M = N = K = 256, L = 16 DCT-II
        A1 = inputs.smoothed_field(256, 256, sigma=4.0, seed=inputs.SEED_CFG1_A)
        B1 = inputs.gaussian_matrix(256, 256, seed=inputs.SEED_CFG1_B)
        A1d = torch.from_numpy(A1).to(dev)
        B1d = torch.from_numpy(B1).to(dev)
        b16 = pg.Basis("dct2", 16)
        C16, D16 = oracle.basis("dct2", 16)
        ex = A1 @ B1
        rows = []
        for rr in (1, 2, 4, 8, 16):
            Rr = torch.empty((256, 256), dtype=torch.float64, device=dev)
            ws = torch.empty(pg.gemm_workspace_bytes(256, 256, 256, 16, rr, "f64"), dtype=torch.uint8, device=dev)
            t = timed_ms(lambda: pg.gemm(A1d, B1d, rr, b16, prec="f64", out=Rr, workspace=ws), 20, warmup=3)
            got = Rr.cpu().numpy()
            proj = oracle.gemm_proj(A1, B1, C16, D16, rr)
            rows.append([rr, round(t * 1e3, 2), f3(oracle.rel_fro(got, ex)), f3(oracle.rel_fro(got, proj))])
        return table(["r", "us", "err_exact", "err_proj"], rows)

    def sec_static_database():
        # the database (8192 images) packed once at r = 64 (a projection-major
        # pack serves every r <= 64); each step projects the 1024 queries and
        # contracts -- the deployment where the database is static
        Bp64 = pg.pack_b(Bd, 64, basis, prec="f32", transB=True)
        torch.cuda.synchronize()
        rows = []
        for rr in (1, 4, 8, 16, 64):
            cfg_s = autotune.tune_gemm(M, W, K, L, rr, "f32", reps=3, basis=basis)
            Ap = torch.empty(pg.packed_bytes(M, K, L, rr, "f32"), dtype=torch.uint8, device=dev)
            R_s = torch.empty((M, W), dtype=torch.float32, device=dev)

            def st():
                pg.pack_a(Ad, rr, basis, prec="f32", out=Ap)
                pg.gemm_packed(Ap, Bp64, rr, M, W, K, L, rr, 64, prec="f32", out=R_s, tile_cfg=cfg_s)
            t = timed_ms(st, args.steps, warmup=args.warmup)
            e_exact, e_proj, _ = sampled_errors(rr, R_s)
            rows.append([rr, round(t, 4), cfg_s, round(exact_flops / (t * 1e-3) / 1e12, 1), f3(e_exact), f3(e_proj)])
            del R_s, Ap
        del Bp64
        return table(["r", "ms", "cfg", "tflops_eq", "err_exact", "err_proj"], rows)

    def sec_klt():
        # data-adaptive basis: block second moments of 2048 database images on
        # the device, eigenbasis on the host; then the headline workload with
        # that basis against the DCT-II at each r (sampled errors vs FP64)
        train = Bd[:2048]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Mm = pg.block_moments(train, L)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kb, eig = pg.klt_basis(Mm)
        t2 = time.perf_counter()
        # the oracle's own eigenbasis of the same training blocks (moments in
        # FP64 on the host) for the projected reference
        Ck, Dk, _ = oracle.basis_klt(oracle.block_moments(Bt[:2048].astype(np.float64), L))
        rows = []
        for rr in (1, 2, 4, 8, 16):
            ms_k, _, _, R_k, cfg_k = timed(rr, "f32", 10, 3, b=kb, Lb=L, warm_s=0.1)
            got = R_k[torch.from_numpy(srows).to(dev)][:, torch.from_numpy(scols).to(dev)].double().cpu().numpy()
            e_klt = oracle.rel_fro(got, exact_block)
            proj = oracle.gemm_proj_block(A, np.ascontiguousarray(Bt.T), Ck, Dk, rr, srows, scols)
            ms_d, _, _, R_d, _ = timed(rr, "f32", 10, 3, warm_s=0.1)
            e_dct, _, _ = sampled_errors(rr, R_d)
            rows.append([rr, round(ms_k, 4), round(ms_d, 4), f3(e_klt), f3(e_dct), f3(oracle.rel_fro(got, proj))])
            del R_k, R_d
        res = table(["r", "klt_ms", "dct_ms", "err_exact_klt", "err_exact_dct", "err_proj_klt"], rows)
        res.update({"train_images": 2048, "moments_ms": round((t1 - t0) * 1e3, 3),
                    "eigen_host_ms": round((t2 - t1) * 1e3, 3)})
        return res

    def sec_pca2d():
        # 2D-PCA on the Yale-A shape (15 classes x 11 images of 288 x 288, the
        # first 5 per class for training, 10 axes): the GEMMs of the scatter
        # matrix and of the training / test features on one of L projections,
        # against the same GEMMs exact; recognition rate of the full pipeline
        from paper_1411_2860_amd.pca2d import PCA2D
        imgs, labels, idx = inputs.face_classes()
        tr = torch.from_numpy(imgs[idx < 5]).float().to(dev)
        te = torch.from_numpy(imgs[idx >= 5]).float().to(dev)
        ltr, lte = labels[idx < 5], labels[idx >= 5]
        J, m, n = tr.shape
        mean = tr.mean(0)
        Ast = (tr - mean).reshape(J * m, n).contiguous()
        Bst = (te - mean).reshape(te.shape[0] * m, n).contiguous()
        rows = []
        for lab, b, rr in [("exact", pg.Basis("identity", 1), 1), ("dct2 L=8", pg.Basis("dct2", 8), 1),
                           ("dct2 L=12", pg.Basis("dct2", 12), 1), ("dct2 L=16", pg.Basis("dct2", 16), 1)]:
            model = PCA2D(b, rr, 10).fit(tr)
            rate = float(np.mean(ltr[model.match(te).cpu().numpy()] == lte))
            X = model.X
            t_g = timed_ms(lambda: pg.gemm(Ast, Ast, rr, b, transA=True), 20, warmup=3)
            t_s = timed_ms(lambda: pg.gemm(Ast, X, rr, b), 20, warmup=3)
            t_t = timed_ms(lambda: pg.gemm(Bst, X, rr, b), 20, warmup=3)
            rows.append([lab, rr, round(rate, 4), round(t_g, 4), round(t_s, 4), round(t_t, 4),
                         round(t_g + t_s + t_t, 4)])
        ex = rows[0][-1]
        for row in rows:
            row.append(round(ex / row[-1], 2))
        res = table(["basis", "r", "recognition", "scatter_ms", "train_ms", "test_ms", "gemm_ms", "speedup"], rows)
        res["images"] = [int(J), int(te.shape[0]), int(m), int(n)]
        return res

    def sec_conv():
        Wc, Lc = 1 << 22, 256
        s = inputs.ar2_signal(Wc, seed=inputs.SEED_AR2)
        sd = torch.from_numpy(s.astype(np.float32)).to(dev)
        bc = pg.Basis("dct2", Lc)
        Cc, Dc = oracle.basis("dct2", Lc)
        ident = pg.Basis("identity", Lc)
        full, block, plain_rows = [], [], []
        rsweep = [1, 2, 4, 8, 16, 32, 64, 128, 256]
        for N in (1024, 4096, 16384):
            k, o = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
            kd = torch.from_numpy(k.astype(np.float32)).to(dev)
            nout = Wc - N + 1
            y = torch.empty(nout, dtype=torch.float32, device=dev)
            ms_rng = np.random.default_rng(N)
            msel = np.unique(np.concatenate([[0, nout - 1, o], ms_rng.integers(0, nout, 61)]))
            mt = torch.from_numpy(msel).to(dev)
            exact = np.array([np.dot(k, s[m:m + N]) for m in msel])
            flops = 2.0 * nout * N
            runs = [(rr, "full") for rr in rsweep] + ([(rr, "block") for rr in rsweep] if N == 16384 else [])
            for rr, rate in runs:
                ws = torch.empty(pg.conv1d_workspace_bytes(Wc, N, Lc, rr, rate=rate), dtype=torch.uint8, device=dev)
                t = timed_ms(lambda: pg.conv1d(sd, kd, rr, bc, out=y, workspace=ws, rate=rate), 10, warmup=3)
                got = y[mt].double().cpu().numpy()
                if rate == "full":
                    proj = oracle.xcorr_proj_at(s, k, Cc, Dc, rr, msel)
                else:
                    proj = oracle.xcorr_proj_block_rate_at(s, k, Cc, Dc, rr, msel)
                row = [N, rr, round(t, 4), round(flops / (t * 1e-3) / 1e12, 1), f3(oracle.rel_fro(got, exact)),
                       f3(oracle.rel_fro(got, proj))]
                (full if rate == "full" else block).append(row)
                del ws
            # plain cross-correlation through the same kernels: identity basis,
            # all 256 projections kept (the exact result)
            ws = torch.empty(pg.conv1d_workspace_bytes(Wc, N, Lc, Lc), dtype=torch.uint8, device=dev)
            t = timed_ms(lambda: pg.conv1d(sd, kd, Lc, ident, out=y, workspace=ws), 10, warmup=3)
            got = y[mt].double().cpu().numpy()
            plain_rows.append([N, round(t, 4), round(flops / (t * 1e-3) / 1e12, 1), f3(oracle.rel_fro(got, exact))])
            del ws
        cols = ["N", "r", "ms", "tflops_eq", "err_exact", "err_proj"]
        res = {"W": Wc, "L": Lc, "full_rate": table(cols, full), "block_rate": table(cols, block),
               "plain": table(["N", "ms", "tflops", "err_exact"], plain_rows)}
        # the two realisations of the full rate on long kernels: the direct
        # contraction and the frequency-domain one, with the library's choice
        frows = []
        for Lf, N, rr in [(16, 16384, 1), (16, 16384, 16), (8, 8192, 8), (32, 32768, 32), (4, 4096, 4),
                          (16, 1024, 16), (64, 65536, 8), (256, 16384, 16)]:
            bf = pg.Basis("dct2", Lf)
            Cf, Df = oracle.basis("dct2", Lf)
            k, _ = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
            kd = torch.from_numpy(k.astype(np.float32)).to(dev)
            nout = Wc - N + 1
            y = torch.empty(nout, dtype=torch.float32, device=dev)
            msel = np.unique(np.random.default_rng(N + Lf).integers(0, nout, 61))
            proj = oracle.xcorr_proj_at(s, k, Cf, Df, rr, msel)
            times = {}
            for meth in ("direct", "fft"):
                nb = pg.conv1d_method_workspace_bytes(Wc, N, Lf, rr, meth)
                if nb == 0:
                    times[meth] = (None, None)
                    continue
                ws = torch.empty(nb, dtype=torch.uint8, device=dev)
                t = timed_ms(lambda: pg.conv1d_method(sd, kd, rr, bf, method=meth, out=y, workspace=ws), 5, warmup=2)
                got = y[torch.from_numpy(msel).to(dev)].double().cpu().numpy()
                times[meth] = (round(t, 4), f3(oracle.rel_fro(got, proj)))
                del ws
            auto = "fft" if pg.conv1d_method_workspace_bytes(Wc, N, Lf, rr, "auto") == \
                pg.conv1d_method_workspace_bytes(Wc, N, Lf, rr, "fft") else "direct"
            frows.append([Lf, N, rr, times["direct"][0], times["fft"][0], auto, times["direct"][1], times["fft"][1]])
        res["fft_vs_direct"] = table(["L", "N", "r", "direct_ms", "fft_ms", "auto", "err_proj_direct",
                                      "err_proj_fft"], frows)
        # circular mode on the same signal (period 2^22), N = 16384
        k, _ = inputs.excerpt_kernel(s, 16384, seed=inputs.SEED_KERNEL)
        kd = torch.from_numpy(k.astype(np.float32)).to(dev)
        yc = torch.empty(Wc, dtype=torch.float32, device=dev)
        crows = []
        for rr in (16, 64, 256):
            ws = torch.empty(pg.lib().pj_conv1d_circular_workspace_bytes(Wc, 16384, Lc, rr, 1), dtype=torch.uint8,
                             device=dev)
            t = timed_ms(lambda: pg.conv1d_circular(sd, kd, rr, bc, out=yc, workspace=ws), 10, warmup=3)
            crows.append([rr, round(t, 4), round(2.0 * Wc * 16384 / (t * 1e-3) / 1e12, 1)])
            del ws
        res["circular_N16384"] = table(["r", "ms", "tflops_eq"], crows)
        # the paper's CONV operating points: kernels of 600 and 1200 samples,
        # Haar L = 2 and 4, one projection or all, every or every L-th output
        # (the rest interpolated), on a block of 20000 samples and on 2^22
        prow = []
        for Wp in (20000, 1 << 22):
            sp = inputs.ar2_signal(Wp, seed=inputs.SEED_AR2)
            spd = torch.from_numpy(sp.astype(np.float32)).to(dev)
            for Lh in (2, 4):
                hb = pg.Basis("haar", Lh)
                for N in (600, 1200):
                    kp, _ = inputs.excerpt_kernel(sp, N, seed=inputs.SEED_KERNEL)
                    kpd = torch.from_numpy(kp.astype(np.float32)).to(dev)
                    nout = Wp - N + 1
                    y = torch.empty(nout, dtype=torch.float32, device=dev)
                    msel = np.unique(np.random.default_rng(N + Lh).integers(0, nout, 2000))
                    exact = np.array([np.dot(kp, sp[m:m + N]) for m in msel])
                    for rr in sorted({1, Lh}):
                        for rate in ("block", "full"):
                            ws = torch.empty(pg.conv1d_workspace_bytes(Wp, N, Lh, rr, rate=rate), dtype=torch.uint8,
                                             device=dev)
                            call = lambda: pg.conv1d(spd, kpd, rr, hb, out=y, workspace=ws, rate=rate)
                            t = timed_ms(call, 30, warmup=5)
                            got = y[torch.from_numpy(msel).to(dev)].double().cpu().numpy()
                            tg = graph_us(call, y)
                            prow.append([Wp, N, Lh, rr, rate[0], round(t * 1e3, 1), round(nout / (t * 1e-3) / 1e6),
                                         round(oracle.snr_db(exact, got), 1), None if tg is None else round(tg, 2)])
                            del ws
        res["paper_points"] = table(["W", "N", "L", "r", "rate(b=block,f=full)", "us", "msamples_s", "snr_db",
                                     "us_graph"], prow)
        res["paper_points"]["note"] = ("us: per call issued from Python (at 20000 samples mostly host submission); "
                                       "us_graph: per call replayed from a captured HIP graph, GPU time only")
        return res

    def sec_batched():
        shapes = inputs.batched_shapes()
        As, Bs = [], []
        for i, (m, w, k) in enumerate(shapes):
            As.append(torch.from_numpy(inputs.smoothed_rows(m, k, sigma=4.0, seed=6400 + i).astype(np.float32)).to(dev))
            Bs.append(torch.from_numpy(inputs.gaussian_matrix(k, w, seed=64000 + i).astype(np.float32)).to(dev))
        flops = sum(2.0 * m * w * k for m, w, k in shapes)
        io_bytes = sum(4.0 * (m * k + k * w + m * w) for m, w, k in shapes)
        Lb = 16
        bb = pg.Basis("dct2", Lb)
        Cb, Db = oracle.basis("dct2", Lb)
        rows = []
        plan = [(p, rr) for p in ("bf16x3", "bf16") for rr in (1, 2, 4, 8, 16)] + [("fp8", rr) for rr in (1, 2, 4, 8)]
        for prec, rr in plan:
            cfg_b = autotune.tune_batched(As, Bs, rr, bb, prec=prec, reps=2, candidates=[0, 6, 9, 11, 13, 16, 17])
            outs = pg.gemm_batched(As, Bs, rr, bb, prec=prec, tile_cfg=cfg_b)
            descs = pg._descs(As, Bs, outs)
            ws = torch.empty(pg.gemm_batched_workspace_bytes(descs, Lb, rr, prec, cfg_b), dtype=torch.uint8,
                             device=dev)
            t = timed_ms(lambda: pg.gemm_batched(As, Bs, rr, bb, prec=prec, outs=outs, tile_cfg=cfg_b,
                                                 workspace=ws), 5, warmup=2)
            errs = []
            rng = np.random.default_rng(rr)
            for i in range(0, len(shapes), 8):      # every 8th problem, 8 x 8 samples
                m, w, k = shapes[i]
                rws = np.sort(rng.choice(m, 8, replace=False))
                cls = np.sort(rng.choice(w, 8, replace=False))
                got = outs[i][torch.from_numpy(rws).to(dev)][:, torch.from_numpy(cls).to(dev)].double().cpu().numpy()
                A64 = As[i].double().cpu().numpy()
                B64 = Bs[i].double().cpu().numpy()
                proj = oracle.gemm_proj_block(A64, B64, Cb, Db, rr, rws, cls)
                errs.append((oracle.rel_fro(got, proj), oracle.rel_fro(got, A64[rws] @ B64[:, cls])))
            rows.append([prec, rr, cfg_b, round(t, 3), round(flops / (t * 1e-3) / 1e12, 1),
                         round(io_bytes / (t * 1e-3) / 1e9, 1), f3(max(e[0] for e in errs)),
                         f3(max(e[1] for e in errs))])
            del ws, outs
        res = table(["prec", "r", "cfg", "ms", "tflops_eq", "io_gbs", "err_proj_max", "err_exact_max"], rows)
        res.update({"problems": len(shapes), "L": Lb, "io_bytes": io_bytes,
                    "io_note": "A, B read and R written once (FP32), the floor of any implementation"})
        return res

    def sec_mlp():
        from paper_1411_2860_amd.autograd import proj_matmul
        Bsz, Din, Dh, Dout = 4096, 4096, 4096, 1024
        X = (inputs.image_rows(Bsz, seed_base=8000) / 255.0)
        W1 = inputs.gaussian_matrix(Din, Dh, seed=5, scale=1 / 64.0)
        W2 = inputs.gaussian_matrix(Dh, Dout, seed=6, scale=1 / 64.0)
        T = inputs.gaussian_matrix(Bsz, Dout, seed=8)
        Xd = torch.from_numpy(X.astype(np.float32)).to(dev)
        Td = torch.from_numpy(T.astype(np.float32)).to(dev)
        W1d = torch.from_numpy(W1.astype(np.float32)).to(dev).requires_grad_()
        W2d = torch.from_numpy(W2.astype(np.float32)).to(dev).requires_grad_()
        bm = pg.Basis("dct2", L)
        Cm, Dm = oracle.basis("dct2", L)
        rows = []
        plain_flops = 2.0 * Bsz * Din * Dh * 2 + 2.0 * Bsz * Dh * Dout * 3    # fwd + dW1 + fwd + dH + dW2
        for r1, r2 in [(8, 64), (16, 64), (32, 64), (64, 64), (8, 16)]:
            def it():
                W1d.grad = None
                W2d.grad = None
                H = torch.nn.functional.gelu(proj_matmul(Xd, W1d, r1, bm, "bf16"), approximate="tanh")
                Y = proj_matmul(H, W2d, r2, bm, "bf16")
                loss = 0.5 * torch.mean((Y - Td) ** 2)
                loss.backward()
                return loss
            t = timed_ms(it, 5, warmup=2)
            loss = float(it().item())
            # FP64 reference loss through the oracle's closed form A Q B
            H0 = oracle.gemm_proj_closed(X, W1, Cm, Dm, r1)
            Hr = 0.5 * H0 * (1.0 + np.tanh(0.7978845608028654 * (H0 + 0.044715 * H0 ** 3)))
            Yr = oracle.gemm_proj_closed(Hr, W2, Cm, Dm, r2)
            loss_ref = 0.5 * float(np.mean((Yr - T) ** 2))
            rows.append([r1, r2, round(t, 4), round(plain_flops / (t * 1e-3) / 1e12, 1), round(loss, 6),
                         f3(abs(loss - loss_ref) / loss_ref)])
        return table(["r1", "r2", "ms_fwd_bwd", "tflops_eq", "loss", "loss_err_vs_fp64"], rows)

    section("sweep", sec_sweep)
    section("precisions", sec_precisions)
    section("plain", sec_plain)
    section("cfg1", sec_cfg1)
    section("static_database", sec_static_database)
    section("klt", sec_klt)
    section("pca2d", sec_pca2d)
    section("conv", sec_conv)
    section("batched", sec_batched)
    section("mlp", sec_mlp)

    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(A, Bt, r)
    # key order of the printed line: the contract keys first, then the
    # sections, the most looked-at last (a reader of only the end of a long
    # line still sees them)
    order = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
             "vs_baseline", "dtype", "data", "config", "static_database", "klt", "pca2d", "cfg1", "plain", "batched",
             "mlp", "conv", "precisions", "sweep", "rel_err_vs_fp64_exact", "rel_err_vs_fp64_projected", "warm",
             "pack", "roofline", "cpu_baseline"]
    final = {k: out[k] for k in order if k in out}
    final.update({k: v for k, v in out.items() if k not in final})
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(final, f, indent=1)
    print(json.dumps(final, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
