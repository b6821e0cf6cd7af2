#!/usr/bin/env python3
"""Benchmark of the projected GEMM / cross-correlation on one MI355X.

Headline workload (recognition-shaped projected GEMM): 1024 query images x
8192 database images, each a 64 x 64 Gaussian-smoothed noise image with values
0..255 (K = 4096); the database is stored as 8192 rows of 4096 (B^T).  L = 64
DCT-II, FP32 operands and accumulation, r = 16.  One step = the whole hot path
on inputs already resident in HBM: one launch that projects and packs A and B,
then the reduced MFMA contraction over r * K / L projected indices (paper
Sec. III-B), with the tile chosen by the autotuner.

Prints ONE JSON line.  `value` is exact-equivalent TFLOP/s (2 M K W flops per
step, whatever r).  Extra sections: the r sweep with errors against FP64 (exact
product and projected oracle) on sampled outputs, the precision ladder, the
plain FP32 GEMM through the same kernels, the 2^22-sample projected
cross-correlation, the 64-problem batch, and the MLP forward + backward.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("PROJGEMM_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "projgemm_tune_bench.json"))

M, K, W, L = 1024, 4096, 8192, 64
HEADLINE_R = 16
SWEEP = [1, 2, 4, 8, 12, 16, 24, 32, 48, 64]
PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0, "bf16x3": 2500.0, "f16x3": 2500.0,
        "fp8": 5000.0, "fp8x2": 5000.0}      # dense MFMA TFLOP/s of the operand format
MFMA_PER_PRODUCT = {"bf16x3": 3, "f16x3": 3, "fp8x2": 3}
PEAK_HBM = 8000.0                            # GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f32_recognition_traffic.md")
SECTIONS = ["sweep", "precisions", "plain", "static_database", "klt", "pca2d", "conv", "batched", "mlp"]


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


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in ("gemm.hip", "pack.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_1411_2860_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(A, Bt, r):
    """The FP64 oracle on a bounded sample: the first `rows` query rows against
    all 8192 database columns (the B projection is included in full), sized
    from a short calibration to about 15 s of host time."""
    import oracle
    C, D = oracle.basis("dct2", L)
    cols = np.arange(W)
    Bk = np.ascontiguousarray(Bt.T)

    def run(n):
        t0 = time.perf_counter()
        oracle.gemm_proj_block(A, Bk, C, D, r, np.arange(n), cols)
        return time.perf_counter() - t0
    t8, t40 = run(16), run(144)      # the B projection is a fixed cost: two sizes separate it
    per_row = max((t40 - t8) / 128.0, 1e-4)
    rows = int((15.0 - t8) / per_row) + 16 if t8 < 15.0 else 16
    rows = min(M, max(8, rows // 8 * 8))
    t = run(rows)
    return {"value": round(2.0 * rows * K * W / t / 1e12, 6), "unit": "exact-equivalent TFLOP/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{rows} of {M} query rows x all {W} database columns, r={r}, L={L}, "
                      f"FP64 pipeline (project A, project B, accumulate); {t:.1f} s"}


def f3(x):
    return float(f"{x:.3e}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--r", type=int, default=HEADLINE_R)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma list of extra sections (" + ",".join(SECTIONS) + ") or 'none'")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="headline only, few steps, no CPU leg, plus a plain copy of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the projected GEMM path is single-GPU "
              "(sharding over the database columns is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_2860_amd import autotune, inputs, projgemm as pg

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    pg.lib()
    dev = torch.device("cuda:0")
    sections = [] if args.sections == "none" else [s for s in args.sections.split(",") if s]
    if args.profile:
        sections, args.no_cpu = [], True
        args.steps, args.warmup = min(args.steps, 5), min(args.warmup, 2)

    log("generating inputs")
    A = inputs.image_rows(M, seed_base=inputs.SEED_IMG_BASE)
    Bt = inputs.image_rows(W, seed_base=inputs.SEED_IMG_BASE, first=M)
    Ad = torch.from_numpy(A.astype(np.float32)).to(dev)
    Bd = torch.from_numpy(Bt.astype(np.float32)).to(dev)
    basis = pg.Basis("dct2", L)
    import oracle
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

    def timed(r, prec, steps, warmup, b=basis, Lb=L, warm_s=0.0):
        """steps timed steps after `warmup` untimed ones; with warm_s > 0 the
        warm-up also runs until that much wall time has passed (the extra
        sections follow host-only work, after which the GPU clocks ramp up
        again only under load)."""
        cfg = autotune.tune_gemm(M, W, K, Lb, r, prec, reps=3, basis=b)
        Ap = torch.empty(pg.packed_bytes(M, K, Lb, r, prec), dtype=torch.uint8, device=dev)
        Bp = torch.empty(pg.packed_bytes(W, K, Lb, r, prec), dtype=torch.uint8, device=dev)
        R = torch.empty((M, W), dtype=torch.float32, device=dev)

        def step(ev=None):
            pg.pack_ab(Ad, Bd, r, b, prec=prec, transB=True, out_a=Ap, out_b=Bp)
            if ev is not None:
                ev[0].record()
            pg.gemm_packed(Ap, Bp, r, M, W, K, Lb, r, r, prec=prec, out=R, tile_cfg=cfg)
            if ev is not None:
                ev[1].record()
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t_warm = time.perf_counter() + warm_s
        while time.perf_counter() < t_warm:
            for _ in range(10):
                step()
            torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for i in range(steps):
            step(evs[i])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        kms = float(np.mean([a.elapsed_time(e) for a, e in evs]))
        return ms, kms, R, cfg

    rng_s = np.random.default_rng(1234)
    srows = np.sort(rng_s.choice(M, 64, replace=False))
    scols = np.sort(rng_s.choice(W, 64, replace=False))
    exact_block = A[srows] @ Bt[scols].T
    proj_cache = {}

    def sampled_errors(r, R):
        import oracle
        got = R[torch.from_numpy(srows).to(dev)][:, torch.from_numpy(scols).to(dev)].double().cpu().numpy()
        if r not in proj_cache:
            proj_cache[r] = oracle.gemm_proj_block(A, np.ascontiguousarray(Bt.T), C, D, r, srows, scols)
        proj = proj_cache[r]
        return oracle.rel_fro(got, exact_block), oracle.rel_fro(got, proj), oracle.rel_fro(proj, exact_block)

    exact_flops = 2.0 * M * K * W
    r = args.r
    log(f"headline r={r}")
    ms, kms, R, cfg = timed(r, "f32", args.steps, args.warmup)
    value = exact_flops / (ms * 1e-3) / 1e12
    gemm_flops = 2.0 * M * W * r * (K // L)
    achieved = gemm_flops / (kms * 1e-3) / 1e12

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
        if tr.get("sources_hash") == kernel_sources_hash() and tr.get("r") == r and tr.get("tile_cfg") == cfg:
            traffic = tr.get("gemm_bytes_per_launch")

    out = {
        "metric": "exact-equivalent TFLOP/s and rel. error vs FP64 per projection count r",
        "value": round(value, 3),
        "unit": "TFLOP/s (exact-equivalent, 2*M*K*W per step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded smoothed 64x64 images, 0..255)",
        "config": {"workload": f"recognition-shaped projected GEMM: {M} queries x {W} database images "
                               f"of 64x64 (K={K}), database stored {W}x{K}, L={L} DCT-II, r={r}, FP32",
                   "M": M, "K": K, "W": W, "L": L, "r": r, "basis": "dct2", "prec": "f32", "tile_cfg": cfg,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f32"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["f32"], 4), "traffic": traffic,
                     "kernel": "gemm_kernel (reduced contraction, FP32)",
                     "kernel_ms": round(kms, 5), "algorithmic_flops_per_launch": gemm_flops},
    }
    e_exact, e_proj, _ = sampled_errors(r, R)
    out["rel_err_vs_fp64_exact"] = f3(e_exact)
    out["rel_err_vs_fp64_projected"] = f3(e_proj)
    del R

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
        res = []
        for rr in SWEEP:
            ms_r, kms_r, R_r, cfg_r = timed(rr, "f32", 10, 3, warm_s=0.1)
            e1, e2, e3 = sampled_errors(rr, R_r)
            res.append({"r": rr, "ms_per_step": round(ms_r, 5), "gemm_ms": round(kms_r, 5), "tile_cfg": cfg_r,
                        "exact_equiv_tflops": round(exact_flops / (ms_r * 1e-3) / 1e12, 3),
                        "gemm_frac_of_fp32_peak": round(2.0 * M * W * rr * (K // L) / (kms_r * 1e-3) / 1e12
                                                        / PEAK["f32"], 4),
                        "rel_err_vs_fp64_exact": f3(e1), "rel_err_vs_fp64_projected": f3(e2),
                        "method_rel_err": f3(e3)})
            del R_r
        return res

    def sec_precisions():
        res = []
        for prec, rr in [("bf16x3", r), ("f16x3", r), ("bf16", r), ("f16", r), ("bf16x3", 64), ("bf16", 64),
                         ("fp8", 8), ("fp8x2", 8), ("fp8", 1)]:
            ms_p, kms_p, R_p, cfg_p = timed(rr, prec, 10, 3, warm_s=0.1)
            e1, e2, _ = sampled_errors(rr, R_p)
            mfma_flops = 2.0 * M * W * rr * (K // L) * MFMA_PER_PRODUCT.get(prec, 1)
            res.append({"prec": prec, "r": rr, "ms_per_step": round(ms_p, 5), "gemm_ms": round(kms_p, 5),
                        "tile_cfg": cfg_p, "exact_equiv_tflops": round(exact_flops / (ms_p * 1e-3) / 1e12, 3),
                        "gemm_frac_of_peak": round(mfma_flops / (kms_p * 1e-3) / 1e12 / PEAK[prec], 4),
                        "rel_err_vs_fp64_exact": f3(e1), "rel_err_vs_fp64_projected": f3(e2)})
            del R_p
        return res

    def sec_static_database():
        # the database (8192 images) packed once at r = 64 (a projection-major
        # pack serves every r <= 64); each step projects the 1024 queries and
        # contracts -- the deployment where the database is static
        Bp64 = pg.pack_b(Bd, 64, basis, prec="f32", transB=True)
        torch.cuda.synchronize()
        out = []
        for rr in (1, 4, 8, 16, 64):
            cfg_s = autotune.tune_gemm(M, W, K, L, rr, "f32", reps=3, basis=basis)
            Ap = torch.empty(pg.packed_bytes(M, K, L, rr, "f32"), dtype=torch.uint8, device=dev)
            R_s = torch.empty((M, W), dtype=torch.float32, device=dev)

            def st():
                pg.pack_a(Ad, rr, basis, prec="f32", out=Ap)
                pg.gemm_packed(Ap, Bp64, rr, M, W, K, L, rr, 64, prec="f32", out=R_s, tile_cfg=cfg_s)
            t = timed_ms(st, args.steps, warmup=args.warmup)
            e_exact, e_proj, _ = sampled_errors(rr, R_s)
            out.append({"r": rr, "ms_per_step": round(t, 5), "tile_cfg": cfg_s,
                        "exact_equiv_tflops": round(exact_flops / (t * 1e-3) / 1e12, 3),
                        "rel_err_vs_fp64_exact": f3(e_exact), "rel_err_vs_fp64_projected": f3(e_proj)})
            del R_s, Ap
        del Bp64
        return out

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
        import oracle
        # the oracle's own eigenbasis of the same training blocks (moments in
        # FP64 on the host) for the projected reference
        Ck, Dk, _ = oracle.basis_klt(oracle.block_moments(Bt[:2048].astype(np.float64), L))
        res = {"train_images": 2048, "moments_ms": round((t1 - t0) * 1e3, 3),
               "eigen_host_ms": round((t2 - t1) * 1e3, 3), "points": []}
        import oracle
        for rr in (1, 2, 4, 8, 16):
            ms_k, kms_k, R_k, cfg_k = timed(rr, "f32", 10, 3, b=kb, Lb=L, warm_s=0.1)
            got = R_k[torch.from_numpy(srows).to(dev)][:, torch.from_numpy(scols).to(dev)].double().cpu().numpy()
            e_klt = oracle.rel_fro(got, exact_block)
            proj = oracle.gemm_proj_block(A, np.ascontiguousarray(Bt.T), Ck, Dk, rr, srows, scols)
            ms_d, _, R_d, _ = timed(rr, "f32", 10, 3, warm_s=0.1)
            e_dct, _, _ = sampled_errors(rr, R_d)
            res["points"].append({"r": rr, "klt_ms_per_step": round(ms_k, 5), "dct_ms_per_step": round(ms_d, 5),
                                  "rel_err_vs_fp64_exact_klt": f3(e_klt), "rel_err_vs_fp64_exact_dct": f3(e_dct),
                                  "rel_err_klt_vs_fp64_projected": f3(oracle.rel_fro(got, proj)),
                                  "tile_cfg": cfg_k})
            del R_k, R_d
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
        out = []
        for lab, b, rr in [("exact", pg.Basis("identity", 1), 1), ("dct2 L=8", pg.Basis("dct2", 8), 1),
                           ("dct2 L=12", pg.Basis("dct2", 12), 1), ("dct2 L=16", pg.Basis("dct2", 16), 1)]:
            model = PCA2D(b, rr, 10).fit(tr)
            rate = float(np.mean(ltr[model.match(te).cpu().numpy()] == lte))
            X = model.X
            t_g = timed_ms(lambda: pg.gemm(Ast, Ast, rr, b, transA=True), 20, warmup=3)
            t_s = timed_ms(lambda: pg.gemm(Ast, X, rr, b), 20, warmup=3)
            t_t = timed_ms(lambda: pg.gemm(Bst, X, rr, b), 20, warmup=3)
            out.append({"basis": lab, "r": rr, "recognition_rate": round(rate, 4), "scatter_ms": round(t_g, 4),
                        "train_features_ms": round(t_s, 4), "test_features_ms": round(t_t, 4),
                        "gemm_total_ms": round(t_g + t_s + t_t, 4)})
        ex = out[0]["gemm_total_ms"]
        for o in out:
            o["gemm_speedup_vs_exact"] = round(ex / o["gemm_total_ms"], 3)
        return {"images": [int(J), int(te.shape[0]), int(m), int(n)], "axes": 10, "points": out}

    def sec_plain():
        # plain (unprojected) FP32 GEMM through the same kernels: the identity
        # basis with all projections kept only permutes the contraction index
        plain = pg.Basis("identity", 4)
        ms_p, kms_p, R_p, cfg_p = timed(4, "f32", 10, 3, b=plain, Lb=4)
        import oracle
        got = R_p[torch.from_numpy(srows).to(dev)][:, torch.from_numpy(scols).to(dev)].double().cpu().numpy()
        return {"ms_per_step": round(ms_p, 5), "gemm_ms": round(kms_p, 5), "tile_cfg": cfg_p,
                "tflops": round(exact_flops / (ms_p * 1e-3) / 1e12, 3),
                "gemm_frac_of_fp32_peak": round(exact_flops / (kms_p * 1e-3) / 1e12 / PEAK["f32"], 4),
                "rel_err_vs_fp64_exact": f3(oracle.rel_fro(got, exact_block)),
                "speedup_of_headline_r": round(ms_p / ms, 3)}

    def sec_conv():
        import oracle
        Wc, Lc = 1 << 22, 256
        s = inputs.ar2_signal(Wc, seed=inputs.SEED_AR2)
        sd = torch.from_numpy(s.astype(np.float32)).to(dev)
        bc = pg.Basis("dct2", Lc)
        Cc, Dc = oracle.basis("dct2", Lc)
        ident = pg.Basis("identity", 32)
        res = {"full_rate": [], "block_rate": [], "paper_points": []}
        for N in (1024, 4096, 16384):
            k, o = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
            kd = torch.from_numpy(k.astype(np.float32)).to(dev)
            nout = Wc - N + 1
            y = torch.empty(nout, dtype=torch.float32, device=dev)
            ms_rng = np.random.default_rng(N)
            ms = np.unique(np.concatenate([[0, nout - 1, o], ms_rng.integers(0, nout, 61)]))
            exact = np.array([np.dot(k, s[m:m + N]) for m in ms])
            flops = 2.0 * nout * N
            runs = [(1, bc, "dct2", "full"), (16, bc, "dct2", "full"), (64, bc, "dct2", "full"),
                    (256, bc, "dct2", "full"), (32, ident, "plain", "full")]
            if N == 16384:
                runs += [(16, bc, "dct2", "block"), (64, bc, "dct2", "block"), (256, bc, "dct2", "block")]
            for rr, b, lab, rate in runs:
                ws = torch.empty(pg.conv1d_workspace_bytes(Wc, N, b.L, rr, rate=rate), dtype=torch.uint8, device=dev)
                fn = lambda: pg.conv1d(sd, kd, rr, b, out=y, workspace=ws, rate=rate)
                t = timed_ms(fn, 10, warmup=3)
                got = y[torch.from_numpy(ms).to(dev)].double().cpu().numpy()
                ent = {"N": N, "basis": lab, "L": b.L, "r": rr, "rate": rate, "ms": round(t, 5),
                       "exact_equiv_tflops": round(flops / (t * 1e-3) / 1e12, 3),
                       "rel_err_vs_fp64_exact": f3(oracle.rel_fro(got, exact))}
                if lab == "dct2":
                    if rate == "full":
                        proj = oracle.xcorr_proj_at(s, k, Cc, Dc, rr, ms)
                    else:
                        proj = oracle.xcorr_proj_block_rate_at(s, k, Cc, Dc, rr, ms)
                    ent["rel_err_vs_fp64_projected"] = f3(oracle.rel_fro(got, proj))
                res["full_rate" if rate == "full" else "block_rate"].append(ent)
                del ws
        # circular mode on the same signal (period 2^22), N = 16384
        res["circular"] = []
        k, _ = inputs.excerpt_kernel(s, 16384, seed=inputs.SEED_KERNEL)
        kd = torch.from_numpy(k.astype(np.float32)).to(dev)
        yc = torch.empty(Wc, dtype=torch.float32, device=dev)
        for rr in (16, 64, 256):
            ws = torch.empty(lib_ws := pg.lib().pj_conv1d_circular_workspace_bytes(Wc, 16384, Lc, rr, 1),
                             dtype=torch.uint8, device=dev)
            fn = lambda: pg.conv1d_circular(sd, kd, rr, bc, out=yc, workspace=ws)
            t = timed_ms(fn, 10, warmup=3)
            res["circular"].append({"N": 16384, "L": Lc, "r": rr, "ms": round(t, 5),
                                    "exact_equiv_tflops": round(2.0 * Wc * 16384 / (t * 1e-3) / 1e12, 3),
                                    "workspace_bytes": int(lib_ws)})
            del ws
        # the paper's CONV operating points: a block of 20000 samples, kernels
        # of 600 and 1200 samples, L = 2 Haar, one projection at half or full
        # sampling rate, and the exact result (both projections) for reference
        s20 = inputs.ar2_signal(20000, seed=inputs.SEED_AR2)
        s20d = torch.from_numpy(s20.astype(np.float32)).to(dev)
        h2 = pg.Basis("haar", 2)
        for N in (600, 1200):
            k20, _ = inputs.excerpt_kernel(s20, N, seed=inputs.SEED_KERNEL)
            k20d = torch.from_numpy(k20.astype(np.float32)).to(dev)
            exact = np.correlate(s20, k20, "valid")
            nout = exact.size
            y = torch.empty(nout, dtype=torch.float32, device=dev)
            for rr, rate, lab in [(1, "block", "1 projection, half samples"), (1, "full", "1 projection, all samples"),
                                  (2, "full", "all projections (exact)")]:
                ws = torch.empty(pg.conv1d_workspace_bytes(20000, N, 2, rr, rate=rate), dtype=torch.uint8,
                                 device=dev)
                fn = lambda: pg.conv1d(s20d, k20d, rr, h2, out=y, workspace=ws, rate=rate)
                t = timed_ms(fn, 50, warmup=5)
                got = y.double().cpu().numpy()
                res["paper_points"].append({"W": 20000, "N": N, "L": 2, "basis": "haar", "r": rr, "rate": rate,
                                            "label": lab, "ms": round(t, 5),
                                            "msamples_per_s": round(nout / (t * 1e-3) / 1e6, 2),
                                            "snr_db_vs_fp64_exact": round(oracle.snr_db(exact, got), 2)})
                del ws
        return res

    def sec_batched():
        import oracle
        shapes = inputs.batched_shapes()
        As, Bs = [], []
        for i, (m, w, k) in enumerate(shapes):
            As.append(torch.from_numpy(inputs.smoothed_rows(m, k, sigma=4.0, seed=6400 + i).astype(np.float32)).to(dev))
            Bs.append(torch.from_numpy(inputs.gaussian_matrix(k, w, seed=64000 + i).astype(np.float32)).to(dev))
        flops = sum(2.0 * m * w * k for m, w, k in shapes)
        Lb = 16
        bb = pg.Basis("dct2", Lb)
        Cb, Db = oracle.basis("dct2", Lb)
        res = []
        for prec, rr in [("bf16x3", 4), ("bf16", 4), ("bf16", 16), ("fp8", 8), ("f16x3", 16)]:
            cfg_b = autotune.tune_batched(As, Bs, rr, bb, prec=prec, reps=2, candidates=[0, 5, 6, 9])
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
                rows = np.sort(rng.choice(m, 8, replace=False))
                cols = np.sort(rng.choice(w, 8, replace=False))
                got = outs[i][torch.from_numpy(rows).to(dev)][:, torch.from_numpy(cols).to(dev)].double().cpu().numpy()
                A64 = As[i].double().cpu().numpy()
                B64 = Bs[i].double().cpu().numpy()
                proj = oracle.gemm_proj_block(A64, B64, Cb, Db, rr, rows, cols)
                errs.append((oracle.rel_fro(got, proj), oracle.rel_fro(got, A64[rows] @ B64[:, cols])))
            res.append({"prec": prec, "r": rr, "L": Lb, "problems": len(shapes), "tile_cfg": cfg_b,
                        "ms": round(t, 4), "exact_equiv_tflops": round(flops / (t * 1e-3) / 1e12, 3),
                        "reduced_tflops": round(flops * rr / Lb / (t * 1e-3) / 1e12, 3),
                        "rel_err_vs_fp64_projected_max": f3(max(e[0] for e in errs)),
                        "rel_err_vs_fp64_exact_max": f3(max(e[1] for e in errs))})
            del ws, outs
        return res

    def sec_mlp():
        from paper_1411_2860_amd.autograd import proj_matmul
        import oracle
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
        res = []
        plain_flops = 2.0 * Bsz * Din * Dh * 2 + 2.0 * Bsz * Dh * Dout * 3    # fwd + dW1 + fwd + dH + dW2
        for r1, r2 in [(16, 64), (64, 64), (8, 16)]:
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
            res.append({"r1": r1, "r2": r2, "prec": "bf16", "ms_fwd_bwd": round(t, 4),
                        "exact_equiv_tflops": round(plain_flops / (t * 1e-3) / 1e12, 3),
                        "loss": round(loss, 6), "loss_rel_err_vs_fp64": f3(abs(loss - loss_ref) / loss_ref)})
        return res

    section("sweep", sec_sweep)
    section("precisions", sec_precisions)
    section("plain", sec_plain)
    section("static_database", sec_static_database)
    section("klt", sec_klt)
    section("pca2d", sec_pca2d)
    section("conv", sec_conv)
    section("batched", sec_batched)
    section("mlp", sec_mlp)

    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(A, Bt, r)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
