"""Autotuner for the workgroup tile of the reduced contraction.

The library offers several tile configurations (``pj_gemm_tile_configs``).
The best one depends on the problem shape, the contraction length r * G and
the operand format; this module times every configuration on the device for a
given problem (or batch), keeps the fastest, and caches the choice in a JSON
file keyed by the operand format, L, r and power-of-two buckets of M, W and
K.  The cache lives at $PROJGEMM_TUNE_CACHE (default
~/.cache/projgemm/tune.json).

The timings run the library's own kernels on synthetic operands of the
requested shape; nothing else is executed.
"""
from __future__ import annotations

import json
import math
import os
import threading

__all__ = ["cache_path", "shape_key", "batch_key", "lookup", "record", "tune_gemm", "tune_batched",
           "tune_batched_tiles", "clear_memory_cache"]

_lock = threading.Lock()
_mem: dict | None = None


def cache_path() -> str:
    return os.environ.get("PROJGEMM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "projgemm", "tune.json"))


def _bucket(n: int) -> int:
    """Smallest power of two >= n (shapes within a factor of two share a choice)."""
    return 1 << max(0, math.ceil(math.log2(max(1, int(n)))))


def shape_key(M: int, W: int, K: int, L: int, r: int, prec: str) -> str:
    return f"gemm/{prec}/L{L}/r{r}/M{_bucket(M)}/W{_bucket(W)}/K{_bucket(K)}"


def batch_key(shapes, L: int, r: int, prec: str) -> str:
    """Key of a batch: its size and the buckets of its total and largest work."""
    flops = sum(2.0 * m * w * k for m, w, k in shapes)
    big = max(m * w for m, w, _ in shapes)
    return f"batched/{prec}/L{L}/r{r}/n{_bucket(len(shapes))}/F{_bucket(int(flops // 1e6))}/B{_bucket(big)}"


def _load() -> dict:
    global _mem
    if _mem is None:
        try:
            with open(cache_path()) as f:
                _mem = json.load(f)
        except (OSError, ValueError):
            _mem = {}
    return _mem


def clear_memory_cache():
    global _mem
    with _lock:
        _mem = None


def lookup(key: str):
    """The cached tile configuration index for `key`, or None."""
    with _lock:
        v = _load().get(key)
    return None if v is None else int(v["cfg"])


def record(key: str, cfg: int, timings_ms: dict):
    """Stores a choice (and the timings it was based on) and writes the cache."""
    with _lock:
        d = _load()
        d[key] = {"cfg": int(cfg), "ms": {str(k): round(float(v), 5) for k, v in timings_ms.items()}}
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def _time_ms(fn, reps: int, warmup: int = 2) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_gemm(M: int, W: int, K: int, L: int, r: int, prec: str = "f32", reps: int = 5, force: bool = False,
              basis=None) -> int:
    """Times every tile configuration of the reduced contraction for this
    shape on synthetic packed operands and returns (and caches) the fastest."""
    key = shape_key(M, W, K, L, r, prec)
    if not force:
        c = lookup(key)
        if c is not None:
            return c
    import torch
    from . import projgemm as pg
    basis = basis or pg.Basis("dct2", L)
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(1234)
    A = torch.randn((M, K), device="cuda", dtype=dt, generator=g)
    B = torch.randn((K, W), device="cuda", dtype=dt, generator=g)
    Ap, Bp = pg.pack_ab(A, B, r, basis, prec=prec)
    R = torch.empty((M, W), device="cuda", dtype=dt)
    times = {}
    for i, _ in enumerate(pg.tile_configs(prec)):
        times[i] = _time_ms(lambda: pg.gemm_packed(Ap, Bp, r, M, W, K, L, r, r, prec=prec, out=R, tile_cfg=i), reps)
    best = pick(times)
    record(key, best, times)
    return best


def pick(times: dict, tie: float = 0.03) -> int:
    """The highest-numbered configuration (the table ends with the largest
    tiles) within `tie` (relative) of the fastest: configurations that time
    alike are chosen the same way on every run, whatever the timing noise."""
    t_min = min(times.values())
    return max(i for i, t in times.items() if t <= t_min * (1.0 + tie))


def tune_batched(As, Bs, r: int, basis, prec: str = "bf16", transA=False, transB=False, reps: int = 3,
                 force: bool = False, candidates=None) -> int:
    """Times the persistent batched launch with every tile configuration (or
    `candidates`) on the given operands and returns (and caches) the fastest."""
    shapes = []
    for A, B in zip(As, Bs):
        M, K = (A.shape[1], A.shape[0]) if transA else tuple(A.shape)
        W = B.shape[0] if transB else B.shape[1]
        shapes.append((M, W, K))
    key = batch_key(shapes, basis.L, r, prec)
    if not force:
        c = lookup(key)
        if c is not None:
            return c
    from . import projgemm as pg
    outs = pg.gemm_batched(As, Bs, r, basis, prec=prec, transA=transA, transB=transB, tile_cfg=0)
    cands = list(candidates) if candidates is not None else list(range(len(pg.tile_configs(prec))))
    times = {}
    for i in cands:
        need = pg.gemm_batched_workspace_bytes(pg._descs(As, Bs, outs, transA, transB), basis.L, r, prec, i)
        ws = pg._byte_buffer(need, As[0].device)
        times[i] = _time_ms(lambda: pg.gemm_batched(As, Bs, r, basis, prec=prec, transA=transA, transB=transB,
                                                    outs=outs, tile_cfg=i, workspace=ws), reps, warmup=1)
        del ws
    best = pick(times)
    record(key, best, times)
    return best


def tune_batched_tiles(As, Bs, r: int, basis, prec: str = "bf16", tile_cfg: int = 0, transA=False, transB=False,
                       reps: int = 3, force: bool = False):
    """Per-problem tile of a batch for the persistent launch of `tile_cfg`:
    times each problem alone with the configuration's tile and with its small
    tile and keeps the faster (one flag per problem, True = small), cached
    per batch."""
    from . import projgemm as pg
    shapes = []
    for A, B in zip(As, Bs):
        M, K = (A.shape[1], A.shape[0]) if transA else tuple(A.shape)
        W = B.shape[0] if transB else B.shape[1]
        shapes.append((M, W, K))
    key = batch_key(shapes, basis.L, r, prec) + f"/tiles/c{int(tile_cfg)}"
    if not force:
        with _lock:
            v = _load().get(key)
        if v is not None and len(v.get("small", [])) == len(shapes):
            return [bool(f) for f in v["small"]]
    flags, ms = [], []
    for A, B in zip(As, Bs):
        outs = pg.gemm_batched([A], [B], r, basis, prec=prec, transA=transA, transB=transB, tile_cfg=tile_cfg,
                               small=[False])
        t = []
        for f in (False, True):
            need = pg.gemm_batched_workspace_bytes(pg._descs([A], [B], outs, transA, transB), basis.L, r, prec,
                                                   tile_cfg, [f])
            ws = pg._byte_buffer(need, A.device)
            t.append(_time_ms(lambda: pg.gemm_batched([A], [B], r, basis, prec=prec, transA=transA, transB=transB,
                                                      outs=outs, tile_cfg=tile_cfg, workspace=ws, small=[f]),
                              reps, warmup=1))
            del ws
        flags.append(t[1] < t[0] * 0.97)
        ms.append([round(t[0], 5), round(t[1], 5)])
    with _lock:
        d = _load()
        d[key] = {"small": [int(f) for f in flags], "ms": ms}
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return flags
