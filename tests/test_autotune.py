"""Autotuner cache logic (CPU) and a tuning run on the device (GPU)."""
import json

import numpy as np
import pytest

from paper_1411_2860_amd import autotune


@pytest.fixture()
def tmp_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("PROJGEMM_TUNE_CACHE", str(tmp_path / "tune.json"))
    autotune.clear_memory_cache()
    yield tmp_path / "tune.json"
    autotune.clear_memory_cache()


def test_keys_bucket_shapes():
    assert autotune.shape_key(1000, 8192, 4096, 64, 16, "f32") == autotune.shape_key(600, 5000, 3000, 64, 16, "f32")
    assert autotune.shape_key(1000, 8192, 4096, 64, 16, "f32") != autotune.shape_key(1000, 8192, 4096, 64, 8, "f32")
    assert autotune.shape_key(1, 1, 1, 1, 1, "bf16").endswith("M1/W1/K1")
    k1 = autotune.batch_key([(128, 128, 128)] * 3, 16, 4, "bf16")
    assert k1.startswith("batched/bf16/L16/r4/n4/")


def test_record_lookup_persist(tmp_cache):
    key = autotune.shape_key(64, 64, 64, 8, 2, "f32")
    assert autotune.lookup(key) is None
    autotune.record(key, 3, {0: 1.0, 3: 0.5})
    assert autotune.lookup(key) == 3
    autotune.clear_memory_cache()
    assert autotune.lookup(key) == 3
    d = json.loads(tmp_cache.read_text())
    assert d[key]["cfg"] == 3 and d[key]["ms"]["3"] == 0.5


def test_pick_breaks_ties_by_index():
    assert autotune.pick({0: 2.0, 9: 0.99, 10: 1.01}) == 10         # within 3 %: highest index
    assert autotune.pick({0: 2.0, 9: 1.00, 10: 1.05}) == 9          # a clear winner
    assert autotune.pick({3: 1.0}) == 3


@pytest.mark.gpu
def test_tune_gemm_and_batched_on_device(tmp_cache):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2860_amd import projgemm as pg
    cfg = autotune.tune_gemm(512, 1024, 1024, 64, 8, "bf16x3", reps=2)
    assert 0 <= cfg < len(pg.tile_configs("bf16x3"))
    assert autotune.tune_gemm(512, 1024, 1024, 64, 8, "bf16x3") == cfg     # cached
    basis = pg.Basis("dct2", 16)
    rng = np.random.default_rng(0)
    As = [torch.from_numpy(rng.standard_normal((m, k))).float().cuda() for m, k in [(100, 64), (300, 200)]]
    Bs = [torch.from_numpy(rng.standard_normal((k, w))).float().cuda() for k, w in [(64, 50), (200, 400)]]
    c2 = autotune.tune_batched(As, Bs, 4, basis, prec="bf16", reps=1, candidates=[0, 4, 6])
    assert c2 in (0, 4, 6)
    flags = autotune.tune_batched_tiles(As, Bs, 4, basis, prec="bf16", tile_cfg=6, reps=1)
    assert len(flags) == 2 and all(isinstance(f, bool) for f in flags)
    assert autotune.tune_batched_tiles(As, Bs, 4, basis, prec="bf16", tile_cfg=6) == flags     # cached
