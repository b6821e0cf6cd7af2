"""Work counts (Sec. III-C, eq. (16)-(20)), the SNR of eq. (9) and the
dimension examples the paper prints, checked against tests/golden/."""
import json
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_gemm_work_ratio_single_projection():
    g = _golden()["gemm_work_ratio"]
    N, L, l = g["N"], g["L"], g["l"]
    ratio = oracle.work_gemm_proj(N, l, L) / oracle.work_gemm_plain(N)
    # eq. (17) at l = 0: N^2 (N / L + 2) over N^3 = 1/L + 2/N
    assert abs(ratio - (1.0 / L + 2.0 / N)) < 1e-15
    assert round(100 * ratio, 1) == g["percent_rounded"]


def test_gemm_work_full_projections_exceeds_plain():
    # with all L projections the projection overhead makes the count exceed N^3
    assert oracle.work_gemm_proj(144, 7, 8) > oracle.work_gemm_plain(144)


def test_memory_saving_and_conv_examples():
    g = _golden()
    for row in g["memory_saving"]:
        assert abs(100 * (1 - (row["l"] + 1) / row["L"]) - row["percent"]) < 1e-12
    c = g["conv_half_length"]
    assert c["W"] // c["L"] == c["W_projected"] and c["N"] // c["L"] == c["N_projected"]
    # eq. (20) vs eq. (18): the reduced CONV term is 1/L^2 of the plain one
    N, L = c["N"], c["L"]
    assert 2 * (N // L) ** 2 * L * L == oracle.work_conv_plain_time(N)
    assert oracle.work_conv_proj_time(N, 0, L) == (4 * N + 1) + 2 * (N // L) ** 2


def test_snr_definition():
    ref = np.array([1.0, 1.0])
    approx = np.array([1.0, 0.9])
    assert abs(oracle.snr_db(ref, approx) - 10 * math.log10(2.0 / 0.01)) < 1e-12
    assert oracle.snr_db(ref, ref) == math.inf
    assert abs(oracle.rel_fro(approx, ref) - 0.1 / math.sqrt(2.0)) < 1e-15


def test_conv_time_counts_match_hand_worked_values():
    # eq. (18) and (20) against values worked by hand from the printed
    # formulas (a dropped term, a missing ceil or a wrong factor fails)
    for c in _golden()["conv_work_counts"]["cases"]:
        assert oracle.work_conv_plain_time(c["N"]) == c["plain_time"]
        assert oracle.work_conv_proj_time(c["N"], c["l"], c["L"]) == c["proj_time"]


def test_conv_freq_counts_match_hand_worked_values():
    # eq. (19) and (21) at N = 341 (3N + 1 = 1024, an exact power of two)
    g = _golden()["conv_work_counts_freq"]
    assert oracle.work_conv_plain_freq(g["N"]) == g["plain_freq"]
    want = (g["proj_freq_projection"] + g["proj_freq_fft_coef"] * math.log2(g["proj_freq_log2_arg"])
            + g["proj_freq_tail"])
    assert abs(oracle.work_conv_proj_freq(g["N"], g["l"], g["L"]) - want) < 1e-9 * want
    # the frequency-domain model favours projections more as N grows
    r1 = oracle.work_conv_proj_freq(1 << 14, 0, 256) / oracle.work_conv_plain_freq(1 << 14)
    r2 = oracle.work_conv_proj_freq(1 << 20, 0, 256) / oracle.work_conv_plain_freq(1 << 20)
    assert r2 < r1 < 1.0
