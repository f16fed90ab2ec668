"""Host-side checks of the P7Viterbi entry points of the C-ABI library (no
GPU needed): its quantizer and length model against the oracle's
(independent float64 implementations of the same definitions), argument
checks before any launch, and the default plans."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import p7 as op7

hm = pytest.importorskip("paper_1707_09683_amd")


def test_p7_quantizer_matches_oracle_bit_for_bit():
    rng = np.random.default_rng(41)
    for M in (1, 2, 7, 48, 400, 1000, 2815):
        e = synth.sample_emissions(rng, M)
        t = synth.sample_transitions(rng, M)
        if M > 2:
            # zero probabilities quantize to -inf on both sides
            e[1, 3] = 0.0
            t[0, 2] = 0.0
            t[M // 2, 4] = 0.0
        a = hm.p7_quantize(e, t, synth.BG)
        b = op7.quantize(e, t, synth.BG)
        assert a["tbm"] == b["tbm"], M
        assert (a["msc"] == b["msc"]).all(), M
        assert (a["trans"] == b["trans"]).all(), M


def test_p7_length_model_matches_oracle():
    for L in (0, 1, 2, 3, 4, 10, 16, 17, 100, 350, 1000, 4096, 35000, 10 ** 6, (1 << 24) - 5):
        lm = op7.length_model(L)
        assert hm.p7_length_model(L) == (lm["NN"], lm["NB"]), L
        assert lm["NN"] == lm["JJ"] == lm["CC"] and lm["NB"] == lm["JB"] == lm["CT"]
    with pytest.raises(hm.HmsvError):
        hm.p7_length_model(-1)


def test_p7_quantizer_rejects_bad_input():
    e = np.full((4, 20), 0.05)
    t = np.full((4, 7), 0.3)
    with pytest.raises(hm.HmsvError):
        hm.p7_quantize(e, t, np.zeros(20))
    bad = t.copy()
    bad[1, 1] = np.nan
    with pytest.raises(hm.HmsvError):
        hm.p7_quantize(e, bad, synth.BG)
    bad[1, 1] = -0.5
    with pytest.raises(hm.HmsvError):
        hm.p7_quantize(e, bad, synth.BG)
    with pytest.raises(hm.HmsvError):
        hm.p7_quantize(np.full((2816, 20), 0.05), np.full((2816, 7), 0.3), synth.BG)


def test_p7_score_rejects_bad_arguments_before_launch():
    one = ctypes.c_void_p(1)
    ws = ctypes.c_void_p(256)
    prof = hm._CP7Profile(0, -100, 1, 1)                 # M = 0
    assert hm._lib.hmsv_p7_score(ctypes.byref(prof), one, 1, 1, ws, None, None) == -1
    prof = hm._CP7Profile(2816, -100, 1, 1)              # beyond HMSV_P7_MAX_M
    assert hm._lib.hmsv_p7_score(ctypes.byref(prof), one, 1, 1, ws, None, None) == -2
    prof = hm._CP7Profile(100, -100, 1, None)            # transitions missing
    assert hm._lib.hmsv_p7_score(ctypes.byref(prof), one, 1, 1, ws, None, None) == -1
    prof = hm._CP7Profile(100, -100, 1, 1)
    assert hm._lib.hmsv_p7_score(ctypes.byref(prof), None, 1, 1, ws, None, None) == -1
    assert hm._lib.hmsv_p7_score(ctypes.byref(prof), one, 1, 1, ctypes.c_void_p(8), None,
                                 None) == -1                     # workspace not 256-aligned
    for plan in (hm.make_plan(8, 6),                   # 95 < 100 nodes
                 hm.make_plan(6, 9),                   # G not a power of two
                 hm.make_plan(8, 7, waves_per_block=9),
                 hm.make_plan(32, 2, waves_per_block=9),
                 hm.make_plan(64, 19, waves_per_block=9),   # spills as 1024 threads
                 hm.make_plan(64, 16, waves_per_block=17)):
        assert hm._lib.hmsv_p7_score(ctypes.byref(prof), one, 1, 1, ws, ctypes.byref(plan),
                                     None) == -1, plan.as_tuple()
    unbuilt = hm.make_plan(4, 17)                      # Q beyond the G = 4 kernels
    assert hm._lib.hmsv_p7_score(ctypes.byref(prof), one, 1, 1, ws, ctypes.byref(unbuilt),
                                 None) == -5



def test_pipeline_calls_reject_bad_arguments_before_launch():
    """hmsv_select and hmsv_p7_score_selected refuse null pointers, a bad
    filter switch and a misaligned workspace without touching the device
    (null scores and flags are refused only for a non-empty database, which
    needs a device to build: the GPU tests cover the empty one)."""
    one = ctypes.c_void_p(1)
    ws = ctypes.c_void_p(256)
    sel = hm._lib.hmsv_select
    assert sel(None, one, one, 1, 0, one, one, ws, None) == -1
    assert sel(one, one, one, 1, 0, None, one, ws, None) == -1
    assert sel(one, one, one, 1, 0, one, None, ws, None) == -1
    assert sel(one, one, one, 1, 0, one, one, None, None) == -1
    assert sel(one, one, one, 2, 0, one, one, ws, None) == -1          # is_msv not 0/1
    assert sel(one, one, one, 0, 0, one, one, ctypes.c_void_p(8), None) == -1
    prof = hm._CP7Profile(100, -100, 1, 1)
    p7s = hm._lib.hmsv_p7_score_selected
    assert p7s(ctypes.byref(prof), one, None, one, 1, 1, ws, None, None) == -1
    assert p7s(ctypes.byref(prof), one, one, None, 1, 1, ws, None, None) == -1
    assert p7s(ctypes.byref(prof), None, one, one, 1, 1, ws, None, None) == -1
    prof = hm._CP7Profile(2816, -100, 1, 1)
    assert p7s(ctypes.byref(prof), one, one, one, 1, 1, ws, None, None) == -2


TUNED = {30: (8, 4), 64: (8, 4), 100: (8, 8), 200: (8, 4), 400: (16, 4), 700: (32, 8),
         1000: (32, 8), 1100: (64, 16), 1500: (64, 16), 2047: (64, 16), 2200: (64, 16),
         2400: (64, 16), 2815: (64, 8)}


def max_waves(G, Q):
    return 16 if G == 64 and (Q <= 18 or Q == 20) else 8


def test_p7_default_plans_cover_every_length():
    import math
    for M in list(range(1, 300)) + list(range(300, 2816, 29)) + [2815]:
        p = hm.p7_default_plan(M)
        assert 2 * p.G * p.Q - 1 >= M and 64 % p.G == 0, M
        qmin = -(-(M + 1) // (2 * p.G))
        # the fewest registers (64 x 19 runs as 64 x 20 in 16-wavefront blocks)
        assert p.Q == qmin or (p.G, qmin, p.Q, p.waves_per_block) == (64, 19, 20, 16), M
        assert p.Q <= (22 if p.G == 64 else 16)
        assert 1 <= p.waves_per_block <= max_waves(p.G, p.Q)
        assert 0 < hm.p7_lds_bytes(p.G, p.Q) <= 160 * 1024
        # the nearest measured bin's plan where its group holds the profile
        b = min(TUNED, key=lambda v: (abs(math.log(v) - math.log(M)), v))
        G, wpb = TUNED[b]
        if -(-(M + 1) // (2 * G)) <= (22 if G == 64 else 16):
            assert (p.G, p.waves_per_block) == (G, min(wpb, max_waves(p.G, p.Q))), (M, b)
    with pytest.raises(hm.HmsvError):
        hm.p7_default_plan(2816)


def test_p7_lds_bytes():
    """28 table rows (21 emission rows, 7 transition rows) in the MSV image's
    chunk layout; invalid shapes give 0."""
    assert hm.p7_lds_bytes(64, 22) == 28 * 22 * 64 * 4
    assert hm.p7_lds_bytes(8, 16) == 28 * 16 * 16 * 4
    assert hm.p7_lds_bytes(64, 23) > 160 * 1024
    for G, Q in ((0, 4), (3, 4), (128, 1), (8, 0)):
        assert hm.p7_lds_bytes(G, Q) == 0
