"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/hmsv.h declares, and
reject bad arguments on the host before touching the device.  Its own
quantizer and length-model constants are compared with the oracle's
(independent implementations of the same definitions)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle import quant as oq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmsv.h")

hm = pytest.importorskip("paper_1707_09683_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hmsv_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(hm.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(hm.EXPORTED) == set(names)


def test_constants_match_oracle():
    for M in (1, 2, 3, 48, 100, 400, 1000, 2400, 3839):
        assert hm.tbm(M) == oq.tbm(M)
    for L in (0, 1, 2, 3, 20, 21, 45, 350, 1000, 35000, 10 ** 6):
        assert hm.tjb(L) == oq.tjb(L)
    assert hm.tbm(0) == -1 and hm.tjb(-1) == -1


def test_quantizer_matches_oracle_bit_for_bit():
    rng = np.random.default_rng(31)
    for M in (1, 7, 48, 400, 1000, 2400, 3839):
        e = synth.sample_emissions(rng, M)
        a = hm.quantize(e, synth.BG)
        b = oq.quantize(e, synth.BG)
        assert a["dbias"] == b["bias"]
        assert (a["cost"] == b["cost"]).all() and (a["sc"] == b["sc"]).all()


def test_quantizer_rejects_bad_input():
    e = np.full((4, 20), 0.05)
    with pytest.raises(hm.HmsvError):
        hm.quantize(e, np.zeros(20))
    bad = e.copy()
    bad[0, 0] = np.nan
    with pytest.raises(hm.HmsvError):
        hm.quantize(bad, synth.BG)
    bad[0, 0] = -0.1
    with pytest.raises(hm.HmsvError):
        hm.quantize(bad, synth.BG)
    with pytest.raises(hm.HmsvError):
        hm.quantize(np.full((3840, 20), 0.05), synth.BG)


def test_db_create_validates_on_host():
    P = ctypes.c_void_p
    h = P()
    res = np.array([1, 2, 32], np.uint8)          # code 32 is out of range
    off = np.array([0, 3], np.int64)
    rc = hm._lib.hmsv_db_create(hm._np_ptr(res), hm._np_ptr(off), 1, ctypes.byref(h))
    assert rc == -1 and not h.value
    off = np.array([0, 2, 1], np.int64)           # decreasing offsets
    res = np.array([1, 2, 3], np.uint8)
    assert hm._lib.hmsv_db_create(hm._np_ptr(res), hm._np_ptr(off), 2, ctypes.byref(h)) == -1
    assert hm._lib.hmsv_db_create(hm._np_ptr(res), None, 2, ctypes.byref(h)) == -1
    assert hm._lib.hmsv_db_create(hm._np_ptr(res), hm._np_ptr(off), 2, None) == -1
    # a sequence longer than 2^24 - 4 residues does not fit a record's row field
    big = np.zeros((1 << 24) - 3, np.uint8)
    off = np.array([0, 0, big.size], np.int64)
    assert hm._lib.hmsv_db_create(hm._np_ptr(big), hm._np_ptr(off), 2, ctypes.byref(h)) == -2
    assert not h.value


def test_score_rejects_bad_arguments_before_launch():
    prof = hm._CProfile(0, 10, 1, 1)              # M = 0
    ws = ctypes.c_void_p(1)
    rc = hm._lib.hmsv_msv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws, None, None)
    assert rc == -1
    prof = hm._CProfile(10, 65, 1, 1)             # dbias above the bound
    assert hm._lib.hmsv_msv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws, None,
                                  None) == -1
    prof = hm._CProfile(4000, 10, 1, 1)           # longer than HMSV_MAX_M
    assert hm._lib.hmsv_ssv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws, None,
                                  None) == -2
    prof = hm._CProfile(10, 10, 1, None)          # SSV table missing
    assert hm._lib.hmsv_ssv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws, None,
                                  None) == -1
    prof = hm._CProfile(100, 10, 1, 1)
    bad_plan = hm.make_plan(8, 2)                 # covers 31 < 100 nodes
    assert hm._lib.hmsv_msv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws,
                                  ctypes.byref(bad_plan), None) == -1
    odd_plan = hm.make_plan(6, 9)                 # G not a power of two
    assert hm._lib.hmsv_msv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws,
                                  ctypes.byref(odd_plan), None) == -1
    many_waves = hm.make_plan(8, 7, waves_per_block=9)
    assert hm._lib.hmsv_msv_score(ctypes.byref(prof), ctypes.c_void_p(1), 1, 1, ws,
                                  ctypes.byref(many_waves), None) == -1
    assert hm._lib.hmsv_msv_score(ctypes.byref(prof), None, 1, 1, ws, None, None) == -1


def test_default_plans_cover_every_length():
    for filt in ("msv", "ssv"):
        for M in list(range(1, 200)) + list(range(200, 3840, 37)) + [3839]:
            p = hm.default_plan(filt, M)
            assert 2 * p.G * p.Q - 1 >= M and 64 % p.G == 0
    with pytest.raises(hm.HmsvError):
        hm.default_plan("msv", 3840)


def test_default_plan_is_the_tuned_plan():
    """The C library's default plan equals the autotuner's table
    (tuned_plans.json, MI355X entry) looked up the documented way, at every
    tuned M-bin and at lengths between and beyond them."""
    from paper_1707_09683_amd import autotune
    table = autotune.load_table()
    key = autotune.DEVICE_KEY
    assert key in table
    for filt in ("msv", "ssv"):
        bins = sorted(int(b) for b in table[key][filt])
        Ms = set(bins) | {1, 2, 17, 29, 35, 44, 55, 70, 300, 450, 1100, 2222, 3500, 3839}
        Ms |= {int(round((a * b) ** 0.5)) for a, b in zip(bins[:-1], bins[1:])}
        for M in sorted(Ms):
            exp = autotune.lookup(table, key, filt, M)
            got = hm.default_plan(filt, M).as_tuple()
            assert exp is not None and got == tuple(exp), (filt, M, got, exp)
            assert hm.plan_for(filt, M).as_tuple() == got
    # the compiled-in table is the one generated from the JSON
    assert open(autotune.HEADER).read() == autotune.emit_header(table)


def test_plan_lds_bytes():
    """LDS footprint: 21 table rows of the lane groups' chunk regions; every
    default plan fits one CU's 160 KiB; invalid shapes give 0."""
    assert hm.plan_lds_bytes(8, 26) == 21 * 7 * 64 * 4       # 6 full chunks + a partial one
    assert hm.plan_lds_bytes(64, 30) == 21 * 30 * 64 * 4     # one dword per lane and register
    assert hm.plan_lds_bytes(32, 7) == 21 * (3 * 64 + 64) * 4  # 3 two-dword chunks + 1-dword tail
    for G, Q in ((0, 4), (3, 4), (128, 1), (8, 0)):
        assert hm.plan_lds_bytes(G, Q) == 0
    for filt in ("msv", "ssv"):
        for M in (1, 48, 63, 64, 127, 128, 400, 1000, 2400, 3839):
            p = hm.default_plan(filt, M)
            assert 0 < hm.plan_lds_bytes(p.G, p.Q) <= 160 * 1024


def test_score_nats():
    """Raw scores in nats: third-bits (3 / ln 2 per nat) minus the length
    and entry costs, 3 nats for the length loops, +inf on overflow.  Values
    worked by hand with tjb(21) = 9, tjb(0) = 0 and tbm(48) = 31."""
    ln2 = math.log(2.0)
    got = hm.score_nats("msv", 48, np.array([199, 202, 255], np.uint8),
                        np.array([0, 0, 1], np.uint8), np.array([21, 21, 21]))
    assert got[0] == pytest.approx(-3.0, abs=1e-12)
    assert got[1] == pytest.approx(ln2 - 3.0, abs=1e-12)
    assert math.isinf(got[2]) and got[2] > 0
    got = hm.score_nats("ssv", 48, np.array([100, -128], np.int8), np.array([0, 0], np.uint8),
                        np.array([21, 0]))
    assert got[0] == pytest.approx(176 * ln2 / 3 - 3.0, abs=1e-12)     # 100+128-31-18-3
    assert got[1] == pytest.approx(-34 * ln2 / 3 - 3.0, abs=1e-12)     # -128+128-31-0-3
    with pytest.raises(hm.HmsvError):
        hm.score_nats("msv", 48, np.array([1], np.uint8), np.array([0], np.uint8),
                      np.array([-1]))


def test_gumbel_pvalue():
    """Gumbel survival 1 - exp(-exp(-lambda (x - mu))): 1 - 1/e at the
    location, the exponential tail exp(-lambda (x - mu)) far above it
    (computed without cancellation), 0 for +inf, and monotone."""
    mu, lam = 2.5, 0.7
    x = np.array([mu, mu + 60.0, mu - 3.0, np.inf, mu + 1.0])
    p = hm.gumbel_pvalue(x, mu, lam)
    assert p[0] == pytest.approx(1.0 - math.exp(-1.0), rel=1e-14)
    assert p[1] == pytest.approx(math.exp(-lam * 60.0), rel=1e-9)
    assert p[2] == pytest.approx(1.0 - math.exp(-math.exp(lam * 3.0)), rel=1e-14)
    assert p[3] == 0.0
    assert p[1] < p[4] < p[0] < p[2]
    with pytest.raises(hm.HmsvError):
        hm.gumbel_pvalue(x, mu, 0.0)
