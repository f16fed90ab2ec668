"""Pins of the CPU oracle against things other than itself.

Each check below would fail on a plausible slip in the oracle: a dropped or
mis-signed transition cost, a rotate instead of a shift at node 1, a reset of
scB/scJ in the wrong place, a missing saturation, a banker's rounding, an
off-by-one in the length model.  None of them re-types the oracle's recurrence:
they use closed forms, an unbounded-integer dynamic programme, enumeration of
all segment paths, the maximum over all diagonal segments, and hand-derived
values (tests/golden/).
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import quant as q
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NEG = q.NEG_INF


# ---------------------------------------------------------------- constants

def test_rhaz_rounds_half_away_from_zero():
    assert list(q.rhaz([0.5, -0.5, 1.5, 2.5, -2.5, 0.49999999999999994, 7.0])) == \
        [1, -1, 2, 3, -3, 0, 7]


def test_closed_form_constants():
    # Exact powers of two: 3*log2 is an integer.
    assert q.tec() == 3
    assert q.tjb(3) == 3 and q.tjb(21) == 9 and q.tjb(45) == 12 and q.tjb(0) == 0
    assert q.tbm(1) == 0
    # Hand-evaluated: 3*log2(6) = 7.75, 3*log2(48*49/2) = 30.6, 3*log2(400*401/2) = 48.9,
    # 3*log2(2400*2401/2) = 64.4
    assert q.tbm(3) == 8 and q.tbm(48) == 31 and q.tbm(400) == 49 and q.tbm(2400) == 64
    # 3*log2(23/3) = 8.82, 3*log2(353/3) = 20.6, 3*log2(35003/3) = 40.6
    assert q.tjb(20) == 9 and q.tjb(350) == 21 and q.tjb(35000) == 41
    # vectorised form agrees with the scalar one
    Ls = np.array([0, 1, 3, 20, 21, 350, 35000])
    assert list(q.tjb(Ls)) == [q.tjb(int(x)) for x in Ls]


def _read_pow2():
    nodes = []
    for line in open(os.path.join(GOLD, "quant_pow2.txt")):
        if line.startswith("#") or not line.strip():
            continue
        toks = line.split()[1:]
        nodes.append(toks)
    return nodes


def test_quantizer_powers_of_two_fixture():
    nodes = _read_pow2()
    bg = np.full(20, 1.0 / 20)
    emis = np.zeros((len(nodes), 20))
    for k, toks in enumerate(nodes):
        for x, t in enumerate(toks):
            emis[k, x] = 0.0 if t == "z" else bg[x] * 2.0 ** int(t)
    assert np.allclose(emis.sum(1), 1.0)
    p = q.quantize(emis, bg)
    assert p["bias"] == 12 and p["M"] == 3
    cost, sc = p["cost"].astype(int), p["sc"].astype(int)
    assert list(cost[:4, 0]) == [3, 6, 9, 9] and set(cost[4:20, 0]) == {18}
    assert set(cost[:20, 1]) == {12}
    assert cost[0, 2] == 0 and cost[11, 2] == 6
    assert set(np.delete(cost[:20, 2], [0, 11])) == {255}
    assert set(np.delete(sc[:20, 2], [0, 11])) == {-128}
    # degenerate codes 21..26 (B, J, Z, U, O, X): the mean of the members'
    # exponents (uniform bg), times 3, rounded half away from zero
    assert list(cost[21:27, 0]) == [14, 18, 14, 6, 18, 16]
    assert (cost[21:27, 1] == 12).all() and (cost[21:27, 2] == 255).all()
    for c in (20, 27, 28, 29, 30, 31):
        assert (cost[c] == 255).all() and (sc[c] == -128).all()
    assert (sc[:20, :2] == 12 - cost[:20, :2]).all()


def test_quantizer_properties_random_profiles():
    rng = np.random.default_rng(7)
    for M in (1, 5, 48, 400):
        e = synth.sample_emissions(rng, M)
        p = q.quantize(e, synth.BG)
        cost, sc = p["cost"].astype(int), p["sc"].astype(int)
        # bias is the largest log-odds; the best residue of some node costs 0
        assert cost[:20].min() == 0 and 0 <= p["bias"] <= 64
        # recomputation with math.log2 per entry (independent of numpy's log2)
        for k in range(min(M, 6)):
            for x in range(20):
                ratio = e[k, x] / synth.BG[x]
                if ratio == 0:
                    assert cost[x, k] == 255
                    continue
                t = 3 * math.log2(ratio)
                r = int(math.floor(abs(t) + 0.5)) * (1 if t >= 0 else -1)
                assert cost[x, k] == min(255, p["bias"] - r)
        assert (sc == np.maximum(-128, p["bias"] - cost)).all()


# --------------------------------------------------------- hand-worked fixture

def _hand_cases():
    out = []
    for line in open(os.path.join(GOLD, "hand_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, M, bias, ca, cc, tgt, ms, mf, ss, sf = line.split()
        M, bias = int(M), int(bias)
        cost = np.full((32, M), 255, np.uint8)
        cost[0] = [int(v) for v in ca.split(",")]
        cost[1] = [int(v) for v in cc.split(",")]
        sc = np.maximum(-128, bias - cost.astype(int)).astype(np.int8)
        prof = {"cost": cost, "sc": sc, "bias": bias, "M": M, "tbm": q.tbm(M)}
        x = np.array(["AC".index(c) for c in tgt], np.uint8)
        out.append((name, prof, x, (int(ms), int(mf)), (int(ss), int(sf))))
    return out


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c[0])
def test_hand_worked_examples(case):
    name, prof, x, msv_exp, ssv_exp = case
    assert oracle.msv_seq(prof, x) == msv_exp
    assert oracle.ssv_seq(prof, x) == ssv_exp
    # the same profile built from its cost table alone (the non-scoring
    # rows 20 and 27..31 given as anything) scores the same
    cost = prof["cost"].copy()
    cost[20] = 7
    cost[27:] = 7
    p2 = q.from_costs(cost, prof["bias"])
    assert (p2["sc"] == prof["sc"]).all() and (p2["cost"][20] == 255).all()
    assert (p2["cost"][27:] == 255).all()
    assert oracle.msv_seq(p2, x) == msv_exp
    assert oracle.ssv_seq(p2, x) == ssv_exp


# -------------------------------------------- independent implementations

def unbounded_msv(r, M, bias, tbm, x):
    """MSV as an unbounded integer DP over log-odds r (no saturation anywhere).

    V(i,k) = max(V(i-1,k-1), XB(i-1)) + r_k(x_i); XE(i) = max_k V(i,k);
    XJ(i) = max(XJ(i-1), XE(i) - tec); XB(i) = max(base, XJ(i)) - (tjb + tbm).
    The 8-bit filter equals clamp-at-0 of this, with overflow iff some
    XE(i) + bias >= 255.  Returns (score, flag)."""
    L = len(x)
    tjbm = q.tjb(L) + tbm
    tec = q.tec()
    ninf = -math.inf
    V = [ninf] * (M + 1)
    XJ = ninf
    XB = q.BASE - tjbm
    for i in range(L):
        rr = r[int(x[i])]
        newV = [ninf] * (M + 1)
        for k in range(1, M + 1):
            rv = ninf if rr[k - 1] <= NEG // 2 else int(rr[k - 1])
            newV[k] = max(V[k - 1], XB) + rv
        V = newV
        XE = max(V[1:])
        if XE != ninf and XE + bias >= 255:
            return 255, 1
        XJ = max(XJ, XE - tec)
        XB = max(q.BASE, XJ) - tjbm
    return (0 if XJ == ninf else max(0, int(XJ))), 0


def enumerate_msv(r, M, bias, tbm, x):
    """MSV by enumerating every non-empty ordered list of diagonal segments.

    A segment covers rows i0..i0+l-1 and nodes k0..k0+l-1; later segments
    start on a later row than the previous one ends; model positions are
    free.  A list of n segments with sums S_j reaches, at the row its last
    segment ends, E = base - n*tjbm - (n-1)*tec + sum S_j.  The filter
    overflows iff some E + bias >= 255, else scores max(0, max E - tec)."""
    L = len(x)
    tjbm = q.tjb(L) + tbm
    tec = q.tec()
    segs = []
    for i0 in range(L):
        for k0 in range(M):
            s = 0
            for ln in range(1, min(L - i0, M - k0) + 1):
                rv = r[int(x[i0 + ln - 1])][k0 + ln - 1]
                if rv <= NEG // 2:
                    break
                s += int(rv)
                segs.append((i0, i0 + ln - 1, s))
    best = -math.inf

    def rec(last_end, n, total):
        nonlocal best
        for (a, b, s) in segs:
            if a > last_end:
                E = q.BASE - (n + 1) * tjbm - n * tec + total + s
                best = max(best, E)
                rec(b, n + 1, total + s)

    rec(-1, 0, 0)
    if best != -math.inf and best + bias >= 255:
        return 255, 1
    return (0 if best == -math.inf else max(0, int(best) - tec)), 0


def segment_ssv(sc, x, M):
    """SSV as -128 + max(0, best sum of sc over any diagonal segment)."""
    L = len(x)
    best = 0
    for i0 in range(L):
        for k0 in range(M):
            s = 0
            for ln in range(min(L - i0, M - k0)):
                s += int(sc[int(x[i0 + ln])][k0 + ln])
                best = max(best, s)
    if best >= 255:
        return 127, 1
    return best - 128, 0


def _tiny_profile(rng, M, hi):
    """Random log-odds in [-20, hi] with some -inf entries; tables derived."""
    r = np.full((32, M), NEG, np.int64)
    r[:20] = rng.integers(-20, hi + 1, size=(20, M))
    r[:20][rng.random((20, M)) < 0.1] = NEG
    r[0, 0] = max(r[0, 0], 0)           # bias >= 0
    bias = int(r[:20].max())
    cost = np.full((32, M), 255, np.int64)
    cost[:20] = np.minimum(255, bias - r[:20])
    sc = np.maximum(-128, bias - cost)
    return {"r": r, "cost": cost.astype(np.uint8), "sc": sc.astype(np.int8),
            "bias": bias, "M": M, "tbm": q.tbm(M)}


def test_msv_matches_path_enumeration_tiny():
    rng = np.random.default_rng(11)
    seen = {"ovf": 0, "multi": 0, "zero": 0}
    for trial in range(500):
        M = int(rng.integers(1, 4))
        L = int(rng.integers(0, 7))
        prof = _tiny_profile(rng, M, int(rng.integers(5, 60)))
        x = rng.integers(0, 22, size=L).astype(np.uint8)   # some invalid codes
        exp = enumerate_msv(prof["r"], M, prof["bias"], prof["tbm"], x)
        got = oracle.msv_seq(prof, x)
        assert got == exp, (trial, M, L, x, exp, got)
        seen["ovf"] += exp[1]
        seen["multi"] += int(exp[0] > q.BASE)
        seen["zero"] += int(exp == (0, 0))
    # the sample exercised every regime: overflow, the J loop above base, empty
    assert min(seen.values()) > 5, seen


def test_msv_matches_unbounded_dp_random():
    rng = np.random.default_rng(12)
    regimes = {"ovf": 0, "j": 0, "plain": 0}
    for trial in range(60):
        M = int(rng.choice([1, 2, 7, 16, 48]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 8, 0, 90)
        synth.implant(rng, db.res, db.offsets, [emis], 0.5)
        for s in range(db.n):
            x = db.seq(s)
            exp = unbounded_msv(prof["r"], M, prof["bias"], prof["tbm"], x)
            assert oracle.msv_seq(prof, x) == exp, (trial, s)
            regimes["ovf" if exp[1] else ("j" if exp[0] > q.BASE else "plain")] += 1
    assert min(regimes.values()) > 3, regimes


def test_ssv_matches_segment_max():
    rng = np.random.default_rng(13)
    seen_ovf = 0
    for trial in range(200):
        M = int(rng.integers(1, 30))
        L = int(rng.integers(0, 40))
        prof = _tiny_profile(rng, M, int(rng.integers(5, 64)))
        x = rng.integers(0, 24, size=L).astype(np.uint8)
        exp = segment_ssv(prof["sc"].astype(int), x, M)
        assert oracle.ssv_seq(prof, x) == exp, (trial, M, L)
        seen_ovf += exp[1]
    assert seen_ovf > 5


def test_special_cases():
    rng = np.random.default_rng(14)
    for M in (1, 3, 48):
        prof = q.quantize(synth.sample_emissions(rng, M), synth.BG)
        # empty and all-invalid targets
        for x in (np.zeros(0, np.uint8), np.full(17, 20, np.uint8), np.full(5, 31, np.uint8)):
            assert oracle.msv_seq(prof, x) == (0, 0)
            assert oracle.ssv_seq(prof, x) == (-128, 0)
        # L = 1: one row from scB0
        for a in range(20):
            x = np.array([a], np.uint8)
            xb = q.BASE - (q.tjb(1) + prof["tbm"])
            cells = [max(0, xb + prof["bias"] - int(prof["cost"][a, k])) for k in range(M)]
            e = max(cells)
            exp = (255, 1) if e >= 255 - prof["bias"] else (max(0, e - 3), 0)
            assert oracle.msv_seq(prof, x) == exp
            s = max(-128, min(127, max(int(v) for v in prof["sc"][a, :M]) - 128))
            assert oracle.ssv_seq(prof, x) == ((127, 1) if s == 127 else (s, 0))


def test_single_node_multi_hit_closed_form():
    """M = 1: every segment is one cell, so the score is
    max(0, base + best subset sum of (s_i - tjbm - tec)), where the best
    subset takes all positive terms (or the largest single term)."""
    rng = np.random.default_rng(15)
    hits = 0
    for trial in range(300):
        bias = int(rng.integers(0, 40))
        cost = np.full((32, 1), 255, np.uint8)
        cost[:20, 0] = rng.integers(0, 60, size=20)
        cost[int(rng.integers(20)), 0] = 0
        prof = {"cost": cost, "bias": bias, "M": 1, "tbm": q.tbm(1),
                "sc": np.maximum(-128, bias - cost.astype(int)).astype(np.int8)}
        L = int(rng.integers(1, 12))
        x = rng.integers(0, 20, size=L).astype(np.uint8)
        tjbm = q.tjb(L)
        terms = [bias - int(cost[int(c), 0]) - tjbm - 3 for c in x]
        pos = [t for t in terms if t > 0]
        best = sum(pos) if pos else max(terms)
        # overflow: some prefix-chain's E = base + (chain sum) + 3 reaches 255 - bias
        got = oracle.msv_seq(prof, x)
        # the largest E over chains is base + best + tec
        if q.BASE + best + 3 + bias >= 255:
            assert got == (255, 1)
        else:
            assert got == (max(0, q.BASE + best), 0)
            hits += int(len(pos) > 1)
    assert hits > 10


def test_batch_driver_matches_single_calls():
    rng = np.random.default_rng(16)
    prof = q.quantize(synth.sample_emissions(rng, 30), synth.BG)
    db = synth.random_db(rng, 200, 0, 120)
    synth.implant(rng, db.res, db.offsets, [synth.sample_emissions(rng, 30)], 0.2)
    for filt, one in (("msv", oracle.msv_seq), ("ssv", oracle.ssv_seq)):
        s, f = oracle.score_db(filt, prof, db.res, db.offsets, nthreads=4)
        for i in range(db.n):
            assert (int(s[i]), int(f[i])) == one(prof, db.seq(i))
        ids = np.array([5, 3, 99])
        s2, f2 = oracle.score_db(filt, prof, db.res, db.offsets, ids=ids)
        assert (s2[ids] == s[ids]).all() and (f2[ids] == f[ids]).all()


# ------------------------------------------------------ nats and P-values

def test_nats_hand_worked():
    """Raw scores of the hand-worked fixture in nats (s = 3 / ln 2):
    MSV two_node: 197 - tjb(3)=3 - 190 = 4 units -> 4 ln2 / 3 - 3;
    SSV two_node: -110 + 128 - tbm(2)=5 - 2*3 - 3 = 4 units, the same;
    the single best segment (10 + 8 = 18 units) pays the same entry and
    length costs in both filters."""
    from oracle import pvalue as pv
    want = 4 * math.log(2) / 3 - 3
    assert abs(pv.nats("msv", 197, 0, 3, 2) - want) < 1e-15
    assert abs(pv.nats("ssv", -110, 0, 3, 2) - want) < 1e-15
    assert pv.nats("msv", 255, 1, 3, 2) == math.inf
    assert pv.nats("ssv", 127, 1, 3, 2) == math.inf
    # base level: an MSV score of base + tjb is exactly -3 nats
    assert pv.nats("msv", 190 + q.tjb(350), 0, 350, 400) == -3.0
    # 3 units per bit: 3 more units is ln 2 nats more
    d = pv.nats("ssv", 10, 0, 100, 48) - pv.nats("ssv", 7, 0, 100, 48)
    assert abs(d - math.log(2)) < 1e-14


def test_gumbel_closed_forms():
    from oracle import pvalue as pv
    mu, lam = -2.5, 0.69
    # at the location, P = 1 - 1/e
    assert abs(pv.gumbel_p(mu, mu, lam) - (1 - math.exp(-1))) < 1e-15
    # far right tail: P ~ exp(-lambda (x - mu)) with relative error ~ y/2,
    # y = exp(-lambda (x - mu))
    for dx in (20.0, 40.0, 80.0):
        y = math.exp(-lam * dx)
        p = pv.gumbel_p(mu + dx, mu, lam)
        assert abs(p / y - 1) < y
    # far left tail: P -> 1
    assert pv.gumbel_p(mu - 30, mu, lam) == 1.0
    assert pv.gumbel_p(math.inf, mu, lam) == 0.0
    # monotone, and the CDF identity against a direct evaluation where no
    # cancellation occurs
    xs = [mu - 3 + 0.5 * i for i in range(13)]
    ps = [pv.gumbel_p(x, mu, lam) for x in xs]
    assert all(a > b for a, b in zip(ps, ps[1:]))
    for x, p in zip(xs, ps):
        assert abs(p - (1 - math.exp(-math.exp(-lam * (x - mu))))) < 1e-12
