"""Pins of the oracle's degenerate-residue scores (codes 21..26).

Reading: a degenerate code (B = {D, N}, J = {I, L}, Z = {E, Q}, U = {C},
O = {K}, X = any of the twenty) scores the background-weighted mean of its
members' log2 odds ratios, in the units of each filter; the paper's score
table has 32 entries per node (Alg. 4, Sec. 3.3) but does not say how
ambiguous residues score.  Pinned by a hand-worked fixture
(tests/golden/degenerate.txt), single-member sets, bounds, and the DP on
sequences where a single-member code replaces its member."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import p7 as op7
from oracle import quant as oq

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "degenerate.txt")
A = synth.ALPHABET


def _fixture_profile():
    bg = np.full(20, 0.05)
    bg[A.index("D")] = 0.08
    bg[A.index("N")] = 0.02
    e = np.tile(bg, (3, 1))
    e[0, A.index("D")] = 0.16
    e[0, A.index("N")] = 0.08
    e[0, A.index("I")] = 0.40
    e[0, A.index("L")] = 0.025
    e[0, A.index("E")] = 0.0
    e[0, A.index("C")] = 0.20
    e[1, A.index("A")] = 0.10
    e[1, A.index("C")] = 0.20
    e[2, A.index("N")] = 0.005
    return e, bg


def _golden():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        node, code, msv, p7v = line.split()
        rows.append((int(node), int(code), msv, p7v))
    return rows


def test_hand_worked_degenerate_scores():
    e, bg = _fixture_profile()
    r = oq.log_odds(e, bg)
    prof = oq.quantize(e, bg)
    p7 = op7.quantize(e, np.full((3, 7), 0.5), bg)
    bias = prof["bias"]
    assert bias == 9                     # node 1, I: RHAZ(3 * 3)
    rows = _golden()
    assert len(rows) == 18
    for node, code, msv, p7v in rows:
        k = node - 1
        if msv == "-inf":
            assert r[code, k] == oq.NEG_INF and prof["cost"][code, k] == 255
        else:
            assert r[code, k] == int(msv), (node, code)
            assert prof["cost"][code, k] == bias - int(msv)
            assert prof["sc"][code, k] == int(msv)
        expect = op7.NEG if p7v == "-inf" else int(p7v)
        assert p7["msc"][code, k] == expect, (node, code)


def test_single_member_codes_equal_their_member():
    rng = np.random.default_rng(5)
    for M in (1, 17, 400):
        e = synth.sample_emissions(rng, M)
        prof = oq.quantize(e, synth.BG)
        p7 = op7.quantize(e, synth.sample_transitions(rng, M), synth.BG)
        for code, letter in ((24, "C"), (25, "K")):
            assert (prof["cost"][code] == prof["cost"][A.index(letter)]).all()
            assert (p7["msc"][code] == p7["msc"][A.index(letter)]).all()


def test_degenerate_scores_lie_between_their_members():
    rng = np.random.default_rng(6)
    e = synth.sample_emissions(rng, 300, conc=2.0)
    r = oq.log_odds(e, synth.BG)
    p7 = op7.quantize(e, synth.sample_transitions(rng, 300), synth.BG)["msc"].astype(np.int64)
    for code, members in oq.DEGENERATE.items():
        mem = np.array(members)
        assert (r[code] >= r[mem].min(0)).all() and (r[code] <= r[mem].max(0)).all()
        assert (p7[code] >= p7[mem].min(0)).all() and (p7[code] <= p7[mem].max(0)).all()
    # X is the background-weighted mean over all twenty: with e = bg it is 0
    flat = oq.log_odds(np.tile(synth.BG, (4, 1)), synth.BG)
    assert (flat[21:27] == 0).all()


def test_non_scoring_codes_stay_minus_infinity():
    rng = np.random.default_rng(7)
    e = synth.sample_emissions(rng, 50)
    prof = oq.quantize(e, synth.BG)
    p7 = op7.quantize(e, synth.sample_transitions(rng, 50), synth.BG)
    for code in (20, 27, 28, 29, 30, 31):
        assert (prof["cost"][code] == 255).all() and (prof["sc"][code] == -128).all()
        assert (p7["msc"][code] == op7.NEG).all()
    # tables given directly keep their degenerate rows and lose the others
    cost = rng.integers(0, 256, size=(32, 50)).astype(np.uint8)
    fc = oq.from_costs(cost, 20)
    assert (fc["cost"][21:27] == cost[21:27]).all()
    assert (fc["cost"][20] == 255).all() and (fc["cost"][27:] == 255).all()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dp_scores_single_member_code_like_its_member(seed):
    """U and O score exactly like C and K in all three filters."""
    rng = np.random.default_rng(seed)
    M = 40
    e = synth.sample_emissions(rng, M)
    t = synth.sample_transitions(rng, M)
    prof = oq.quantize(e, synth.BG)
    p7 = op7.quantize(e, t, synth.BG)
    x = rng.integers(0, 20, size=200).astype(np.uint8)
    x[:60] = np.tile(np.argmax(e, axis=1), 2)[:60]
    y = x.copy()
    y[x == A.index("C")] = 24
    y[x == A.index("K")] = 25
    assert (y >= 24).sum() > 5
    assert oracle.msv_seq(prof, x) == oracle.msv_seq(prof, y)
    assert oracle.ssv_seq(prof, x) == oracle.ssv_seq(prof, y)
    assert oracle.p7_seq(p7, x) == oracle.p7_seq(p7, y)
    # and X, a genuinely new score, changes them
    z = x.copy()
    z[::3] = 26
    assert oracle.p7_seq(p7, z) != oracle.p7_seq(p7, x)
