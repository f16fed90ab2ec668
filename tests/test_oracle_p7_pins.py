"""Pins of the oracle's gapped Plan-7 Viterbi (P7Viterbi, paper Eq. 1):
closed-form constants of its quantizer, a hand-worked example, brute force
over every path through the model on tiny inputs, the no-gap case against
an enumeration of multi-segment ungapped paths, and saturation."""
import itertools
import math

import numpy as np

import oracle
from oracle import p7
import synth

NEG = p7.NEG


def test_quantizer_constants():
    # exact powers of two: 32 * log2 is an integer
    assert int(p7.q(0.5)) == -32 and int(p7.q(1.0)) == 0 and int(p7.q(2.0)) == 32
    assert int(p7.q(0.25)) == -64 and int(p7.q(0.0)) == NEG
    # hand-evaluated: 32 log2(3/4) = -13.28, 32 log2(1/6) = -82.72,
    # 32 log2(350/353) = -0.39, 32 log2(3/353) = -220.1
    assert int(p7.q(0.75)) == -13 and int(p7.q(1 / 6)) == -83
    lm = p7.length_model(350)
    assert lm["NN"] == 0 and lm["NB"] == -220 and lm["EC"] == -32
    lm = p7.length_model(3)                     # 3 / 6 = 1/2: both -32
    assert lm["NN"] == -32 and lm["NB"] == -32 and lm["CT"] == -32
    assert p7.length_model(0)["NN"] == NEG and p7.length_model(0)["NB"] == 0
    prof = p7.quantize(np.full((3, 20), 0.05), synth.sample_transitions(
        np.random.default_rng(0), 3), np.full(20, 0.05))
    assert prof["tbm"] == -83                   # 2 / (3 * 4) = 1/6
    # e = bg: every residue and every degenerate code (21..26) scores 0;
    # the non-scoring codes 20 and 27..31 are -inf
    assert (prof["msc"][:20] == 0).all() and (prof["msc"][21:27] == 0).all()
    assert (prof["msc"][20] == NEG).all() and (prof["msc"][27:] == NEG).all()
    # node M has no successor and no insert state
    assert (prof["trans"][:, 2] == NEG).all()


def _hand_profile():
    """M = 2, scores chosen by hand (1/32 bit units)."""
    msc = np.full((32, 2), NEG, np.int16)
    msc[:20] = -40
    msc[0] = [100, -20]          # residue 0 ("A") scores 100 at node 1
    msc[1] = [-30, 90]           # residue 1 ("C") scores 90 at node 2
    trans = np.full((7, 2), NEG, np.int16)
    #        MM   MI   MD   IM   II   DM   DD   (out of node 1)
    trans[:, 0] = [-5, -60, -70, -10, -30, -15, -25]
    return {"M": 2, "msc": msc, "trans": trans, "tbm": -40}


def test_hand_worked_example():
    """Sequence A, G (code 5), C: the best path is N->B->M1 (A) ->I1 (G)
    ->M2 (C) ->E->C->T.  Length model for L = 3: loops and moves -32,
    E->C and E->J -32.
      B(0) = 0 + tNB = -32
      M1 on A: -32 + tbm(-40) + 100 = 28
      I1 on G: 28 + tMI(-60) + 0 = -32
      M2 on C: -32 + tIM(-10) + 90 = 48
      E = 48, C = 48 - 32 = 16, score = C + tCT = 16 - 32 = -16.
    Rivals: M1 (A) -> M2 on G (-20 ... -40) scores less; the N loop over
    A, G then B->M2 on C gives -32 -32 -32 -40 + 90 - 32 - 32 = -110;
    M1 (A) then E, C loops over G, C gives 28 - 32 - 32 - 32 - 32 = -100;
    two hits, M1 on A, E->J, J loop over G, J->B, M2 on C:
    28 - 32 - 32 - 32 - 40 + 90 - 32 - 32 = -82."""
    prof = _hand_profile()
    x = np.array([0, 5, 1], np.uint8)
    assert oracle.p7_seq(prof, x) == (-16, 0)
    # without the insert (M->I at -inf) the two-hit path through J wins
    prof2 = _hand_profile()
    prof2["trans"][1, 0] = NEG
    assert oracle.p7_seq(prof2, x) == (-82, 0)


def _brute(prof, x):
    """Best path score through the Plan-7 model by depth-first enumeration
    of every state path (exact integers, -inf = None), from the model's
    definition: N, J, C emit on their loops; M and I emit on entry (insert
    score 0); D is silent; B->M_j (local entry), M_j->E (local exit)."""
    M, msc, tr = prof["M"], prof["msc"].astype(int), prof["trans"].astype(int)
    lm = p7.length_model(len(x))
    tbm = prof["tbm"]
    L = len(x)
    MM, MI, MD, IM, II, DM, DD = (tr[t] for t in range(7))
    best = [None]

    def val(v):
        return None if v == NEG else v

    def add(s, *ts):
        for t in ts:
            t = val(int(t))
            if s is None or t is None:
                return None
            s = s + t
        return s

    def go(state, j, i, s):
        if s is None:
            return
        if state == "N":
            if i < L:
                go("N", 0, i + 1, add(s, lm["NN"]))
            go("B", 0, i, add(s, lm["NB"]))
        elif state == "B":
            if i < L:
                for k in range(M):
                    go("M", k, i + 1, add(s, tbm, msc[x[i], k]))
        elif state == "M":
            go("E", 0, i, s)
            if i < L:
                if k_ok(j + 1):
                    go("M", j + 1, i + 1, add(s, MM[j], msc[x[i], j + 1]))
                go("I", j, i + 1, add(s, MI[j]))
            if k_ok(j + 1):
                go("D", j + 1, i, add(s, MD[j]))
        elif state == "I":
            if i < L:
                go("I", j, i + 1, add(s, II[j]))
                if k_ok(j + 1):
                    go("M", j + 1, i + 1, add(s, IM[j], msc[x[i], j + 1]))
        elif state == "D":
            if k_ok(j + 1):
                go("D", j + 1, i, add(s, DD[j]))
                if i < L:
                    go("M", j + 1, i + 1, add(s, DM[j], msc[x[i], j + 1]))
        elif state == "E":
            go("C", 0, i, add(s, lm["EC"]))
            go("J", 0, i, add(s, lm["EJ"]))
        elif state == "J":
            if i < L:
                go("J", 0, i + 1, add(s, lm["JJ"]))
            go("B", 0, i, add(s, lm["JB"]))
        elif state == "C":
            if i < L:
                go("C", 0, i + 1, add(s, lm["CC"]))
            else:
                f = add(s, lm["CT"])
                if f is not None and (best[0] is None or f > best[0]):
                    best[0] = f

    def k_ok(k):
        return k < M

    go("N", 0, 0, 0)
    return best[0]


def _random_profile(rng, M, neg_frac=0.0):
    msc = np.full((32, M), NEG, np.int16)
    msc[:20] = rng.integers(-120, 121, size=(20, M))
    trans = rng.integers(-200, 0, size=(7, M)).astype(np.int16)
    trans[rng.random(size=(7, M)) < neg_frac] = NEG
    trans[[0, 2, 3, 5, 6], M - 1] = NEG
    trans[[1, 4], M - 1] = NEG
    return {"M": M, "msc": msc, "trans": trans, "tbm": int(rng.integers(-120, 1))}


def test_brute_force_all_paths():
    """Every path through the model, enumerated, on tiny inputs: the DP's
    int16 result equals the best path (no value saturates at these sizes;
    probability-zero transitions, -inf, included)."""
    rng = np.random.default_rng(71)
    gapped = 0
    for trial in range(120):
        M = int(rng.integers(1, 4))
        L = int(rng.integers(0, 5))
        prof = _random_profile(rng, M, neg_frac=0.2 if trial % 2 else 0.0)
        if trial % 3 == 0:
            # cheap gaps, dear matches: the best paths insert and delete
            g = prof["trans"] != NEG
            prof["trans"][1:][g[1:]] = rng.integers(-20, 0, size=int(g[1:].sum()))
            prof["trans"][0][g[0]] = rng.integers(-200, -100, size=int(g[0].sum()))
        x = rng.integers(0, 21, size=L).astype(np.uint8)   # code 20: -inf emissions
        exp = _brute(prof, x)
        got = oracle.p7_seq(prof, x)
        if exp is None:
            assert got[0] <= -32000 and got[1] == 0, (trial, got)
        else:
            assert got == (exp, 0), (trial, M, L, got, exp)
        # how often an optimal path used a gap: rescore with I/D removed
        nogap = dict(prof, trans=prof["trans"].copy())
        nogap["trans"][[1, 2, 3, 4, 5, 6]] = NEG
        b2 = _brute(nogap, x)
        gapped += exp is not None and b2 is not None and exp > b2
    assert gapped > 5, gapped


def _segments_brute(prof, x):
    """No gaps (M->I, M->D, I->*, D->* all -inf): the best score is the best
    ordered list of ungapped diagonal segments.  Enumerated directly: the
    N loop emits the residues before the first segment, J the ones between
    segments, C the ones after the last."""
    M, msc, tr = prof["M"], prof["msc"].astype(int), prof["trans"].astype(int)
    L = len(x)
    lm = p7.length_model(L)
    tbm = prof["tbm"]
    # a segment: (start residue a, start node k, length n): residues
    # a..a+n-1 on nodes k..k+n-1, entry tbm, M->M between, exit 0
    segs = []
    for a in range(L):
        for k in range(M):
            s = tbm
            for n in range(1, min(L - a, M - k) + 1):
                if n > 1:
                    s += tr[0, k + n - 2]
                s += msc[x[a + n - 1], k + n - 1]
                segs.append((a, n, s))

    from functools import lru_cache

    @lru_cache(maxsize=None)
    def rest(pos, first):
        """Best score of what follows position pos (None: no completion):
        either close (E->C, C loops over the rest, C->T) or take a next
        segment starting at or after pos."""
        out = None if first else lm["EC"] + lm["CC"] * (L - pos) + lm["CT"]
        for a, n, sc in segs:
            if a < pos:
                continue
            gap = a - pos
            lead = lm["NN"] * gap + lm["NB"] if first else \
                lm["EJ"] + lm["JJ"] * gap + lm["JB"]
            tail = rest(a + n, False)
            v = lead + sc + tail
            out = v if out is None else max(out, v)
        return out

    return rest(0, True)


def test_no_gaps_equals_segment_enumeration():
    rng = np.random.default_rng(72)
    multi = 0
    for trial in range(60):
        M = int(rng.integers(1, 6))
        L = int(rng.integers(1, 12))
        prof = _random_profile(rng, M)
        prof["trans"][[1, 2, 3, 4, 5, 6]] = NEG
        x = rng.integers(0, 20, size=L).astype(np.uint8)
        exp = _segments_brute(prof, x)
        assert oracle.p7_seq(prof, x) == (exp, 0), (trial, M, L)
        if L <= 4 and M <= 3:
            assert _brute(prof, x) == exp
    # larger profiles with planted high scores: several segments win
    for trial in range(20):
        M, L = 6, 30
        prof = _random_profile(rng, M)
        prof["trans"][[1, 2, 3, 4, 5, 6]] = NEG
        prof["msc"][0] = 200
        x = rng.choice([0, 1, 2], size=L).astype(np.uint8)
        exp = _segments_brute(prof, x)
        assert oracle.p7_seq(prof, x) == (exp, 0)
        multi += 1
    assert multi == 20


def test_single_node_single_residue_closed_form():
    """M = 1, L = 1: N->B->M1->E->C->T, score = tNB + tBM + msc + tEC + tCT
    (tNB = tCT = q(3/4) = -13, tEC = -32, tBM(1) = q(1) = 0)."""
    rng = np.random.default_rng(73)
    for _ in range(10):
        e = rng.dirichlet(np.ones(20), size=1)
        t = synth.sample_transitions(rng, 1)
        prof = p7.quantize(e, t, synth.BG)
        x = int(rng.integers(0, 20))
        exp = -13 + 0 + int(prof["msc"][x, 0]) - 32 - 13
        assert oracle.p7_seq(prof, np.array([x], np.uint8)) == (exp, 0)
    assert oracle.p7_seq(prof, np.zeros(0, np.uint8)) == (NEG, 0)


def test_saturation_flags_overflow():
    """A profile whose emissions are all at the int16 ceiling: a long
    matching sequence saturates and is flagged; a short one is not."""
    M = 50
    msc = np.full((32, M), NEG, np.int16)
    msc[:20] = -100
    msc[3] = 800
    trans = np.zeros((7, M), np.int16)
    trans[[0, 2, 3, 5, 6], M - 1] = NEG
    trans[[1, 4], M - 1] = NEG
    prof = {"M": M, "msc": msc, "trans": trans, "tbm": 0}
    assert oracle.p7_seq(prof, np.full(45, 3, np.uint8)) == (32767, 1)
    s, f = oracle.p7_seq(prof, np.full(20, 3, np.uint8))
    assert f == 0 and s == 20 * 800 + p7.length_model(20)["NB"] - 32 + \
        p7.length_model(20)["CT"]


def test_batch_equals_single():
    rng = np.random.default_rng(74)
    e = synth.sample_emissions(rng, 25)
    t = synth.sample_transitions(rng, 25)
    prof = p7.quantize(e, t, synth.BG)
    db = synth.random_db(rng, 60, 0, 150)
    synth.implant_gapped(rng, db.res, db.offsets, e, t, 0.5)
    s, f = oracle.p7_score_db(prof, db.res, db.offsets, nthreads=3)
    for i in range(db.n):
        assert (int(s[i]), int(f[i])) == oracle.p7_seq(prof, db.seq(i))
