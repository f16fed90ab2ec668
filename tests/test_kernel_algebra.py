"""CPU model of the reformulations the GPU kernels rely on, checked against the oracle.

The kernels do not run the oracle's loop literally.  They rely on four facts,
each checked here on random inputs in every regime (no hit, J loop, overflow):

I1  a running maximum of the match scores (never reset per row) yields the
    same scJ, because max and "minus tec, floored at 0" commute;
I2  before the first overflow row the 255 (MSV) / 127 (SSV) caps never fire,
    so the kernels can work without the upper clamp and flag overflow once
    the running maximum reaches the threshold;
I3  rows of non-scoring residues appended after a target (row padding) change
    neither the running maximum nor the score;
I4  scB only changes when the running maximum passes max(base + tec, the value
    scB was last computed from), so rows can be run in tiles with scB fixed,
    checked at the tile end, and replayed row by row only when it moved;
I5  with scB fixed, the MSV cell update max(0, max(v, scB) + s) becomes one
    floored add on w = max(v, scB) - scB:  w' = max(w + s, 0).  When scB
    rises by d, every w becomes max(w - d, 0).  A row whose w are all 0 has
    maximum max(0, scB + max_k s_k(x)), so a sequence that never rises above
    scB has running maximum max(0, scB + max over its residues of max_k s_k);
I6  cell values only grow with scB, and scB stays at its start value until
    the running maximum passes base + tec.  So one pass with scB fixed gives
    the exact result when its running maximum stays <= base + tec or reaches
    the overflow threshold; only sequences in between need the pass with
    per-row scB updates;
I7  a cell depends only on the M rows above it along its diagonal, so a
    long target can be cut into segments, each run from `warm` >= M - 1 rows
    before its first row with fresh cells: the maximum over the segments of
    their running maxima (SSV, and MSV with scB fixed) is the target's, since
    warm-up rows only see parts of their diagonals and so never exceed the
    true cells;
I8  with scB fixed, relative cells follow one recurrence whatever scB is,
    and an exact run only lowers them at each rise of scB, so they never
    exceed their fixed-scB values.  scB rises (and a first overflow happens)
    only in a row where a cell passes tjb + tbm + tec above scB, the level a
    fixed-scB cell must pass for the running max to pass base + tec.  Call a
    step loud if a fixed-scB cell in it passes that level: an exact run over
    the rows from `warm` >= M - 1 before the first loud step to the end of
    the last one, with fresh cells, gives the exact score (before the first
    loud step scB never moved; after the last one nothing can change).

and, for P7Viterbi (Eq. 1), on the striped layout of 2G elements of Q
slots with a dummy slot 0:

I9  a D value of row i reaches later results only through D->M into row
    i + 1, where every cell also takes the B->M score; since B >= N + move,
    a D value d with d + max_k tDM_k below sat(sat(N_i + move) + tBM) can
    change no M, no E and no score.  So the D chains need completing across
    elements (Farrar's lazy passes) only while some element's last D rises
    to at least that threshold; any lower threshold is also safe, so the
    kernel takes, for a whole 16-row step, the one of the step's last row
    (N only falls).  The dummy slot may hold any value (all its
    transitions are -inf).
"""
import numpy as np

import oracle
from oracle import quant as q
import synth


def model_msv(prof, x, tile=8, pad=4):
    M, bias = prof["M"], prof["bias"]
    s = bias - prof["cost"].astype(np.int64)          # score added per cell
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    tjbm = q.tjb(L) + prof["tbm"]
    tec, base = q.tec(), q.BASE

    def xb_of(m):
        return max(0, max(base, m - tec) - tjbm)

    R = np.zeros(M, np.int64)
    run = 0                       # running max of cell values (I1)
    built_from = -(1 << 30)       # running max that scB was computed from
    xB = xb_of(built_from)
    flag = False
    i = 0
    while i < len(rows):
        n = min(tile, len(rows) - i)
        ck_R, ck_run = R.copy(), run
        for t in range(n):                             # fast rows: scB fixed
            g = np.concatenate(([0], R[:-1]))
            R = np.maximum(0, np.maximum(g, xB) + s[rows[i + t]])   # no cap (I2)
            run = max(run, int(R.max()))
        moved = run > max(base + tec, built_from) or run >= 255 - bias
        if moved and not flag:                         # replay exactly (I4)
            R, run = ck_R, ck_run
            for t in range(n):
                g = np.concatenate(([0], R[:-1]))
                R = np.maximum(0, np.maximum(g, xB) + s[rows[i + t]])
                run = max(run, int(R.max()))
                if run >= 255 - bias:
                    flag = True
                xB = xb_of(run)
                built_from = run
        i += n
    return (255, 1) if flag else (max(0, run - tec), 0)


def model_msv_w(prof, x, tile=8, pad=4):
    """The kernel's MSV: relative cells w (I5), lazy scB tiles (I4)."""
    M, bias = prof["M"], prof["bias"]
    s = bias - prof["cost"].astype(np.int64)
    best = s.max(axis=1)                      # max_k s_k(x) per residue
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    tjbm = q.tjb(L) + prof["tbm"]
    tec, base = q.tec(), q.BASE

    def xb_of(m):
        return max(0, max(base, m - tec) - tjbm)

    xb = xb_of(-(1 << 30))
    Wc = np.zeros(M, np.int64)            # relative cells
    run = 0                               # running max of w in this scB epoch
    cm = -1                               # exact running max of earlier epochs
    built = -(1 << 30)
    flag = False

    def cummax():
        return max(cm, run + xb if run > 0 else -1)

    i = 0
    while i < len(rows):
        n = min(tile, len(rows) - i)
        ck_W, ck_run = Wc.copy(), run
        for t in range(n):
            g = np.concatenate(([0], Wc[:-1]))
            Wc = np.maximum(0, g + s[rows[i + t]])
            run = max(run, int(Wc.max()))
        c = cummax()
        moved = c > max(base + tec, built) or c >= 255 - bias
        if moved and not flag:
            Wc, run = ck_W, ck_run
            for t in range(n):
                g = np.concatenate(([0], Wc[:-1]))
                Wc = np.maximum(0, g + s[rows[i + t]])
                run = max(run, int(Wc.max()))
                c = cummax()
                if c >= 255 - bias:
                    flag = True
                xbn = xb_of(c)
                if xbn > xb:                    # new scB epoch
                    Wc = np.maximum(0, Wc - (xbn - xb))
                    cm = max(cm, c)
                    run = 0
                    xb = xbn
                built = c
        i += n
    c = cummax()
    if c < 0:                                   # never above scB: exact from the residues
        c = max(0, xb + int(max(best[r] for r in rows)))
    if flag or c >= 255 - bias:
        return 255, 1
    return max(0, c - tec), 0


def model_msv_two_pass(prof, x, pad=4):
    """Pass 1 with scB fixed (I6, I5 cells); pass 2 (exact, per-row scB) only
    for sequences whose fixed-scB maximum lies in (base + tec, 255 - dbias)."""
    M, bias = prof["M"], prof["bias"]
    s = bias - prof["cost"].astype(np.int64)
    best = s.max(axis=1)
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    tjbm = q.tjb(L) + prof["tbm"]
    tec, base = q.tec(), q.BASE
    xb0 = max(0, base - tjbm)
    Wc = np.zeros(M, np.int64)
    run = 0
    for r in rows:
        Wc = np.maximum(0, np.concatenate(([0], Wc[:-1])) + s[r])
        run = max(run, int(Wc.max()))
    c = run + xb0 if run > 0 else max(0, xb0 + int(max(best[r] for r in rows)))
    if c >= 255 - bias:
        return (255, 1), "pass1"
    if c <= base + tec:
        return (max(0, c - tec), 0), "pass1"
    # pass 2: exact, scB updated after every row, cells relative to scB
    xb, cm, run, flag = xb0, -1, 0, False
    Wc = np.zeros(M, np.int64)
    for r in rows:
        Wc = np.maximum(0, np.concatenate(([0], Wc[:-1])) + s[r])
        run = max(run, int(Wc.max()))
        c = max(cm, run + xb if run > 0 else -1)
        if c >= 255 - bias:
            flag = True
        xbn = max(0, max(base, c - tec) - tjbm)
        if xbn > xb:
            Wc = np.maximum(0, Wc - (xbn - xb))
            cm, run, xb = c, 0, xbn
    c = max(cm, run + xb if run > 0 else -1)
    if c < 0:
        c = max(0, xb + int(max(best[r] for r in rows)))
    if flag or c >= 255 - bias:
        return (255, 1), "pass2"
    return (max(0, c - tec), 0), "pass2"


def test_msv_two_pass_matches_oracle():
    rng = np.random.default_rng(24)
    seen = {"pass1": 0, "pass2": 0}
    for trial in range(40):
        M = int(rng.choice([1, 3, 16, 48, 130]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 12, 0, 200)
        synth.implant(rng, db.res, db.offsets, [emis], 0.4)
        for sidx in range(db.n):
            x = db.seq(sidx)
            got, how = model_msv_two_pass(prof, x)
            assert got == oracle.msv_seq(prof, x), (trial, sidx, how)
            seen[how] += 1
    assert min(seen.values()) > 3, seen


def model_ssv(prof, x, pad=4):
    M = prof["M"]
    sc = prof["sc"].astype(np.int64)
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    R = np.full(M, -128, np.int64)
    run = -128
    for r in rows:
        g = np.concatenate(([-128], R[:-1]))
        R = np.maximum(-128, g + sc[r])                # no cap (I2)
        run = max(run, int(R.max()))
    return (127, 1) if run >= 127 else (run, 0)


def test_msv_kernel_reformulation_matches_oracle():
    rng = np.random.default_rng(21)
    regimes = {"ovf": 0, "j": 0, "plain": 0}
    for trial in range(40):
        M = int(rng.choice([1, 3, 16, 48, 130]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 12, 0, 200)
        synth.implant(rng, db.res, db.offsets, [emis], 0.4)
        for sidx in range(db.n):
            x = db.seq(sidx)
            exp = oracle.msv_seq(prof, x)
            for tile in (4, 8, 32):
                assert model_msv(prof, x, tile) == exp, (trial, sidx, tile)
                assert model_msv_w(prof, x, tile) == exp, (trial, sidx, tile, "w")
            regimes["ovf" if exp[1] else ("j" if exp[0] > q.BASE else "plain")] += 1
    assert min(regimes.values()) > 3, regimes


def test_msv_relative_cells_edge_cases():
    """I5 on sequences that never rise above scB (all-invalid, empty, and
    residues whose best score is negative) and on a profile where every
    residue but one scores below zero."""
    rng = np.random.default_rng(23)
    for M in (1, 5, 40):
        prof = q.quantize(synth.sample_emissions(rng, M), synth.BG)
        for x in (np.zeros(0, np.uint8), np.full(7, 20, np.uint8), np.full(3, 31, np.uint8)):
            assert model_msv_w(prof, x) == oracle.msv_seq(prof, x)
        s = prof["bias"] - prof["cost"].astype(int)
        neg = [a for a in range(20) if s[a].max() < 0]
        if neg:
            for L in (1, 4, 9, 30):
                x = rng.choice(neg, size=L).astype(np.uint8)
                assert model_msv_w(prof, x) == oracle.msv_seq(prof, x)
    # a hand-made profile: only residue 0 scores positive anywhere
    M = 6
    cost = np.full((32, M), 255, np.uint8)
    cost[:20] = 40
    cost[0] = 0
    prof = {"cost": cost, "sc": np.maximum(-128, 20 - cost.astype(int)).astype(np.int8),
            "bias": 20, "M": M, "tbm": q.tbm(M)}
    for xs in ([1, 2, 3], [5] * 11, [0, 1, 0, 1], [3, 0, 0, 0, 0, 0, 0, 9]):
        x = np.array(xs, np.uint8)
        assert model_msv_w(prof, x) == oracle.msv_seq(prof, x)


def test_ssv_kernel_reformulation_matches_oracle():
    rng = np.random.default_rng(22)
    nov = 0
    for trial in range(40):
        M = int(rng.choice([1, 3, 16, 48, 130]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 12, 0, 200)
        synth.implant(rng, db.res, db.offsets, [emis], 0.4)
        for sidx in range(db.n):
            x = db.seq(sidx)
            exp = oracle.ssv_seq(prof, x)
            assert model_ssv(prof, x) == exp
            nov += exp[1]
    assert nov > 3


def model_split_max(prof, x, filt, T, warm, pad=4):
    """I7: running maximum of a target run in segments of T rows, each with
    `warm` rows before it (SSV cells, or MSV cells with scB fixed)."""
    M = prof["M"]
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    R = len(rows)
    if filt == "ssv":
        add, floor = prof["sc"].astype(np.int64), -128
    else:
        add, floor = prof["bias"] - prof["cost"].astype(np.int64), 0
    best = floor
    for beg in range(0, R, T):
        cells = np.full(M, floor, np.int64)
        for r in rows[max(0, beg - warm):min(R, beg + T)]:
            cells = np.maximum(floor, np.concatenate(([floor], cells[:-1])) + add[r])
            best = max(best, int(cells.max()))
    return best


def test_split_targets_keep_the_running_max():
    """I7 for both filters on random profiles and targets with hits, for
    segment lengths from 4 rows up and the smallest warm-up M - 1; one row
    less of warm-up must fail somewhere (the bound is tight)."""
    rng = np.random.default_rng(25)
    short_fails = 0
    for trial in range(30):
        M = int(rng.choice([2, 3, 16, 48]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 6, 40, 300)
        synth.implant(rng, db.res, db.offsets, [emis], 0.5)
        for sidx in range(db.n):
            x = db.seq(sidx)
            for filt in ("ssv", "msv"):
                whole = model_split_max(prof, x, filt, 1 << 20, 0)
                for T in (4, 16, 52):
                    assert model_split_max(prof, x, filt, T, M - 1) == whole, (trial, sidx, T)
                    assert model_split_max(prof, x, filt, T, M + 7) == whole
                    if M > 1:
                        short_fails += model_split_max(prof, x, filt, T, M - 2) != whole
            # the whole-target maximum is the kernels' pass-1 quantity
            whole_ssv = model_split_max(prof, x, "ssv", 1 << 20, 0)
            assert model_ssv(prof, x) == ((127, 1) if whole_ssv >= 127 else (whole_ssv, 0))
    assert short_fails > 0


def model_msv_split(prof, x, T, warm, pad=4):
    """The kernels' MSV on a split target: each segment's pass-1 maximum
    (I5 form, including the never-above-scB case), combined by max; an exact
    pass only when the combined maximum lies in (base + tec, 255 - dbias),
    and then only from the first segment whose own maximum passed base + tec
    (scB cannot move earlier, and that segment's warm-up cells stay below
    the true ones)."""
    bias = prof["bias"]
    s = bias - prof["cost"].astype(np.int64)
    best = s.max(axis=1)
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    R = len(rows)
    tjbm = q.tjb(L) + prof["tbm"]
    xb0 = max(0, q.BASE - tjbm)
    c, hot = 0, None
    for beg in range(0, R, T):
        seg = rows[max(0, beg - warm):min(R, beg + T)]
        W = np.zeros(prof["M"], np.int64)
        run = 0
        for r in seg:
            W = np.maximum(0, np.concatenate(([0], W[:-1])) + s[r])
            run = max(run, int(W.max()))
        cs = run + xb0 if run > 0 else max(0, xb0 + int(max(best[r] for r in seg)))
        c = max(c, cs)
        if cs > q.BASE + q.tec() and hot is None:
            hot = max(0, beg - warm)
    if c >= 255 - bias:
        return 255, 1
    if c <= q.BASE + q.tec():
        return max(0, c - q.tec()), 0
    # exact pass (scB updated after every row) from the first hot segment's
    # first warm-up row, with fresh cells and scB at its start value
    tec, base = q.tec(), q.BASE
    xb, cm, run, flag = xb0, -1, 0, False
    W = np.zeros(prof["M"], np.int64)
    for r in rows[hot:]:
        W = np.maximum(0, np.concatenate(([0], W[:-1])) + s[r])
        run = max(run, int(W.max()))
        cc = max(cm, run + xb if run > 0 else -1)
        if cc >= 255 - bias:
            flag = True
        xbn = max(0, max(base, cc - tec) - tjbm)
        if xbn > xb:
            W = np.maximum(0, W - (xbn - xb))
            cm, run, xb = cc, 0, xbn
    cc = max(cm, run + xb if run > 0 else -1)
    if flag or cc >= 255 - bias:
        return 255, 1
    return max(0, cc - tec), 0


def test_msv_split_matches_oracle():
    rng = np.random.default_rng(26)
    regimes = {"ovf": 0, "j": 0, "plain": 0}
    for trial in range(30):
        M = int(rng.choice([1, 3, 16, 48]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 8, 0, 300)
        synth.implant(rng, db.res, db.offsets, [emis], 0.4)
        for sidx in range(db.n):
            x = db.seq(sidx)
            exp = oracle.msv_seq(prof, x)
            for T in (4, 16, 64):
                assert model_msv_split(prof, x, T, max(0, M - 1)) == exp, (trial, sidx, T)
            regimes["ovf" if exp[1] else ("j" if exp[0] > q.BASE else "plain")] += 1
    assert min(regimes.values()) > 3, regimes


def model_msv_rescore_from_step(prof, x, step, warm, pad=4):
    """MSV as groups of up to 4 lanes run it: pass 1 with scB fixed notes
    the first step (of `step` rows) after which the running max passed
    base + tec; an exact pass, if needed, starts `warm` rows before that
    step (rounded down to 16 rows) with fresh cells."""
    bias = prof["bias"]
    s = bias - prof["cost"].astype(np.int64)
    best = s.max(axis=1)
    L = len(x)
    rows = list(x) + [20] * ((-L) % pad if L else pad)
    tjbm = q.tjb(L) + prof["tbm"]
    tec, base = q.tec(), q.BASE
    xb0 = max(0, base - tjbm)
    W = np.zeros(prof["M"], np.int64)
    run, hot = 0, None
    for i, r in enumerate(rows):
        W = np.maximum(0, np.concatenate(([0], W[:-1])) + s[r])
        run = max(run, int(W.max()))
        if (i + 1) % step == 0 or i + 1 == len(rows):
            if hot is None and run > 0 and run + xb0 > base + tec:
                hot = (i // step) * step                  # the step's first row
    c = run + xb0 if run > 0 else max(0, xb0 + int(max(best[r] for r in rows)))
    if c >= 255 - bias:
        return 255, 1
    if c <= base + tec:
        return max(0, c - tec), 0
    b = hot - warm if hot >= warm else 0
    b -= b % 16
    xb, cm, run, flag = xb0, -1, 0, False
    W = np.zeros(prof["M"], np.int64)
    for r in rows[b:]:
        W = np.maximum(0, np.concatenate(([0], W[:-1])) + s[r])
        run = max(run, int(W.max()))
        cc = max(cm, run + xb if run > 0 else -1)
        if cc >= 255 - bias:
            flag = True
        xbn = max(0, max(base, cc - tec) - tjbm)
        if xbn > xb:
            W = np.maximum(0, W - (xbn - xb))
            cm, run, xb = cc, 0, xbn
    cc = max(cm, run + xb if run > 0 else -1)
    if flag or cc >= 255 - bias:
        return 255, 1
    return max(0, cc - tec), 0


def test_msv_rescore_from_step_matches_oracle():
    rng = np.random.default_rng(27)
    late = 0
    for trial in range(30):
        M = int(rng.choice([1, 3, 16, 48]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 8, 0, 400)
        synth.implant(rng, db.res, db.offsets, [emis], 0.4)
        for sidx in range(db.n):
            x = db.seq(sidx)
            exp = oracle.msv_seq(prof, x)
            for step in (8, 16):
                got = model_msv_rescore_from_step(prof, x, step, max(0, M - 1))
                assert got == exp, (trial, sidx, step)
            late += exp[1] == 0 and exp[0] > q.BASE and len(x) > 100
    assert late > 3


def test_models_across_the_bias_range():
    """The reformulations (I1..I7) hold over the whole accepted dbias range,
    on profiles given directly as cost tables: dbias 0 (no cell ever rises
    above scB), 20 and 40 (J state and overflow), 61..64 (overflow comes
    before the running max can pass base + tec).  Sequences carry consensus
    runs on random and on non-scoring backgrounds."""
    rng = np.random.default_rng(28)
    seen = {"ovf": 0, "j": 0, "plain": 0}
    for dbias in (0, 20, 40, 61, 62, 63, 64):
        for M in (1, 3, 16, 48):
            cost, cons = synth.random_cost_table(rng, M, dbias)
            prof = q.from_costs(cost, dbias)
            db = synth.random_db(rng, 8, 0, 160)
            synth.implant_consensus(rng, db.res, db.offsets, cons, 0.8, 24)
            lad = synth.random_db(rng, 8, 1, 160)
            lad.res[:] = 20
            synth.implant_consensus(rng, lad.res, lad.offsets, cons, 1.0, 24, (1, 3))
            for x in [db.seq(i) for i in range(db.n)] + [lad.seq(i) for i in range(lad.n)]:
                exp = oracle.msv_seq(prof, x)
                for tile in (4, 32):
                    assert model_msv_w(prof, x, tile) == exp, (dbias, M, tile)
                assert model_msv_two_pass(prof, x)[0] == exp, (dbias, M)
                assert model_msv_split(prof, x, 16, max(0, M - 1)) == exp, (dbias, M)
                assert model_msv_rescore_from_step(prof, x, 16, max(0, M - 1)) == exp, \
                    (dbias, M)
                assert model_ssv(prof, x) == oracle.ssv_seq(prof, x), (dbias, M)
                seen["ovf" if exp[1] else ("j" if exp[0] > q.BASE else "plain")] += 1
    assert min(seen.values()) > 10, seen


def exact_run(prof, rows, tjbm):
    """Alg. 2 special states after every row (cells relative to scB, I5),
    from fresh cells: (exact running max or -1, overflow)."""
    bias = prof["bias"]
    s = bias - prof["cost"].astype(np.int64)
    tec, base = q.tec(), q.BASE
    xb = max(0, base - tjbm)
    cm, run, flag = -1, 0, False
    W = np.zeros(prof["M"], np.int64)
    for r in rows:
        W = np.maximum(0, np.concatenate(([0], W[:-1])) + s[r])
        run = max(run, int(W.max()))
        cc = max(cm, run + xb if run > 0 else -1)
        if cc >= 255 - bias:
            flag = True
        xbn = max(0, max(base, cc - tec) - tjbm)
        if xbn > xb:
            W = np.maximum(0, W - (xbn - xb))
            cm, run, xb = cc, 0, xbn
    return max(cm, run + xb if run > 0 else -1), flag


def model_msv_window(prof, x, step, warm, T=None, end_short=0, align=16):
    """I8, as the kernels run MSV: pass 1 with scB fixed (segments of T rows
    after `warm` warm-up rows if T is given, I7) notes the first and last
    loud steps; the exact pass runs only the window from `warm` rows before
    the first loud step (rounded down to 16) to the end of the last one
    (`end_short` steps less, to show the bound is needed)."""
    bias = prof["bias"]
    s = bias - prof["cost"].astype(np.int64)
    best = s.max(axis=1)
    L = len(x)
    rows = list(x) + [20] * ((-L) % step if L else step)
    R = len(rows)
    tjbm = q.tjb(L) + prof["tbm"]
    tec, base = q.tec(), q.BASE
    xb0 = max(0, base - tjbm)
    level = min(base + tec, 254 - bias) - xb0
    T = T or R
    c, first, last = 0, None, None
    for beg in range(0, R, T):
        b0 = max(0, beg - warm)
        W = np.zeros(prof["M"], np.int64)
        run = 0
        for i in range(b0, min(R, beg + T)):
            W = np.maximum(0, np.concatenate(([0], W[:-1])) + s[rows[i]])
            m = int(W.max())
            run = max(run, m)
            if m > level:                              # a loud row: its step is loud
                st0 = b0 + ((i - b0) // step) * step
                first = st0 if first is None else min(first, st0)
                last = st0 if last is None else max(last, st0)
        seg = rows[b0:min(R, beg + T)]
        cs = run + xb0 if run > 0 else max(0, xb0 + int(max(best[r] for r in seg)))
        c = max(c, cs)
    if c >= 255 - bias:
        return 255, 1
    if c <= base + tec:
        return max(0, c - tec), 0
    ws = first - warm if first >= warm else 0
    ws -= ws % align
    we = last + step - end_short * step
    if align == 16:
        # the exact pass runs whole 16-row steps: the sequence's later rows,
        # then non-scoring padding (sequences are stored in 16-row steps)
        rows = rows + [20] * ((-len(rows)) % 16)
        we = min(len(rows), ws + (we - ws + 15) // 16 * 16)
    cc, flag = exact_run(prof, rows[ws:we], tjbm)
    if flag or cc >= 255 - bias:
        return 255, 1
    return max(0, cc - tec), 0


def test_msv_windowed_rescore_matches_oracle():
    """I8 on targets with several hits far apart (quiet stretches between
    them), whole and split into segments, for both step sizes the kernels
    use; a window one step short at its end, or (rows taken one at a time)
    with one row less of warm-up, must fail somewhere."""
    rng = np.random.default_rng(29)
    regimes = {"ovf": 0, "j": 0, "plain": 0}
    short_end = short_warm = 0
    for trial in range(30):
        M = int(rng.choice([1, 3, 16, 48]))
        emis = synth.sample_emissions(rng, M)
        prof = q.quantize(emis, synth.BG)
        db = synth.random_db(rng, 8, 0, 500)
        for _ in range(3):
            synth.implant(rng, db.res, db.offsets, [emis], 0.5)
        for sidx in range(db.n):
            x = db.seq(sidx)
            exp = oracle.msv_seq(prof, x)
            w = max(0, M - 1)
            for step in (8, 16):
                assert model_msv_window(prof, x, step, w) == exp, (trial, sidx, step)
                assert model_msv_window(prof, x, step, w + 16) == exp
                for T in (64, 96):
                    assert model_msv_window(prof, x, step, max(w, 16), T) == exp, \
                        (trial, sidx, step, T)
                short_end += model_msv_window(prof, x, step, w, end_short=1) != exp
            if M > 1:
                # rows one at a time, no rounding: M - 1 rows of warm-up suffice,
                # M - 2 do not
                assert model_msv_window(prof, x, 1, w, align=1) == exp
                short_warm += model_msv_window(prof, x, 1, w - 1, align=1) != exp
            regimes["ovf" if exp[1] else ("j" if exp[0] > q.BASE else "plain")] += 1
    assert min(regimes.values()) > 3, regimes
    assert short_end > 0 and short_warm > 0, (short_end, short_warm)


# ---------------------------------------------------------------- P7Viterbi

def model_p7_striped(prof, x, G, Q, junk_rng):
    """The P7 kernel's row update on the striped layout (slot s = q + Q e,
    element e = 2 lane + half, slot 0 a dummy node) with the thresholded
    lazy completion of the D chains (I9).  The dummy slot's diagonal
    inputs come from another group (random values here).  Returns (score,
    flag, rows that ran a lazy pass)."""
    from oracle import p7 as op7
    NEG, POS = -32768, 32767

    def sat(v):
        return np.clip(v, NEG, POS)

    M, msc, tr, tbm = prof["M"], prof["msc"].astype(np.int64), prof["trans"].astype(np.int64), \
        prof["tbm"]
    E2 = 2 * G
    assert 2 * G * Q - 1 >= M
    slot = np.arange(E2 * Q).reshape(E2, Q)           # [e, q] -> s = q + Q e

    def by_node(row, frm):
        n = slot if frm == "self" else slot - 1
        ok = (n >= 1) & (n <= M)
        return np.where(ok, row[np.clip(n - 1, 0, M - 1)], NEG)

    MM, MI, MD, IM, II, DM, DD = (by_node(tr[t], "self" if t in (1, 4) else "prev")
                                  for t in range(7))
    real = (slot >= 1) & (slot <= M)
    maxdm = int(tr[5].max())
    L = len(x)
    lm = op7.length_model(L)
    loop, move = lm["NN"], lm["NB"]
    Mr = np.full((E2, Q), NEG)
    Ir = Mr.copy()
    Dr = Mr.copy()
    xN, xB, xJ, xC, ovf, lazy_rows = 0, sat(move), NEG, NEG, False, 0

    def shift(a):
        out = np.empty(E2, np.int64)
        out[1:] = a[:-1]
        out[0] = junk_rng.integers(NEG, POS + 1)
        return out

    for i in range(L):
        em = np.where(real, msc[x[i]][np.clip(slot - 1, 0, M - 1)], NEG)
        bc = sat(xB + tbm)
        nN = sat(xN + loop)
        if i % 16 == 0:
            # one bound per 16-row step: the step's last row's (N only falls)
            thr1 = int(np.clip(sat(sat(sat(xN + 16 * loop) + move) + tbm) - maxdm - 1,
                               NEG, POS))
        gM = np.concatenate([shift(Mr[:, Q - 1])[:, None], Mr[:, :-1]], axis=1)
        gI = np.concatenate([shift(Ir[:, Q - 1])[:, None], Ir[:, :-1]], axis=1)
        gD = np.concatenate([shift(Dr[:, Q - 1])[:, None], Dr[:, :-1]], axis=1)
        Ir = np.maximum(sat(Mr + MI), sat(Ir + II))
        c = np.maximum(np.maximum(sat(gM + MM), sat(gI + IM)), np.maximum(sat(gD + DM), bc))
        Mr = sat(c + em)
        Dr = np.full((E2, Q), NEG)
        # slot 0 takes the previous element's last M in the first pass
        Dr[:, 0] = sat(shift(Mr[:, Q - 1]) + MD[:, 0])
        for q in range(1, Q):
            Dr[:, q] = np.maximum(sat(Mr[:, q - 1] + MD[:, q]), sat(Dr[:, q - 1] + DD[:, q]))
        in0 = sat(shift(Dr[:, Q - 1]) + DD[:, 0])
        lim = np.maximum(Dr[:, 0], thr1)
        more = bool((in0 > lim).any())
        lazy_rows += more
        while more:
            last = Dr[:, Q - 1].copy()
            Dr[:, 0] = np.maximum(Dr[:, 0], in0)
            for q in range(1, Q):
                Dr[:, q] = np.maximum(Dr[:, q], sat(Dr[:, q - 1] + DD[:, q]))
            more = bool((Dr[:, Q - 1] > np.maximum(last, thr1)).any())
            in0 = sat(shift(Dr[:, Q - 1]) + DD[:, 0])
        Ev = int(Mr.max())
        if Ev >= POS:
            ovf = True
        e2 = sat(Ev - 32)
        xJ = max(sat(xJ + loop), e2)
        xC = max(sat(xC + loop), e2)
        xN = nN
        xB = sat(max(xN, xJ) + move)
    return (POS if ovf else int(sat(xC + move))), int(ovf), lazy_rows


def test_p7_thresholded_lazy_passes_match_oracle():
    """I9 on random profiles (some with -inf transitions and emissions),
    targets with gapped implants, several striped shapes: the model's
    scores equal the oracle's, rows with and without lazy passes occur."""
    from oracle import p7 as op7
    rng = np.random.default_rng(909)
    lazy = rows = 0
    for trial in range(24):
        M = int(rng.integers(1, 60))
        G = int(rng.choice([1, 2, 4, 8]))
        Q = max(1, -(-(M + 1) // (2 * G))) + int(rng.integers(0, 2))
        e = synth.sample_emissions(rng, M, conc=0.5 if trial % 3 else 5.0)
        t = synth.sample_transitions(rng, M, conc=20.0 if trial % 2 else 2.0)
        if trial % 4 == 3:
            t[rng.random(t.shape) < 0.1] = 0.0
            e[rng.random(e.shape) < 0.05] = 0.0
            e[:, 0] += 1e-3
        prof = op7.quantize(e, t, synth.BG)
        L = rng.integers(0, 90, size=6)
        res, off = synth.sample_residues(rng, L.astype(np.int64))
        synth.implant_gapped(rng, res, off, e, t, 0.7)
        for k in range(len(L)):
            xk = res[off[k]:off[k + 1]]
            got = model_p7_striped(prof, xk, G, Q, rng)
            assert got[:2] == oracle.p7_seq(prof, xk), (trial, M, G, Q, k)
            lazy += got[2]
            rows += len(xk)
    assert 0 < lazy < rows, (lazy, rows)

