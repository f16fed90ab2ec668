"""GPU parity of the pipeline stages chained on the device (Sec. 2.1): the
filter stage (MSV or SSV) over the whole database, the survivors selected
on the device (hmsv_select), then P7Viterbi on those only
(hmsv_p7_score_selected).

The selection is checked, position for position, against its definition
applied to the oracle's filter scores and the database's processing order;
the P7 scores of the survivors against the oracle's P7Viterbi; every other
entry must keep the value it had."""
import numpy as np
import pytest

import oracle
from oracle import p7 as op7
from oracle import quant as oq
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as m
    return m


def _case(seed, M, nseq, lo, hi, frac=0.1):
    rng = np.random.default_rng(seed)
    e = synth.sample_emissions(rng, M)
    t = synth.sample_transitions(rng, M)
    L = rng.integers(lo, hi + 1, size=nseq).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    synth.implant_gapped(rng, res, off, e, t, frac)
    return e, t, res, off


def _expected_positions(order, score, flags, thr):
    """The definition: processing positions p (increasing) whose sequence
    order[p] overflowed or scored at least thr."""
    keep = (flags[order] != 0) | (score[order].astype(np.int64) >= thr)
    return np.nonzero(keep)[0].astype(np.int32)


def _survivor_threshold(score, q):
    return int(np.quantile(score.astype(np.int64), q))


def _check_p7(got_s, got_f, exp_s, exp_f, ids, what):
    bad = ids[(got_s[ids] != exp_s[ids]) | (got_f[ids] != exp_f[ids])]
    assert bad.size == 0, (f"{what}: {bad.size} P7 mismatches at ids {bad[:5]}: gpu "
                           f"{got_s[bad[:5]]}/{got_f[bad[:5]]} oracle {exp_s[bad[:5]]}")


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("M,q", [(40, 0.9), (200, 0.8), (700, 0.95)])
def test_pipeline_end_to_end(hm, filt, M, q):
    e, t, res, off = _case(900 + M, M, 3000, 0, 900)
    fs_o, ff_o = oracle.score_db(filt, oq.quantize(e, synth.BG), res, off)
    thr = _survivor_threshold(fs_o, q)
    db = hm.Database(res, off)
    prof = hm.Profile.from_emissions(e, synth.BG)
    p7 = hm.P7Profile.from_probabilities(e, t, synth.BG)
    print(f"case pipeline {filt} M={M} thr={thr}", flush=True)
    out = hm.pipeline(filt, prof, p7, db, thr)
    torch.cuda.synchronize()
    fs, ff = out.filter_score.cpu().numpy(), out.filter_flags.cpu().numpy()
    assert np.array_equal(fs, fs_o) and np.array_equal(ff, ff_o)
    order = db.order()
    exp_pos = _expected_positions(order, fs_o, ff_o, thr)
    cnt = int(out.count.cpu()[0])
    assert cnt == exp_pos.size and 0 < cnt < db.nseq
    assert np.array_equal(out.positions.cpu().numpy()[:cnt], exp_pos)
    ids = order[exp_pos]
    ps_o, pf_o = oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off, ids=ids)
    ps, pf = out.p7_score.cpu().numpy(), out.p7_flags.cpu().numpy()
    _check_p7(ps, pf, ps_o, pf_o, ids, f"{filt} M={M}")
    rest = np.setdiff1d(np.arange(db.nseq), ids)
    assert (ps[rest] == -32768).all() and (pf[rest] == 0).all()
    db.close()


@pytest.mark.parametrize("filt", ["msv", "ssv"])
def test_select_threshold_extremes(hm, filt):
    """Nothing passes but the overflowed sequences, everything passes, and a
    threshold between: the positions follow the definition exactly."""
    M = 60
    e, t, res, off = _case(950, M, 2500, 0, 600, frac=0.2)
    prof = hm.Profile.from_emissions(e, synth.BG)
    db = hm.Database(res, off)
    fn = hm.msv_score if filt == "msv" else hm.ssv_score
    s, f = fn(prof, db)
    torch.cuda.synchronize()
    sn, fn_ = s.cpu().numpy(), f.cpu().numpy()
    order = db.order()
    lo, hi = (0, 256) if filt == "msv" else (-128, 128)
    for thr in (lo, hi, _survivor_threshold(sn, 0.5), 10**6, -10**6):
        print(f"case select {filt} thr={thr}", flush=True)
        pos, cnt = hm.select(db, s, f, filt, thr)
        torch.cuda.synchronize()
        exp = _expected_positions(order, sn, fn_, thr)
        c = int(cnt.cpu()[0])
        assert c == exp.size, (thr, c, exp.size)
        assert np.array_equal(pos.cpu().numpy()[:c], exp)
    db.close()


def test_select_more_than_a_million_records(hm):
    """More than 1024 blocks of 1024 positions: the one-block scan runs in
    chunks with a carry.  Scores and flags are seeded arrays on the device
    (the selection reads nothing else of them)."""
    n = 1024 * 1024 + 5000
    rng = np.random.default_rng(960)
    L = rng.integers(0, 4, size=n).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    db = hm.Database(res, off)
    sc = rng.integers(0, 256, size=n).astype(np.uint8)
    fl = (rng.random(n) < 0.01).astype(np.uint8)
    s = torch.from_numpy(sc).cuda()
    f = torch.from_numpy(fl).cuda()
    order = db.order()
    for thr in (250, 128):
        print(f"case select 1M thr={thr}", flush=True)
        pos, cnt = hm.select(db, s, f, "msv", thr)
        torch.cuda.synchronize()
        exp = _expected_positions(order, sc, fl, thr)
        c = int(cnt.cpu()[0])
        assert c == exp.size
        assert np.array_equal(pos.cpu().numpy()[:c], exp)
    db.close()


def test_p7_selected_arbitrary_subsets(hm):
    """Positions in any order (each once), an empty selection, and explicit
    plans including 16-wave blocks: the selected records score as the
    oracle's, every other entry keeps the caller's value."""
    M = 300
    e, t, res, off = _case(970, M, 2000, 0, 700, frac=0.3)
    db = hm.Database(res, off)
    p7 = hm.P7Profile.from_probabilities(e, t, synth.BG)
    order = db.order()
    rng = np.random.default_rng(971)
    sub = rng.permutation(db.nseq)[: 333].astype(np.int32)
    ids = order[sub]
    ps_o, pf_o = oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off, ids=ids)
    # the binding asks for room for nseq positions (the count is on the device)
    buf = np.zeros(db.nseq, np.int32)
    buf[: sub.size] = sub
    pos = torch.from_numpy(buf).cuda()
    plans = (None, hm.make_plan(16, 10), hm.make_plan(64, 3, 16), hm.make_plan(64, 3, 16, 2))
    for plan in plans:
        for n_take in (sub.size, 0, 1):
            print(f"case p7 selected plan={plan and plan.as_tuple()} n={n_take}", flush=True)
            cnt = torch.tensor([n_take], dtype=torch.int32, device="cuda")
            s = torch.full((db.nseq,), 12345, dtype=torch.int16, device="cuda")
            f = torch.full((db.nseq,), 7, dtype=torch.uint8, device="cuda")
            hm.p7_score_selected(p7, db, pos, cnt, s, f, plan=plan)
            torch.cuda.synchronize()
            sn, fn_ = s.cpu().numpy(), f.cpu().numpy()
            took = ids[:n_take]
            _check_p7(sn, fn_, ps_o, pf_o, took, f"plan={plan and plan.as_tuple()}")
            rest = np.setdiff1d(np.arange(db.nseq), took)
            assert (sn[rest] == 12345).all() and (fn_[rest] == 7).all()
    db.close()


@pytest.mark.parametrize("filt", ["msv", "ssv"])
def test_pipeline_edge_databases(hm, filt):
    """An empty database, one empty sequence, one sequence, and a database
    of empty sequences only: the survivors follow the definition (at a
    threshold everything passes, and at one nothing but overflow passes) and
    their P7 scores equal the oracle's."""
    M = 40
    rng = np.random.default_rng(990)
    e = synth.sample_emissions(rng, M)
    t = synth.sample_transitions(rng, M)
    one, off1 = synth.sample_residues(rng, np.array([300], np.int64))
    synth.implant_gapped(rng, one, off1, e, t, 1.0)
    cases = {"no sequences": (np.zeros(0, np.uint8), np.zeros(1, np.int64)),
             "one empty": (np.zeros(0, np.uint8), np.zeros(2, np.int64)),
             "one": (one, off1),
             "all empty": (np.zeros(0, np.uint8), np.zeros(101, np.int64))}
    prof = hm.Profile.from_emissions(e, synth.BG)
    p7 = hm.P7Profile.from_probabilities(e, t, synth.BG)
    lo, hi = (0, 256) if filt == "msv" else (-128, 128)
    for name, (res, off) in cases.items():
        db = hm.Database(res, off)
        n = db.nseq
        fs_o, ff_o = oracle.score_db(filt, oq.quantize(e, synth.BG), res, off)
        for thr in (lo, hi):
            print(f"case pipeline edge {filt} {name} thr={thr}", flush=True)
            out = hm.pipeline(filt, prof, p7, db, thr)
            torch.cuda.synchronize()
            assert np.array_equal(out.filter_score.cpu().numpy(), fs_o)
            order = db.order()
            exp = _expected_positions(order, fs_o, ff_o, thr)
            c = int(out.count.cpu()[0])
            assert c == exp.size and np.array_equal(out.positions.cpu().numpy()[:c], exp)
            ids = order[exp]
            ps_o, pf_o = oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off, ids=ids)
            _check_p7(out.p7_score.cpu().numpy(), out.p7_flags.cpu().numpy(), ps_o, pf_o, ids,
                      f"{filt} {name}")
            if thr == lo:
                assert c == n
        db.close()


@pytest.mark.parametrize("filt,M", [("msv", 300), ("ssv", 300), ("msv", 2000)])
def test_pipeline_degenerate_codes(hm, filt, M):
    """Databases holding the degenerate codes 21..26 (27-row tables in every
    stage, and at M = 2000 the selected call's 64-lane P7 image of 34 rows):
    survivors and their P7 scores against the oracle."""
    e, t, res, off = _case(1000 + M, M, 1500, 0, 600, frac=0.2)
    rng = np.random.default_rng(1001 + M)
    deg = rng.random(res.size) < 0.03
    res[deg] = rng.integers(21, 27, size=int(deg.sum())).astype(np.uint8)
    fs_o, ff_o = oracle.score_db(filt, oq.quantize(e, synth.BG), res, off)
    thr = _survivor_threshold(fs_o, 0.85)
    db = hm.Database(res, off)
    assert db.table_rows == 27
    prof = hm.Profile.from_emissions(e, synth.BG)
    p7 = hm.P7Profile.from_probabilities(e, t, synth.BG)
    print(f"case pipeline degenerate {filt} M={M} thr={thr}", flush=True)
    out = hm.pipeline(filt, prof, p7, db, thr)
    torch.cuda.synchronize()
    assert np.array_equal(out.filter_score.cpu().numpy(), fs_o)
    order = db.order()
    exp = _expected_positions(order, fs_o, ff_o, thr)
    c = int(out.count.cpu()[0])
    assert c == exp.size and c > 0 and np.array_equal(out.positions.cpu().numpy()[:c], exp)
    ids = order[exp]
    ps_o, pf_o = oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off, ids=ids)
    _check_p7(out.p7_score.cpu().numpy(), out.p7_flags.cpu().numpy(), ps_o, pf_o, ids,
              f"degenerate {filt} M={M}")
    db.close()
