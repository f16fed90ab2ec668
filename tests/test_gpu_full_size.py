"""GPU parity at the benchmark's full sizes, in the launch configuration the
bench times (tuned plans, persistent grids).

The oracle scores a sample of each output one sequence at a time: every
implanted sequence (hits, overflow), the 200 longest and 200 shortest, and
2,000 drawn at random.  Properties that hold at any size are checked on
every output (flags only with the sentinel score, SSV scores in range)."""
import numpy as np
import pytest

import oracle
from oracle import quant as oq
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as m
    import paper_1707_09683_amd.batch  # noqa: F401
    return m


def _sample(db, implanted, seed, n_random=2000):
    L = np.asarray(db.lengths)
    order = np.argsort(L, kind="stable")
    rng = np.random.default_rng(seed)
    ids = np.concatenate([np.asarray(implanted, np.int64), order[:200], order[-200:],
                          rng.choice(db.n, n_random, replace=False)])
    return np.unique(ids)


def _check(filt, emis, db, ids, gs, gf, what):
    es, ef = oracle.score_db(filt, oq.quantize(emis, synth.BG), db.res, db.offsets, ids=ids)
    bad = ids[(gs[ids] != es[ids]) | (gf[ids] != ef[ids])]
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first {bad[:5]}"
    sentinel = 255 if filt == "msv" else 127
    sv = gs.view(np.int8) if filt == "ssv" else gs
    assert np.all(sv[gf == 1] == sentinel), what
    return int(ef[ids].sum())


@pytest.fixture(scope="module")
def cfg12(hm):
    w = synth.plain_msv_m400()
    gdb = hm.Database(w.db.res, w.db.offsets)
    yield w, gdb
    gdb.close()


def test_msv_m400_500k(hm, cfg12):
    w, gdb = cfg12
    emis = w.emissions[0]
    print("case full msv m400 500k", flush=True)
    prof = hm.Profile.from_emissions(emis, synth.BG)
    s, f = hm.msv_score(prof, gdb, plan=hm.plan_for("msv", 400))
    torch.cuda.synchronize()
    gs, gf = s.cpu().numpy(), f.cpu().numpy()
    ids = _sample(w.db, w.implanted, 11)
    ovf = _check("msv", emis, w.db, ids, gs, gf, "msv m400")
    assert ovf > 0
    assert int(gf.sum()) >= len(w.implanted) // 2          # most implants overflow


@pytest.mark.parametrize("M", [30, 40])
def test_short_profiles_500k_many_segments(hm, M):
    """Short profiles on a 500k lognormal database with 2% implants: the
    tuned plans run one sequence per lane, so the call cuts thousands of
    sequences into segments (as many as a call allows); every sequence of
    both filters against the oracle."""
    st = synth.streams(30 + M)
    emis = synth.sample_emissions(st["profile"], M)
    db, imp = synth.lognormal_db(30 + M, 500_000, [emis], 0.02, st)
    gdb = hm.Database(db.res, db.offsets)
    try:
        for filt in ("msv", "ssv"):
            plan = hm.plan_for(filt, M)
            ns, nseg, T = hm.split_info(filt, M, gdb, plan)
            print(f"case short {filt} M={M} plan={plan.as_tuple()} split={ns} segs={nseg} "
                  f"T={T}", flush=True)
            assert ns > 1000 and nseg > ns
            prof = hm.Profile.from_emissions(emis, synth.BG)
            fn = hm.msv_score if filt == "msv" else hm.ssv_score
            s, f = fn(prof, gdb, plan=plan)
            torch.cuda.synchronize()
            gs, gf = s.cpu().numpy(), f.cpu().numpy()
            es, ef = oracle.score_db(filt, oq.quantize(emis, synth.BG), db.res, db.offsets)
            bad = np.nonzero((gs != es) | (gf != ef))[0]
            assert bad.size == 0, (f"{filt} M={M}: {bad.size} mismatches, first {bad[:5]}: "
                                   f"gpu {gs[bad[:5]]} oracle {es[bad[:5]]}")
            assert (es[imp] > np.median(es)).mean() > 0.5      # the implants score high
    finally:
        gdb.close()


@pytest.mark.parametrize("M", [100, 400, 1000, 2400])
def test_ssv_500k(hm, cfg12, M):
    w, gdb = cfg12
    ws = synth.plain_ssv(db=w.db, implanted=w.implanted)
    emis = ws.emissions[[100, 400, 1000, 2400].index(M)]
    print(f"case full ssv m{M} 500k", flush=True)
    prof = hm.Profile.from_emissions(emis, synth.BG)
    s, f = hm.ssv_score(prof, gdb, plan=hm.plan_for("ssv", M))
    torch.cuda.synchronize()
    gs, gf = s.cpu().numpy(), f.cpu().numpy()
    _check("ssv", emis, w.db, _sample(w.db, w.implanted, 12 + M), gs, gf, f"ssv m{M}")


def test_batched_64_queries_1m(hm):
    w = synth.batched()
    gdb = hm.Database(w.db.res, w.db.offsets)
    profs = [hm.Profile.from_emissions(e, synth.BG) for e in w.emissions]
    print("case full batched 64q 1m", flush=True)
    b = hm.batch.Batch(list(zip(w.filters, profs)), gdb, branches=4)
    b.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    L = np.asarray(w.db.lengths)
    longest = np.argsort(L)[-20:]
    for i, (filt, emis) in enumerate(zip(w.filters, w.emissions)):
        ids = np.unique(np.concatenate([rng.choice(w.db.n, 100, replace=False), longest,
                                        rng.choice(w.implanted, 20, replace=False)]))
        gs, gf = b.scores[i].cpu().numpy(), b.flags[i].cpu().numpy()
        _check(filt, emis, w.db, ids, gs, gf, f"batched query {i} M={emis.shape[0]}")
    b.close()
    gdb.close()
