"""Served path: every request's result is the same alone and in the mix."""
import numpy as np
import pytest

import oracle
from oracle import quant as oq
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as hm
    import paper_1707_09683_amd.serve as sv
    rng = np.random.default_rng(505)
    db = synth.random_db(rng, 6000, 0, 700)
    gdb = hm.Database(db.res, db.offsets)
    yield hm, sv, rng, db, gdb
    gdb.close()


def _alone(hm, gdb, filt, emis):
    prof = hm.Profile.from_emissions(emis, synth.BG)
    fn = hm.msv_score if filt == "msv" else hm.ssv_score
    s, f = fn(prof, gdb)
    torch.cuda.synchronize()
    return s.cpu().numpy(), f.cpu().numpy()


@pytest.mark.parametrize("mode", ["served", "plain"])
def test_served_results_equal_alone(env, mode):
    hm, sv, rng, db, gdb = env
    n = 16
    Ms = rng.integers(30, 900, size=n)
    filt = ["msv" if i % 2 == 0 else "ssv" for i in range(n)]
    emis = [synth.sample_emissions(rng, int(m)) for m in Ms]
    arrivals = np.cumsum(rng.exponential(0.002, size=n)) - 0.002
    if mode == "served":
        srv = sv.Server(gdb, synth.BG, max_inflight=4, depth=3, chunk_cells=2e8)
    else:
        srv = sv.Server(gdb, synth.BG, max_inflight=1, depth=1, chunk_cells=float("inf"))
    print(f"case serve {mode}", flush=True)
    reqs, span = sv.replay(srv, arrivals, filt, emis)
    srv.close()
    assert len(reqs) == n
    for i, r in enumerate(reqs):
        got = r.future.result()
        exp = _alone(hm, gdb, filt[i], emis[i])
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1]), (i, Ms[i])
        if mode == "served":
            assert len(r.chunks) >= 1
    if mode == "served":
        assert max(len(r.chunks) for r in reqs) > 1      # chunking exercised
    # a few against the oracle
    for i in (0, 1):
        es, ef = oracle.score_db(filt[i], oq.quantize(emis[i], synth.BG), db.res, db.offsets)
        got = reqs[i].future.result()
        assert np.array_equal(got[0], es) and np.array_equal(got[1], ef)
    st = sv.latency_stats(reqs)
    assert st["n"] == n and st["p99_ms"] >= st["p50_ms"] > 0


def test_range_calls_cover_database(env):
    """Scoring the processing order in pieces equals one full call."""
    hm, sv, rng, db, gdb = env
    emis = synth.sample_emissions(rng, 300)
    prof = hm.Profile.from_emissions(emis, synth.BG)
    full = hm.msv_score(prof, gdb)
    s = torch.zeros(gdb.nseq, dtype=torch.uint8, device="cuda")
    f = torch.zeros(gdb.nseq, dtype=torch.uint8, device="cuda")
    ws = hm.new_workspace(nseq=gdb.nseq)
    edges = [0, 1, 17, 1000, 3333, gdb.nseq]
    for a, b in zip(edges[:-1], edges[1:]):
        hm.score_range("msv", prof, gdb, a, b - a, s, f, ws)
    torch.cuda.synchronize()
    assert torch.equal(s, full[0]) and torch.equal(f, full[1])
    order = gdb.order()
    assert sorted(order.tolist()) == list(range(gdb.nseq))
    L = db.lengths[order]
    assert (np.diff(L) <= 0).all()


@pytest.mark.parametrize("filt", ["msv", "ssv"])
def test_range_calls_split_long_sequences(env, filt):
    """Ranges whose longest sequences are split into segments (a database
    with 8,000..20,000-residue sequences among short ones, M = 48): every
    range's results equal the oracle's, and the first range does split."""
    hm, sv, rng, _db, _gdb = env
    r = np.random.default_rng(77)
    emis = synth.sample_emissions(r, 48)
    long_db = synth.random_db(r, 6, 8000, 20000)
    short_db = synth.random_db(r, 3000, 20, 300)
    db = synth.Database(np.concatenate([long_db.res, short_db.res]),
                        np.concatenate([long_db.offsets,
                                        short_db.offsets[1:] + long_db.offsets[-1]]))
    synth.implant(r, db.res, db.offsets, [emis], 0.2)
    gdb = hm.Database(db.res, db.offsets)
    prof = hm.Profile.from_emissions(emis, synth.BG)
    sdt = torch.uint8 if filt == "msv" else torch.int8
    s = torch.zeros(gdb.nseq, dtype=sdt, device="cuda")
    f = torch.zeros(gdb.nseq, dtype=torch.uint8, device="cuda")
    ws = hm.new_workspace(nseq=gdb.nseq)
    edges = [0, 200, 1500, gdb.nseq]
    plan = hm.plan_for(filt, 48)
    assert hm.split_info(filt, 48, gdb, plan, 0, 200)[0] > 0
    print(f"case range split {filt}", flush=True)
    for a, b in zip(edges[:-1], edges[1:]):
        hm.score_range(filt, prof, gdb, a, b - a, s, f, ws, plan)
    torch.cuda.synchronize()
    es, ef = oracle.score_db(filt, oq.quantize(emis, synth.BG), db.res, db.offsets)
    gs = s.cpu().numpy().view(np.uint8 if filt == "msv" else np.int8)
    assert np.array_equal(gs, es.view(gs.dtype)) and np.array_equal(f.cpu().numpy(), ef)
    gdb.close()
