"""Batched graph launches: every query's results equal its plain launch and the oracle."""
import numpy as np
import pytest

import oracle
from oracle import quant as oq
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as m
    import paper_1707_09683_amd.batch  # noqa: F401
    return m


@pytest.fixture(scope="module")
def setup(hm):
    rng = np.random.default_rng(404)
    Ms = [30, 48, 100, 257, 400, 700, 1000, 2400, 64, 3000]
    filt = ["msv", "ssv"] * 5
    emis = [synth.sample_emissions(rng, M) for M in Ms]
    db = synth.random_db(rng, 1500, 0, 900)
    synth.implant(rng, db.res, db.offsets, emis, 0.1)
    gdb = hm.Database(db.res, db.offsets)
    profs = [hm.Profile.from_emissions(e, synth.BG) for e in emis]
    yield Ms, filt, emis, db, gdb, profs
    gdb.close()


@pytest.mark.parametrize("branches", [1, 4])
def test_batch_matches_plain_and_oracle(hm, setup, branches):
    Ms, filt, emis, db, gdb, profs = setup
    print(f"case batch branches={branches}", flush=True)
    b = hm.batch.Batch(list(zip(filt, profs)), gdb, branches=branches)
    b.launch()
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(zip(filt, profs)):
        fn = hm.msv_score if f == "msv" else hm.ssv_score
        s, fl = fn(p, gdb, plan=b.plans[i])
        torch.cuda.synchronize()
        assert torch.equal(s, b.scores[i]) and torch.equal(fl, b.flags[i]), (i, Ms[i], f)
        es, ef = oracle.score_db(f, oq.quantize(emis[i], synth.BG), db.res, db.offsets)
        assert np.array_equal(b.scores[i].cpu().numpy(), es), (i, Ms[i], f)
        assert np.array_equal(b.flags[i].cpu().numpy(), ef), (i, Ms[i], f)
    b.close()


def test_batch_replays_with_eager_work_between(hm, setup):
    Ms, filt, emis, db, gdb, profs = setup
    b = hm.batch.Batch(list(zip(filt, profs)), gdb, branches=3)
    b.launch()
    torch.cuda.synchronize()
    ref = [(s.clone(), f.clone()) for s, f in zip(b.scores, b.flags)]
    for rep in range(3):
        for s in b.scores:
            s.zero_()
        # eager work on the default stream between replays
        hm.msv_score(profs[0], gdb)
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for i in range(len(ref)):
            assert torch.equal(b.scores[i], ref[i][0]) and torch.equal(b.flags[i], ref[i][1]), \
                (rep, i)
    b.close()


def test_batch_rejects_shared_workspace(hm, setup):
    import ctypes
    Ms, filt, emis, db, gdb, profs = setup
    b = hm.batch.Batch(list(zip(filt[:2], profs[:2])), gdb)
    arr = b._arr
    arr[1].workspace = arr[0].workspace
    h = ctypes.c_void_p()
    rc = hm._lib.hmsv_batch_create(arr, 2, gdb._h, 2, ctypes.byref(h))
    assert rc == -1 and not h.value
    b.close()
