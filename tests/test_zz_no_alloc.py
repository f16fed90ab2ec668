"""The allocation-free MSV entry point (hmsv_msv_score_noalloc, workspace in
the library's own device array) against hmsv_msv_score with a caller's
workspace: bit-identical scores and flags on two calls in a row, the second
on a smaller database, both also equal to the oracle."""
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
    return m


def _db(rng, emis, n, lo, hi, frac):
    """Random sequences, a fraction with a long segment emitted by the
    profile (overflow) and as many with short ones (5..12 residues: the J
    state opens without overflow, so the exact pass runs)."""
    db = synth.random_db(rng, n, lo, hi)
    synth.implant(rng, db.res, db.offsets, [emis], frac)
    M = emis.shape[0]
    p = emis / emis.sum(axis=1, keepdims=True)
    for i in np.flatnonzero(rng.random(db.n) < frac):
        a, b = int(db.offsets[i]), int(db.offsets[i + 1])
        ln = int(min(rng.integers(5, 13), M, b - a))
        if ln < 1:
            continue
        k0 = int(rng.integers(0, M - ln + 1))
        at = a + int(rng.integers(0, b - a - ln + 1))
        for t in range(ln):
            db.res[at + t] = rng.choice(20, p=p[k0 + t])
    return db


@pytest.mark.parametrize("M", [48, 400])
def test_noalloc_equals_workspace_call(hm, M):
    rng = np.random.default_rng(4100 + M)
    emis = synth.sample_emissions(rng, M)
    prof = hm.Profile.from_emissions(emis, synth.BG)
    oprof = oq.quantize(emis, synth.BG)
    # a larger database (long sequences that get split, many rescoring
    # windows), then a smaller one: the second call reuses the array
    dbs = [_db(rng, emis, 6000, 1, 9000, 0.3), _db(rng, emis, 700, 0, 300, 0.3)]
    for k, db in enumerate(dbs):
        print(f"case noalloc M={M} call {k + 1}: {db.n} sequences", flush=True)
        gdb = hm.Database(db.res, db.offsets)
        s1, f1 = hm.msv_score(prof, gdb)
        s2 = torch.full((db.n,), 0xAB, dtype=torch.uint8, device=prof.device)
        f2 = torch.full((db.n,), 0xCD, dtype=torch.uint8, device=prof.device)
        hm.msv_score_noalloc(prof, gdb, s2, f2)
        torch.cuda.synchronize()
        gdb.close()
        assert torch.equal(s1, s2) and torch.equal(f1, f2), f"call {k + 1}"
        es, ef = oracle.score_db("msv", oprof, db.res, db.offsets)
        assert np.array_equal(s2.cpu().numpy(), es) and np.array_equal(f2.cpu().numpy(), ef)
        assert int(((es > 190) & (ef == 0)).sum()) > 10      # rescoring windows occurred


def test_noalloc_rejects_databases_above_its_limit(hm):
    n = hm.NOALLOC_MAX_SEQ + 1
    offsets = np.arange(n + 1, dtype=np.int64)
    res = np.zeros(n, dtype=np.uint8)
    gdb = hm.Database(res, offsets)
    prof = hm.Profile.from_emissions(synth.sample_emissions(np.random.default_rng(1), 20),
                                     synth.BG)
    s = torch.zeros(n, dtype=torch.uint8, device=prof.device)
    f = torch.zeros(n, dtype=torch.uint8, device=prof.device)
    with pytest.raises(hm.HmsvError) as e:
        hm.msv_score_noalloc(prof, gdb, s, f)
    assert e.value.status == -2
    gdb.close()
