"""GPU parity for profiles given directly as cost tables, across the whole
accepted dbias range (0..64), against the oracle, every sequence.

Profiles quantized from Dirichlet(0.5 bg) emissions keep dbias near 20;
the library accepts up to 64.  Here the tables are drawn directly
(``synth.random_cost_table``): costs of 0 and 255 inside the scoring
residues, a consensus residue per node, and runs of consensus residues
implanted so that sequences land on both sides of the J-state level
(base + tec) and of the overflow level (255 - dbias), including dbias 61..64
where overflow comes before the J state can open.  Rows 21..26 of each
table score the degenerate codes (B, J, Z, U, O, X), which the databases
of M < 2560 carry (their images hold 27 rows; M = 3839 only fits 21).  The
GPU copy of each table carries random bytes in rows 20 and 27..31, which
the kernels must ignore (those codes score as -inf); the oracle gets rows
of 255 there."""
import numpy as np
import pytest

import oracle
from oracle import quant as oq
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DBIAS = [0, 20, 40, 61, 62, 63, 64]
MS = [1, 48, 400, 3839]


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as m
    return m


def _plans(hm, M, rows):
    out = []
    for G in (1, 2, 4, 8, 16, 32, 64):
        Q = -(-(M + 1) // (2 * G))
        if Q <= 32 and 0 < hm.plan_lds_bytes(G, Q) * rows // 21 <= 160 * 1024:
            out.append((G, Q))
    return out


def _database(rng, cons, M):
    """Three parts: random sequences of ragged length with consensus runs
    implanted in 60% of them; "ladder" sequences of non-scoring code 20
    carrying 1..2 consensus runs each (their scores are exact sums of the
    runs' gains, so they land densely around the J-state and overflow
    levels); four long sequences with runs (cut into segments by the
    library).  About 0.3% of the random residues are one code of 20..31
    (above 2559 nodes a degenerate draw becomes 27), and for M < 2560 another
    0.5% are degenerate codes 21..26."""
    n, hi = (700, 500) if M < 1000 else (150, 400)
    db = synth.random_db(rng, n, 0, hi)
    synth.implant_consensus(rng, db.res, db.offsets, cons, 0.6, 40)
    code = int(rng.integers(20, 32))
    if M >= 2560 and 21 <= code <= 26:
        code = 27
    db.res[rng.random(db.res.size) < 0.003] = code
    if M < 2560:
        r3 = np.random.default_rng(11000 + M)
        d = r3.random(db.res.size) < 0.005
        db.res[d] = r3.integers(21, 27, size=int(d.sum()))
    lad = synth.random_db(rng, n, 1, hi)
    lad.res[:] = 20
    synth.implant_consensus(rng, lad.res, lad.offsets, cons, 1.0, 24, (1, 2))
    long_db = synth.random_db(rng, 4, 1500, 5000)
    synth.implant_consensus(rng, long_db.res, long_db.offsets, cons, 1.0, 40)
    parts = [db, lad, long_db]
    off, at = [np.zeros(1, np.int64)], 0
    for p in parts:
        off.append(p.offsets[1:] + at)
        at += int(p.offsets[-1])
    return synth.Database(np.concatenate([p.res for p in parts]), np.concatenate(off))


@pytest.mark.parametrize("M", MS)
@pytest.mark.parametrize("dbias", DBIAS)
def test_table_profiles_every_sequence(hm, dbias, M):
    rng = np.random.default_rng(7000 + 17 * dbias + M)
    cost, cons = synth.random_cost_table(rng, M, dbias)
    db = _database(rng, cons, M)
    # degenerate rows 21..26: costs of their own, read by both sides
    r2 = np.random.default_rng(9000 + 17 * dbias + M)
    cost[21:27] = np.clip(dbias + r2.integers(-3, 12, size=(6, M)), 0, 255)
    oprof = oq.from_costs(cost, dbias)
    # the library's copy: rows 20 and 27..31 hold random bytes it must not read
    g_cost = cost.copy()
    g_sc = np.maximum(-128, dbias - cost.astype(np.int64)).astype(np.int8)
    for rows in (slice(20, 21), slice(27, 32)):
        g_cost[rows] = rng.integers(0, 256, size=g_cost[rows].shape)
        g_sc[rows] = rng.integers(-128, 128, size=g_sc[rows].shape)
    prof = hm.Profile(torch.from_numpy(g_cost).cuda(), torch.from_numpy(g_sc).cuda(), dbias)
    gdb = hm.Database(db.res, db.offsets)
    assert gdb.table_rows == (27 if M < 2560 else 21)
    for filt in ("msv", "ssv"):
        es, ef = oracle.score_db(filt, oprof, db.res, db.offsets)
        fn = hm.msv_score if filt == "msv" else hm.ssv_score
        for G, Q in _plans(hm, M, gdb.table_rows):
            print(f"case tables {filt} dbias={dbias} M={M} G={G} Q={Q}", flush=True)
            s, f = fn(prof, gdb, plan=hm.make_plan(G, Q, 4, 0))
            torch.cuda.synchronize()
            gs, gf = s.cpu().numpy(), f.cpu().numpy()
            bad = np.flatnonzero((gs != es) | (gf != ef))
            assert bad.size == 0, (f"{filt} dbias={dbias} M={M} G={G}: {bad.size} mismatches, "
                                   f"first {bad[:5]} gpu {gs[bad[:5]]}/{gf[bad[:5]]} "
                                   f"oracle {es[bad[:5]]}/{ef[bad[:5]]}")
        if filt == "msv":
            # unflagged scores within 5 of the last value below overflow
            # (254 - dbias - tec for a single hit), and overflow itself
            top = 254 - dbias - 3
            near = int(((ef == 0) & (es.astype(int) >= top - 5)).sum())
            if dbias >= 20 and M > 1 or dbias >= 61:
                assert near > 0, (dbias, M)
            if dbias >= 20 and M > 1:
                assert ef.sum() > 0, (dbias, M)
            if 20 <= dbias <= 40 and M > 1:
                # J state opened without overflow (score above base)
                assert ((ef == 0) & (es.astype(int) > 190)).sum() > 0, (dbias, M)
        elif dbias >= 40 and M >= 400:
            assert ef.sum() > 0, (dbias, M)
    gdb.close()
