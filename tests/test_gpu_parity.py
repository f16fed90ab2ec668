"""GPU parity: every sequence's score and overflow flag, bit for bit, against the oracle.

Both sides quantize the same float64 emissions independently (the library
in C++, the oracle in numpy) and score the same seeded databases."""
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


def _gpu(hm, filt, emis, db, plan=None):
    prof = hm.Profile.from_emissions(emis, synth.BG)
    gdb = hm.Database(db.res, db.offsets)
    fn = hm.msv_score if filt == "msv" else hm.ssv_score
    s, f = fn(prof, gdb, plan=plan)
    torch.cuda.synchronize()
    out = s.cpu().numpy(), f.cpu().numpy()
    gdb.close()
    return out


def _oracle(filt, emis, db, ids=None):
    prof = oq.quantize(emis, synth.BG)
    return oracle.score_db(filt, prof, db.res, db.offsets, ids=ids)


def _assert_same(got, exp, ids=None, what=""):
    gs, gf = got
    es, ef = exp
    if ids is not None:
        gs, gf, es, ef = gs[ids], gf[ids], es[ids], ef[ids]
    bad = np.nonzero((gs != es) | (gf != ef))[0]
    assert bad.size == 0, (f"{what}: {bad.size} mismatches, first at {bad[:5]}: "
                           f"gpu {gs[bad[:5]]}/{gf[bad[:5]]} oracle {es[bad[:5]]}/{ef[bad[:5]]}")


@pytest.fixture(scope="module")
def cfg0():
    return synth.plain_msv_m48()


@pytest.mark.parametrize("filt", ["msv", "ssv"])
def test_m48_2k_default_plan(hm, cfg0, filt):
    emis = cfg0.emissions[0]
    print(f"case m48_2k {filt}", flush=True)
    _assert_same(_gpu(hm, filt, emis, cfg0.db), _oracle(filt, emis, cfg0.db), what=filt)


PLANS_M48 = [(1, 25), (1, 32), (2, 13), (2, 14), (4, 7), (4, 8), (8, 4), (8, 5), (16, 2), (32, 1), (64, 1)]


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("gq", PLANS_M48, ids=lambda t: f"G{t[0]}Q{t[1]}")
def test_m48_every_group_width(hm, cfg0, filt, gq):
    emis = cfg0.emissions[0]
    G, Q = gq
    print(f"case m48 {filt} G={G} Q={Q}", flush=True)
    plan = hm.make_plan(G, Q, waves_per_block=2, blocks=0)
    _assert_same(_gpu(hm, filt, emis, cfg0.db, plan), _oracle(filt, emis, cfg0.db),
                 what=f"{filt} G{G} Q{Q}")


def _implanted_db(rng, emis, n, lo, hi, frac):
    db = synth.random_db(rng, n, lo, hi)
    synth.implant(rng, db.res, db.offsets, [emis], frac)
    return db


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("M", [1, 2, 17, 100, 257, 400, 1000, 2400, 3839])
def test_lengths_and_implants(hm, filt, M):
    """Ragged lengths (0..700, one code of 20..31 sprinkled), 10% implants from the
    query so overflow and the J loop occur, across profile lengths."""
    rng = np.random.default_rng(1000 + M)
    emis = synth.sample_emissions(rng, M)
    n = 600 if M < 1000 else 250
    db = _implanted_db(rng, emis, n, 0, 700, 0.1)
    code = int(rng.integers(20, 32))
    if M >= 2560 and 21 <= code <= 26:
        code = 27              # a degenerate code's 27-row image would not fit the LDS
    db.res[rng.random(db.res.size) < 0.002] = code
    print(f"case lengths {filt} M={M} n={n} code={code}", flush=True)
    got = _gpu(hm, filt, emis, db)
    exp = _oracle(filt, emis, db)
    _assert_same(got, exp, what=f"{filt} M={M}")
    if M >= (17 if filt == "msv" else 100):
        assert exp[1].sum() > 0          # overflow path exercised


@pytest.mark.parametrize("M", [40, 130, 700])
def test_msv_exact_replay_of_j_state_sequences(hm, M):
    """A sequence first runs with scB fixed; one whose maximum lands between
    base + tec and the overflow threshold is replayed in exact mode (scB
    updated where the running max moves it).  Short implants make such
    sequences common; their scores exceed base = 190."""
    rng = np.random.default_rng(77 + M)
    emis = synth.sample_emissions(rng, M)
    db = synth.random_db(rng, 1500, 1, 400)
    synth.implant(rng, db.res, db.offsets, [emis], 0.3)
    print(f"case msv exact replay M={M}", flush=True)
    exp = _oracle("msv", emis, db)
    _assert_same(_gpu(hm, "msv", emis, db), exp, what=f"M={M}")
    j_state = int(((exp[0] > 190) & (exp[1] == 0)).sum())
    assert j_state > 5, j_state


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("M", [48, 400])
def test_long_sequences(hm, filt, M):
    """Sequences of 1500..6000 residues, on both sides of the length above
    which MSV runs exact from the start, with implants (hits, J loop,
    overflow) placed anywhere along them."""
    rng = np.random.default_rng(300 + M)
    emis = synth.sample_emissions(rng, M)
    db = _implanted_db(rng, emis, 300, 1500, 6000, 0.1)
    _short_implants(rng, emis, db, 0.4)
    print(f"case long {filt} M={M}", flush=True)
    exp = _oracle(filt, emis, db)
    _assert_same(_gpu(hm, filt, emis, db), exp, what=f"long {filt} M={M}")
    if filt == "msv":
        assert int(((exp[0] > 190) & (exp[1] == 0)).sum()) > 5
        assert exp[1].sum() > 0


@pytest.mark.parametrize("M,G", [(40, 2), (40, 16), (200, 4), (200, 8)])
def test_msv_mostly_rescored(hm, M, G):
    """Short implants in 90% of 2,000 sequences of 50..3,000 residues: about
    a third of them open the J state without overflowing and are rescored
    in exact mode (many per wavefront at once), half overflow."""
    rng = np.random.default_rng(900 + M)
    emis = synth.sample_emissions(rng, M)
    db = synth.random_db(rng, 2000, 50, 3000)
    _short_implants(rng, emis, db, 0.9)
    Q = -(-(M + 1) // (2 * G))
    print(f"case msv mostly rescored M={M} G={G}", flush=True)
    exp = _oracle("msv", emis, db)
    _assert_same(_gpu(hm, "msv", emis, db, hm.make_plan(G, Q, 4, 0)), exp,
                 what=f"M={M} G={G}")
    assert int(((exp[0] > 190) & (exp[1] == 0)).sum()) > 400
    assert int(exp[1].sum()) > 400


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("M,G", [(16, 2), (48, 4), (130, 16), (400, 8)])
def test_split_sequences(hm, filt, M, G):
    """Twelve sequences of 6,000..30,000 residues among 4,000 of 20..200:
    the long ones are cut into segments scored in parallel (checked with
    split_info), with implants (hits, J loop, overflow) anywhere along them,
    so segment boundaries cross hits and MSV rescoring of a split sequence
    occurs."""
    rng = np.random.default_rng(500 + M)
    emis = synth.sample_emissions(rng, M)
    long_db = _implanted_db(rng, emis, 12, 6000, 30000, 0.5)
    _short_implants(rng, emis, long_db, 1.0)
    short_db = _implanted_db(rng, emis, 4000, 20, 200, 0.05)
    db = synth.Database(np.concatenate([long_db.res, short_db.res]),
                        np.concatenate([long_db.offsets,
                                        short_db.offsets[1:] + long_db.offsets[-1]]))
    Q = -(-(M + 1) // (2 * G))
    plan = hm.make_plan(G, Q, 4, 0)
    gdb = hm.Database(db.res, db.offsets)
    ns, nseg, T = hm.split_info(filt, M, gdb, plan)
    gdb.close()
    print(f"case split {filt} M={M} G={G} Q={Q}: {ns} split into {nseg} x {T}", flush=True)
    assert ns == 12 and nseg > 24, (ns, nseg, T)
    exp = _oracle(filt, emis, db)
    _assert_same(_gpu(hm, filt, emis, db, plan), exp, what=f"split {filt} M={M}")
    if filt == "msv" and M >= 48:
        assert exp[1][:12].sum() > 0                              # an overflow among them
        assert int(((exp[0][:12] > 190) & (exp[1][:12] == 0)).sum()) > 0   # rescored


def _short_implants(rng, emis, db, frac):
    """Overwrite 1..3 segments of 5..12 residues emitted by consecutive
    nodes of the profile into a fraction of the sequences: scores that open
    the J loop without overflowing."""
    M = emis.shape[0]
    p = emis / emis.sum(axis=1, keepdims=True)
    for i in np.flatnonzero(rng.random(db.n) < frac):
        a, b = int(db.offsets[i]), int(db.offsets[i + 1])
        for _ in range(int(rng.integers(1, 4))):
            ln = int(min(rng.integers(5, 13), M, b - a))
            k0 = int(rng.integers(0, M - ln + 1))
            at = a + int(rng.integers(0, b - a - ln + 1))
            for t in range(ln):
                db.res[at + t] = rng.choice(20, p=p[k0 + t])


@pytest.mark.parametrize("filt", ["msv", "ssv"])
def test_edge_sequences(hm, filt):
    """Empty, all-invalid, single-residue, long (5000) sequences and
    single-sequence and sub-group-count databases."""
    rng = np.random.default_rng(5)
    emis = synth.sample_emissions(rng, 64)
    seqs = [np.zeros(0, np.uint8), np.full(9, 20, np.uint8), np.full(3, 31, np.uint8),
            np.array([3], np.uint8), rng.integers(0, 20, 5000).astype(np.uint8),
            rng.integers(0, 20, 4).astype(np.uint8), rng.integers(0, 20, 5).astype(np.uint8)]
    lens = np.array([len(s) for s in seqs])
    off = np.zeros(len(seqs) + 1, np.int64)
    off[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(seqs), off)
    print(f"case edges {filt}", flush=True)
    _assert_same(_gpu(hm, filt, emis, db), _oracle(filt, emis, db), what="edges")
    one = db.subset([4])
    _assert_same(_gpu(hm, filt, emis, one), _oracle(filt, emis, one), what="single")


def test_repeated_calls_share_workspace(hm, cfg0):
    emis = cfg0.emissions[0]
    prof = hm.Profile.from_emissions(emis, synth.BG)
    gdb = hm.Database(cfg0.db.res, cfg0.db.offsets)
    ws = hm.new_workspace(nseq=gdb.nseq)
    outs = []
    for _ in range(3):
        s, f = hm.msv_score(prof, gdb, workspace=ws)
        outs.append((s.clone(), f.clone()))
    torch.cuda.synchronize()
    for s, f in outs[1:]:
        assert torch.equal(s, outs[0][0]) and torch.equal(f, outs[0][1])
    gdb.close()


@pytest.mark.parametrize("M", [30, 48, 130, 700])
def test_msv_windows_at_sequence_edges(hm, M):
    """Rescoring windows that start at a sequence's first row (a hit within
    M rows of the start), end at its last row, or span two hits far apart,
    for every group width of the first pass; the exact pass takes 64-lane
    groups of 1, 1, 2 and 6 registers at these lengths."""
    rng = np.random.default_rng(1300 + M)
    emis = synth.sample_emissions(rng, M)
    db = synth.random_db(rng, 1200, 40, 2500)
    p = emis / emis.sum(axis=1, keepdims=True)
    for i in range(db.n):
        a, b = int(db.offsets[i]), int(db.offsets[i + 1])
        ln = int(min(10, M, b - a))
        k0 = int(rng.integers(0, M - ln + 1))
        where = [a, b - ln, a + (b - a - ln) // 2][i % 3:i % 3 + 1]
        if i % 4 == 3:
            where = [a + 3, b - ln - 2]                     # two hits far apart
        for at in where:
            for t in range(ln):
                db.res[at + t] = rng.choice(20, p=p[k0 + t])
    exp = _oracle("msv", emis, db)
    assert int(((exp[0] > 190) & (exp[1] == 0)).sum()) > 100
    for G in (1, 2, 4, 8, 16, 32, 64):
        Q = -(-(M + 1) // (2 * G))
        if Q > 32 or hm.plan_lds_bytes(G, Q) > 160 * 1024:
            continue
        print(f"case msv windows M={M} G={G} Q={Q}", flush=True)
        _assert_same(_gpu(hm, "msv", emis, db, hm.make_plan(G, Q, 4, 0)), exp,
                     what=f"M={M} G={G}")
