"""GPU parity with degenerate residue codes (21..26: B, J, Z, U, O, X) in
the database: MSV, SSV and P7Viterbi, bit for bit against the oracle.

A database that holds degenerate codes puts 27 table rows in the kernels'
LDS images instead of 21; every filter reads the profile's degenerate rows
(the background-weighted mean of the members' log-odds, written by each
side's own quantizer).  Codes 20 and 27..31 stay non-scoring."""
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
    import paper_1707_09683_amd.batch  # noqa: F401
    return m


def _sprinkle(rng, res, frac=0.05):
    """Replace a fraction of the residues by degenerate codes (and a fifth
    of that by non-scoring codes 20, 27..31)."""
    u = rng.random(res.size)
    d = u < frac
    res[d] = rng.integers(21, 27, size=int(d.sum())).astype(np.uint8)
    z = (u >= frac) & (u < 1.2 * frac)
    res[z] = rng.choice(np.array([20, 27, 28, 29, 30, 31], np.uint8), size=int(z.sum()))


def _short_implants(rng, emis, res, offsets, frac):
    M = emis.shape[0]
    p = emis / emis.sum(axis=1, keepdims=True)
    for i in np.flatnonzero(rng.random(len(offsets) - 1) < frac):
        a, b = int(offsets[i]), int(offsets[i + 1])
        if b - a < 5:
            continue
        ln = int(min(rng.integers(5, 13), M, b - a))
        k0 = int(rng.integers(0, M - ln + 1))
        at = a + int(rng.integers(0, b - a - ln + 1))
        for t in range(ln):
            res[at + t] = rng.choice(20, p=p[k0 + t])


def _db(seed, emis, nseq, lo, hi, frac=0.05):
    rng = np.random.default_rng(seed)
    L = rng.integers(lo, hi + 1, size=nseq).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    synth.implant(rng, res, off, [emis], 0.1)
    _short_implants(rng, emis, res, off, 0.3)
    _sprinkle(rng, res, frac)
    return res, off


def _check(got, exp, what):
    gs, gf = got
    es, ef = exp
    bad = np.nonzero((gs != es) | (gf != ef))[0]
    assert bad.size == 0, (f"{what}: {bad.size} mismatches, first at {bad[:5]}: "
                           f"gpu {gs[bad[:5]]}/{gf[bad[:5]]} oracle {es[bad[:5]]}/{ef[bad[:5]]}")


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("M,G", [(30, 1), (48, 2), (130, 4), (400, 8), (1000, 32), (2559, 64)])
def test_degenerate_codes_msv_ssv(hm, filt, M, G):
    rng = np.random.default_rng(1000 + M)
    emis = synth.sample_emissions(rng, M)
    res, off = _db(2000 + M, emis, 1200, 0, 900)
    gdb = hm.Database(res, off)
    assert gdb.table_rows == 27
    prof = hm.Profile.from_emissions(emis, synth.BG)
    Q = -(-(M + 1) // (2 * G))
    plans = [None, hm.make_plan(G, Q, 4, 0)]
    exp = oracle.score_db(filt, oq.quantize(emis, synth.BG), res, off)
    fn = hm.msv_score if filt == "msv" else hm.ssv_score
    for plan in plans:
        print(f"case degenerate {filt} M={M} plan={None if plan is None else plan.as_tuple()}",
              flush=True)
        s, f = fn(prof, gdb, plan=plan)
        torch.cuda.synchronize()
        _check((s.cpu().numpy(), f.cpu().numpy()), exp, f"{filt} M={M}")
    gdb.close()
    if filt == "msv" and M <= 400:
        assert int(((exp[0] > 190) & (exp[1] == 0)).sum()) > 5     # exact-pass rescoring


@pytest.mark.parametrize("filt", ["msv", "ssv"])
def test_degenerate_long_and_split(hm, filt):
    """Sequences of 6,000..20,000 residues among short ones, split into
    segments, with degenerate codes across segment boundaries."""
    M = 130
    rng = np.random.default_rng(77)
    emis = synth.sample_emissions(rng, M)
    res1, off1 = _db(78, emis, 10, 6000, 20000)
    res2, off2 = _db(79, emis, 3000, 20, 200)
    res = np.concatenate([res1, res2])
    off = np.concatenate([off1, off2[1:] + off1[-1]])
    gdb = hm.Database(res, off)
    plan = hm.make_plan(16, 5, 4, 0)
    ns, nseg, T = hm.split_info(filt, M, gdb, plan)
    print(f"case degenerate split {filt}: {ns} split into {nseg} x {T}", flush=True)
    assert ns == 10
    prof = hm.Profile.from_emissions(emis, synth.BG)
    fn = hm.msv_score if filt == "msv" else hm.ssv_score
    s, f = fn(prof, gdb, plan=plan)
    torch.cuda.synchronize()
    _check((s.cpu().numpy(), f.cpu().numpy()),
           oracle.score_db(filt, oq.quantize(emis, synth.BG), res, off), f"split {filt}")
    gdb.close()


@pytest.mark.parametrize("M", [5, 100, 400, 1000, 2000])
def test_degenerate_codes_p7(hm, M):
    rng = np.random.default_rng(3000 + M)
    e = synth.sample_emissions(rng, M)
    t = synth.sample_transitions(rng, M)
    res, off = _db(4000 + M, e, 1000, 0, 700)
    synth.implant_gapped(rng, res, off, e, t, 0.2)
    _sprinkle(rng, res, 0.04)
    gdb = hm.Database(res, off)
    assert gdb.table_rows == 27
    prof = hm.P7Profile.from_probabilities(e, t, synth.BG)
    print(f"case degenerate p7 M={M}", flush=True)
    s, f = hm.p7_score(prof, gdb)
    torch.cuda.synchronize()
    _check((s.cpu().numpy(), f.cpu().numpy()),
           oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off), f"p7 M={M}")
    gdb.close()


_PLAIN = []


def plain_db(hm):
    if not _PLAIN:
        res, off = synth.sample_residues(np.random.default_rng(6), np.array([50], np.int64))
        _PLAIN.append(hm.Database(res, off))
    return _PLAIN[0]


def test_degenerate_limits_and_plain_databases(hm):
    """Without degenerate codes the images keep 21 rows; with them, MSV
    profiles beyond 2559 nodes (the exact pass's 64-lane image) and P7
    profiles beyond 2047 nodes are refused with HMSV_EUNSUPPORTED."""
    rng = np.random.default_rng(5)
    res, off = synth.sample_residues(rng, np.array([10, 20, 30], np.int64))
    res[3] = 27                              # non-scoring only: still 21 rows
    plain = hm.Database(res, off)
    assert plain.table_rows == 21
    plain.close()
    res[4] = 26
    deg = hm.Database(res, off)
    assert deg.table_rows == 27
    for filt, M in (("msv", 2560), ("msv", 3839), ("ssv", 2560), ("ssv", 3839)):
        with pytest.raises(hm.HmsvError) as ei:
            hm.db_default_plan(deg, filt, M)
        assert ei.value.status == -2
        assert hm.db_default_plan(plain_db(hm), filt, M).G == 64
    for filt in ("msv", "ssv"):
        p = hm.db_default_plan(deg, filt, 2559)
        assert hm.plan_lds_bytes(p.G, p.Q) * 27 // 21 <= 160 * 1024
    e = synth.sample_emissions(rng, 2500)
    t = synth.sample_transitions(rng, 2500)
    with pytest.raises(hm.HmsvError) as ei:
        hm.p7_score(hm.P7Profile.from_probabilities(e, t, synth.BG), deg)
    assert ei.value.status == -2
    deg.close()


def test_degenerate_batch_equals_plain(hm):
    rng = np.random.default_rng(9)
    Ms = [30, 200, 700, 1500]
    filt = ["msv", "ssv", "msv", "ssv"]
    emis = [synth.sample_emissions(rng, M) for M in Ms]
    res, off = _db(10, emis[1], 1500, 0, 600)
    gdb = hm.Database(res, off)
    profs = [hm.Profile.from_emissions(e, synth.BG) for e in emis]
    print("case degenerate batch", flush=True)
    b = hm.batch.Batch(list(zip(filt, profs)), gdb, branches=2)
    b.launch()
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(zip(filt, profs)):
        es, ef = oracle.score_db(f, oq.quantize(emis[i], synth.BG), res, off)
        assert np.array_equal(b.scores[i].cpu().numpy(), es), (i, Ms[i], f)
        assert np.array_equal(b.flags[i].cpu().numpy(), ef), (i, Ms[i], f)
    b.close()
    gdb.close()


def test_fasta_to_scores(hm):
    """FASTA text (made-up sequences with degenerate letters) through the
    library's parser into a database, scored by all three filters."""
    rng = np.random.default_rng(12)
    M = 60
    e = synth.sample_emissions(rng, M)
    t = synth.sample_transitions(rng, M)
    letters = np.array(list(synth.ALPHABET) + ["?"] + list("BJZUOX"))
    L = rng.integers(0, 400, size=300).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    synth.implant(rng, res, off, [e], 0.2)
    _sprinkle(rng, res, 0.03)
    res[res == 20] = 26           # '?' has no letter: write X
    res[res >= 27] = 26
    text = "".join(f">r{i}\n" + "".join(letters[res[off[i]:off[i + 1]]]) + "\n"
                   for i in range(len(L)))
    heads, r2, o2 = hm.parse_fasta(text)
    assert np.array_equal(r2, res) and np.array_equal(o2, off)
    gdb = hm.Database(r2, o2)
    print("case fasta end to end", flush=True)
    for filt in ("msv", "ssv"):
        fn = hm.msv_score if filt == "msv" else hm.ssv_score
        s, f = fn(hm.Profile.from_emissions(e, synth.BG), gdb)
        torch.cuda.synchronize()
        _check((s.cpu().numpy(), f.cpu().numpy()),
               oracle.score_db(filt, oq.quantize(e, synth.BG), res, off), f"fasta {filt}")
    s, f = hm.p7_score(hm.P7Profile.from_probabilities(e, t, synth.BG), gdb)
    torch.cuda.synchronize()
    _check((s.cpu().numpy(), f.cpu().numpy()),
           oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off), "fasta p7")
    gdb.close()
