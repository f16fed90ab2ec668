"""GPU parity of the P7Viterbi filter: every sequence's int16 score and
saturation flag, bit for bit, against the oracle (oracle/p7viterbi.c).

Both sides quantize the same float64 profile independently (the library in
C++, the oracle in numpy) and score the same seeded databases, with gapped
implants emitted along paths through the profile (matches, inserts and
deletes), so that the D chains and insert runs of real alignments are
exercised."""
import numpy as np
import pytest

import oracle
from oracle import p7 as op7
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as m
    return m


def _profile(seed, M, harsh=False):
    rng = np.random.default_rng(seed)
    e = synth.sample_emissions(rng, M)
    t = synth.sample_transitions(rng, M)
    if harsh:
        # zero probabilities (-inf scores) on some emissions and transitions
        e[rng.random(e.shape) < 0.05] = 0.0
        e[:, 0] += 1e-3
        t[rng.random(t.shape) < 0.08] = 0.0
    return e, t


def _db(seed, M, e, t, nseq, lo, hi, frac=0.3, max_len=None):
    rng = np.random.default_rng(seed)
    L = rng.integers(lo, hi + 1, size=nseq).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    synth.implant_gapped(rng, res, off, e, t, frac, max_len=max_len)
    return res, off


def _run(hm, e, t, res, off, plan=None):
    prof = hm.P7Profile.from_probabilities(e, t, synth.BG)
    db = hm.Database(res, off)
    s, f = hm.p7_score(prof, db, plan=plan)
    torch.cuda.synchronize()
    out = s.cpu().numpy(), f.cpu().numpy()
    db.close()
    return out


def _check(got, exp, what):
    gs, gf = got
    es, ef = exp
    bad = np.nonzero((gs != es) | (gf != ef))[0]
    assert bad.size == 0, (f"{what}: {bad.size} mismatches, first at {bad[:5]}: "
                           f"gpu {gs[bad[:5]]}/{gf[bad[:5]]} oracle {es[bad[:5]]}/{ef[bad[:5]]}")


def _oracle(e, t, res, off):
    return oracle.p7_score_db(op7.quantize(e, t, synth.BG), res, off)


@pytest.mark.parametrize("M", [1, 5, 30, 48, 100, 257, 400, 700])
def test_p7_default_plan(hm, M):
    e, t = _profile(100 + M, M)
    res, off = _db(200 + M, M, e, t, 1500, 0, 700)
    print(f"case p7 default M={M} plan={hm.p7_default_plan(M).as_tuple()}", flush=True)
    exp = _oracle(e, t, res, off)
    _check(_run(hm, e, t, res, off), exp, f"M={M}")
    # the implanted paths score well above the background
    if M >= 30:
        assert (exp[0] > 0).sum() > 100


@pytest.mark.parametrize("G,Q", [(4, 13), (8, 7), (16, 4), (32, 2), (64, 1), (8, 16), (64, 3)])
def test_p7_every_group_width(hm, G, Q):
    """M = 100 on every group width; (8, 16) and (64, 3) hold more slots
    than nodes (padding slots past node M)."""
    M = 100
    e, t = _profile(7, M)
    res, off = _db(8, M, e, t, 1200, 0, 400)
    print(f"case p7 G={G} Q={Q}", flush=True)
    exp = _oracle(e, t, res, off)
    _check(_run(hm, e, t, res, off, hm.make_plan(G, Q)), exp, f"G={G} Q={Q}")


@pytest.mark.parametrize("G,Q,M", [(64, 22, 2815), (32, 16, 1023), (4, 16, 127)])
def test_p7_largest_plans(hm, G, Q, M):
    e, t = _profile(11, M)
    res, off = _db(12, M, e, t, 300, 0, 1200, frac=0.5)
    print(f"case p7 largest G={G} Q={Q} M={M}", flush=True)
    exp = _oracle(e, t, res, off)
    _check(_run(hm, e, t, res, off, hm.make_plan(G, Q)), exp, f"G={G} Q={Q} M={M}")


def test_p7_edge_lengths_and_codes(hm):
    """Empty sequences, lengths around the 16-residue step, one long
    sequence, and codes 20..31 inside sequences (non-scoring 20, 27..31 and
    the degenerate 21..26)."""
    M = 64
    e, t = _profile(21, M)
    lens = [0, 1, 2, 3, 4, 15, 16, 17, 31, 32, 33, 0, 5000, 63, 64, 65, 0, 1]
    rng = np.random.default_rng(22)
    res, off = synth.sample_residues(rng, np.array(lens * 20, np.int64))
    synth.implant_gapped(rng, res, off, e, t, 0.5)
    junk = rng.random(res.size) < 0.03
    res[junk] = rng.integers(20, 32, size=int(junk.sum())).astype(np.uint8)
    print("case p7 edges", flush=True)
    exp = _oracle(e, t, res, off)
    for plan in (None, hm.make_plan(4, 9), hm.make_plan(64, 1)):
        _check(_run(hm, e, t, res, off, plan), exp, f"edges {plan}")


def test_p7_harsh_profile_minus_infinity(hm):
    """Zero emission and transition probabilities: -inf (-32768) terms
    reach cells through saturating adds on both sides."""
    M = 150
    e, t = _profile(31, M, harsh=True)
    res, off = _db(32, M, e, t, 1500, 0, 500, frac=0.4)
    print("case p7 harsh", flush=True)
    exp = _oracle(e, t, res, off)
    for plan in (None, hm.make_plan(8, 10), hm.make_plan(32, 3)):
        _check(_run(hm, e, t, res, off, plan), exp, f"harsh {plan}")


def test_p7_saturation(hm):
    """Peaked emissions and long matching stretches drive E to 32767: those
    sequences score 32767 with flag 1; the rest score normally."""
    M = 300
    rng = np.random.default_rng(41)
    cons = rng.integers(0, 20, size=M)
    e = np.full((M, 20), 1e-4)
    e[np.arange(M), cons] = 1.0
    e /= e.sum(1, keepdims=True)
    t = synth.sample_transitions(rng, M, conc=200.0)
    L = rng.integers(50, 1500, size=400).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    for i in range(0, 400, 3):
        a, b = int(off[i]), int(off[i + 1])
        res[a:b] = np.tile(cons, 1 + (b - a) // M)[: b - a].astype(np.uint8)
    print("case p7 saturation", flush=True)
    exp = _oracle(e, t, res, off)
    assert exp[1].sum() > 20 and (exp[1] == 0).sum() > 100
    _check(_run(hm, e, t, res, off), exp, "saturation")


def test_p7_many_records_per_group(hm):
    """A small grid (two blocks): every lane group takes many records, in
    alternating directions, with the next one prefetched."""
    M = 80
    e, t = _profile(51, M)
    res, off = _db(52, M, e, t, 5000, 0, 300)
    print("case p7 two blocks", flush=True)
    exp = _oracle(e, t, res, off)
    for G, Q in ((8, 6), (64, 1)):
        _check(_run(hm, e, t, res, off, hm.make_plan(G, Q, waves_per_block=2, blocks=2)),
               exp, f"G={G} blocks=2")


def test_p7_repeat_calls_share_workspace(hm):
    """Two profiles scored back to back on one stream with one workspace."""
    M1, M2 = 200, 37
    e1, t1 = _profile(61, M1)
    e2, t2 = _profile(62, M2)
    res, off = _db(63, M1, e1, t1, 2000, 0, 600)
    db = hm.Database(res, off)
    ws = hm.new_workspace("cuda", db.nseq)
    p1 = hm.P7Profile.from_probabilities(e1, t1, synth.BG)
    p2 = hm.P7Profile.from_probabilities(e2, t2, synth.BG)
    s1, f1 = hm.p7_score(p1, db, workspace=ws)
    s2, f2 = hm.p7_score(p2, db, workspace=ws)
    torch.cuda.synchronize()
    print("case p7 repeat", flush=True)
    _check((s1.cpu().numpy(), f1.cpu().numpy()), _oracle(e1, t1, res, off), "first")
    _check((s2.cpu().numpy(), f2.cpu().numpy()), _oracle(e2, t2, res, off), "second")
    db.close()


@pytest.mark.parametrize("Q,M", [(2, 200), (16, 2047), (18, 2200), (20, 2400)])
def test_p7_sixteen_wave_blocks(hm, Q, M):
    """64-lane groups of at most 18 registers, or of 20, also run as blocks
    of 16 wavefronts (1024 threads)."""
    e, t = _profile(71 + M, M)
    res, off = _db(72 + M, M, e, t, 600, 0, 900, frac=0.3)
    print(f"case p7 16-wave blocks Q={Q} M={M}", flush=True)
    exp = _oracle(e, t, res, off)
    for wpb in (16, 12):
        _check(_run(hm, e, t, res, off, hm.make_plan(64, Q, wpb)), exp, f"wpb={wpb} Q={Q}")
