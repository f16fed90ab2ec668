"""Scores to nats and P-values end to end: GPU raw scores through the
library's host helpers (hmsv_score_nats, hmsv_gumbel_pvalue) against the
oracle's raw scores through the oracle's own conversion (oracle/pvalue.py),
element by element.

Both conversions are float64 arithmetic on the same integers, so they agree
to rounding: |nats difference| <= 1e-12 and P-values within a relative
1e-12 (absolute 1e-300 where they underflow); saturated scores are +inf
nats and P = 0 on both sides."""
import math

import numpy as np
import pytest

import oracle
from oracle import pvalue as opv
from oracle import quant as oq
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MU, LAM = -2.0, 0.693     # an illustrative null; the paper gives no calibration


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_09683_amd as m
    return m


@pytest.mark.parametrize("filt", ["msv", "ssv"])
@pytest.mark.parametrize("M", [48, 400])
def test_pvalues_match_oracle(hm, filt, M):
    rng = np.random.default_rng(606 + M)
    emis = synth.sample_emissions(rng, M)
    db = synth.random_db(rng, 3000, 0, 900)
    synth.implant(rng, db.res, db.offsets, [emis], 0.1)
    print(f"case pvalue {filt} M={M}", flush=True)
    prof = hm.Profile.from_emissions(emis, synth.BG)
    gdb = hm.Database(db.res, db.offsets)
    s, f = (hm.msv_score if filt == "msv" else hm.ssv_score)(prof, gdb)
    torch.cuda.synchronize()
    gs, gf = s.cpu().numpy(), f.cpu().numpy()
    gdb.close()
    lengths = db.lengths
    g_nats = hm.score_nats(filt, M, gs, gf, lengths)
    g_p = hm.gumbel_pvalue(g_nats, MU, LAM)
    es, ef = oracle.score_db(filt, oq.quantize(emis, synth.BG), db.res, db.offsets)
    e_nats, e_p = opv.pvalues(filt, es, ef, lengths, M, MU, LAM)
    e_nats, e_p = np.array(e_nats), np.array(e_p)
    inf = np.isinf(e_nats)
    assert np.array_equal(inf, np.isinf(g_nats)) and inf.sum() == int(ef.sum())
    assert np.all(g_p[inf] == 0.0)
    assert np.max(np.abs(g_nats[~inf] - e_nats[~inf])) <= 1e-12
    rel = np.abs(g_p - e_p) / np.maximum(np.abs(e_p), 1e-300)
    assert np.all((rel <= 1e-12) | (np.abs(g_p - e_p) <= 1e-300))
    # the implanted hits are the significant ones
    assert (e_p < 1e-3).sum() > 0 and (e_p > 0.5).sum() > 0
