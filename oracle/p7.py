"""Oracle quantizer for the gapped Plan-7 Viterbi filter (P7Viterbi, paper
Sec. 2.1, Eq. 1; the third stage of the pipeline, after SSV and MSV).

Test infrastructure only (see the package docstring).

The paper gives the middle-cell recurrences (Eq. 1: V_M from the diagonal
M, I, D cells and the B state, V_I from the M and I cells above, V_D from
the M and D cells to the left) and the flanking special states of its DP
matrix (Fig. 2), and says the predecessor ran this stage in 16-bit
arithmetic (Sec. 2.3).  It does not give the scores' units, the local
entry and exit, or the length model.  The reading implemented here:

* scores in units of 1/32 bit, int16 saturating ([-32768, 32767]);
  -32768 stands for -inf (probability zero) and is the starting value of
  every cell: ``q(p) = RHAZ(32 * log2(p))`` for p > 0, -32768 for p = 0;
* match emissions ``msc_k(x) = q(e_k(x) / bg(x))`` (a ratio, not a
  probability: RHAZ(32 log2 ratio)), -32768 for e = 0; degenerate codes
  21..26 (the sets of ``quant.DEGENERATE``) score ``RHAZ(32 * mean)`` of the
  background-weighted mean of their members' log2 ratios (-32768 if a
  member has e = 0), as the MSV tables do in third-bits; codes 20 and
  27..31 score -32768;
  insert states emit with score 0 (inserts follow the background);
* transitions out of node k: ``tMM, tMI, tMD, tIM, tII, tDM, tDD`` =
  q(probability); node M has no successor and no insert state, so its
  M->M, M->D, I->M, D->M, D->D, M->I and I->I are -32768;
* local entry B->M_k uniform: ``tBM = q(2 / (M (M + 1)))``; local exit
  M_k->E with probability 1 (score 0, from match states only);
* length model for a target of L residues (as the MSV model's, Sec. 2.1):
  ``tNN = tJJ = tCC = q(L / (L + 3))``, ``tNB = tJB = tCT = q(3 / (L + 3))``,
  E->J and E->C ``tEJ = tEC = q(1/2) = -32``.

Arrays are int16; emissions residue-major ``msc[x, k]`` ([32, M]),
transitions ``trans[t, k]`` ([7, M], rows in synth.TRANS_NAMES order).
"""
from __future__ import annotations

import numpy as np

from .quant import DEGENERATE, degenerate_mean_log2, rhaz

UNITS = 32              # score units per bit
NEG = -32768            # -inf
POS = 32767


def q(p):
    """RHAZ(UNITS * log2(p)) for p > 0, NEG for p == 0; int64 (clamped
    into int16 range)."""
    p = np.asarray(p, dtype=np.float64)
    with np.errstate(divide="ignore"):
        v = np.where(p > 0, UNITS * np.log2(np.where(p > 0, p, 1.0)), -np.inf)
    out = np.where(np.isfinite(v), rhaz(np.where(np.isfinite(v), v, 0.0)), NEG)
    return np.clip(out, NEG, POS).astype(np.int64)


def quantize(emis: np.ndarray, trans: np.ndarray, bg: np.ndarray) -> dict:
    """Float64 match emissions [M, 20], transitions [M, 7] and background
    [20] -> the int16 tables of the reading above."""
    emis = np.asarray(emis, dtype=np.float64)
    trans = np.asarray(trans, dtype=np.float64)
    M = emis.shape[0]
    msc = np.full((32, M), NEG, dtype=np.int64)
    msc[:20] = q(emis / np.asarray(bg, dtype=np.float64)[None, :]).T
    for code in DEGENERATE:
        m = degenerate_mean_log2(emis, bg, code)
        fin = np.isfinite(m)
        v = np.clip(rhaz(UNITS * np.where(fin, m, 0.0)), NEG, POS)
        msc[code] = np.where(fin, v, NEG)
    t = q(trans).T.copy()                       # [7, M]
    t[[0, 2, 3, 5, 6], M - 1] = NEG             # no node M + 1
    t[[1, 4], M - 1] = NEG                      # no insert state at node M
    return {"M": M, "msc": msc.astype(np.int16), "trans": t.astype(np.int16),
            "tbm": int(q(2.0 / (float(M) * float(M + 1))))}


def length_model(L: int) -> dict:
    """Special-state transition scores for a target of L residues."""
    L = int(L)
    loop = int(q(L / (L + 3.0))) if L > 0 else NEG
    move = int(q(3.0 / (L + 3.0)))
    half = int(q(0.5))
    return {"NN": loop, "JJ": loop, "CC": loop, "NB": move, "JB": move, "CT": move,
            "EJ": half, "EC": half}
