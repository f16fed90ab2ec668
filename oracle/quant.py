"""Oracle quantizer: float emissions -> 8-bit MSV/SSV score tables (float64).

Test infrastructure only (see the package docstring).

The paper (Sec. 2.1) takes the MSV/SSV models from HMMER3 and does not spell
out their score arithmetic; Alg. 2 and Alg. 4 only show that the kernels read
a 32-entry per-node table of 8-bit match scores (20 amino acids plus 12
"invalid" entries for padding/end codes) and add an offset ``dbias``.  The
reading implemented here, with every constant, is:

* log-odds in third-bits, rounded half away from zero in float64:
  ``r_k(x) = RHAZ(3 * log2(e_k(x) / bg(x)))`` for x < 20, ``-inf`` if e = 0;
* ``bias = max_{k, x<20} r_k(x)`` (the offset the MSV kernel adds, Alg. 2);
* degenerate codes (the paper's table has 32 entries per node, Alg. 4,
  Sec. 3.3; it does not say how ambiguous residues score): code 21 B =
  {D, N}, 22 J = {I, L}, 23 Z = {E, Q}, 24 U = {C}, 25 O = {K}, 26 X = all
  twenty; each scores the background-weighted mean of its members' log-odds
  (the expected score of a residue drawn from the background restricted to
  the set), ``r_k(D) = RHAZ(3 * (sum_x bg(x) log2(e_k(x)/bg(x))) /
  (sum_x bg(x)))`` summed in ascending code order, ``-inf`` if a member has
  e = 0; codes 20 and 27..31 never score;
* unsigned MSV cost ``cost_k(x) = min(255, bias - r_k(x))`` (bias over
  x < 20 only), 255 for the non-scoring codes and -inf entries;
* signed SSV score ``sc_k(x) = max(-128, bias - cost_k(x))`` (Alg. 7 keeps
  -inf as 0x80, i.e. -128);
* special-state costs from the MSV model's transitions (Sec. 2.1, Fig. 1):
  uniform local entry ``tbm(M) = -RHAZ(3 log2(2/(M(M+1))))``, the E->J/C
  split ``tec = -RHAZ(3 log2(1/2)) = 3``, the length model's move cost
  ``tjb(L) = -RHAZ(3 log2(3/(L+3)))`` for a target of length L, and the N/J
  level ``base = 190``.
"""
from __future__ import annotations

import numpy as np

K = 20
KP = 32
BASE = 190


def rhaz(x):
    """Round half away from zero, exactly, for float64 scalars or arrays."""
    x = np.asarray(x, dtype=np.float64)
    t = np.trunc(x)
    frac = np.abs(x - t)                 # exact for |x| < 2**52
    return (t + np.sign(x) * (frac >= 0.5)).astype(np.int64)


def third_bits(p):
    """RHAZ(3 * log2(p)) for p > 0 (float64)."""
    return rhaz(3.0 * np.log2(np.asarray(p, dtype=np.float64)))


def tec() -> int:
    return int(-third_bits(0.5))


def tbm(M: int) -> int:
    M = int(M)
    return int(-third_bits(2.0 / (float(M) * float(M + 1))))


def tjb(L):
    """Per-target length-model cost; L may be an int or an integer array."""
    L = np.asarray(L, dtype=np.float64)
    out = -third_bits(3.0 / (L + 3.0))
    return out if out.ndim else int(out)


NEG_INF = -(1 << 40)   # stands for -inf in integer log-odds

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
# degenerate code -> member residue codes (ascending)
DEGENERATE = {
    21: tuple(sorted(ALPHABET.index(c) for c in "DN")),    # B
    22: tuple(sorted(ALPHABET.index(c) for c in "IL")),    # J
    23: tuple(sorted(ALPHABET.index(c) for c in "EQ")),    # Z
    24: (ALPHABET.index("C"),),                             # U
    25: (ALPHABET.index("K"),),                             # O
    26: tuple(range(K)),                                    # X
}
DEGENERATE_LETTERS = {"B": 21, "J": 22, "Z": 23, "U": 24, "O": 25, "X": 26}


def degenerate_mean_log2(emis: np.ndarray, bg: np.ndarray, code: int):
    """sum_x bg(x) log2(e_k(x)/bg(x)) / sum_x bg(x) over the members of a
    degenerate code, one float64 per node, summed member by member in
    ascending code order; -inf where a member's emission is 0."""
    emis = np.asarray(emis, dtype=np.float64)
    bg = np.asarray(bg, dtype=np.float64)
    M = emis.shape[0]
    num = np.zeros(M, dtype=np.float64)
    den = 0.0
    dead = np.zeros(M, dtype=bool)
    for x in DEGENERATE[code]:
        ratio = emis[:, x] / bg[x]
        dead |= ~(ratio > 0)
        with np.errstate(divide="ignore"):
            num = num + bg[x] * np.log2(np.where(ratio > 0, ratio, 1.0))
        den = den + bg[x]
    return np.where(dead, -np.inf, num / den)


def log_odds(emis: np.ndarray, bg: np.ndarray) -> np.ndarray:
    """r[x, k] for x in 0..31 (int64; NEG_INF for zero emissions and the
    non-scoring codes 20, 27..31)."""
    emis = np.asarray(emis, dtype=np.float64)
    M = emis.shape[0]
    r = np.full((KP, M), NEG_INF, dtype=np.int64)
    ratio = emis.T / np.asarray(bg, dtype=np.float64)[:, None]   # [20, M]
    pos = ratio > 0
    with np.errstate(divide="ignore"):
        vals = rhaz(3.0 * np.log2(np.where(pos, ratio, 1.0)))
    r[:K] = np.where(pos, vals, NEG_INF)
    for code in DEGENERATE:
        m = degenerate_mean_log2(emis, bg, code)
        fin = np.isfinite(m)
        r[code] = np.where(fin, rhaz(3.0 * np.where(fin, m, 0.0)), NEG_INF)
    return r


def quantize(emis: np.ndarray, bg: np.ndarray):
    """Return dict(cost uint8 [32, M], sc int8 [32, M], bias, M, tbm)."""
    r = log_odds(emis, bg)
    M = r.shape[1]
    bias = int(r[:K].max())
    cost = np.full((KP, M), 255, dtype=np.int64)
    cost[:K] = np.minimum(255, bias - r[:K])
    for code in DEGENERATE:
        cost[code] = np.minimum(255, bias - r[code])
    sc = np.maximum(-128, bias - cost)
    return {"cost": cost.astype(np.uint8), "sc": sc.astype(np.int8), "bias": bias,
            "M": M, "tbm": tbm(M), "r": r}


def from_costs(cost: np.ndarray, bias: int):
    """A profile given directly by its 8-bit MSV cost table [32, M] and
    offset ``bias`` (no emissions): the SSV table is derived as above,
    ``sc = max(-128, bias - cost)``; the degenerate codes 21..26 score
    with the given rows, and codes 20 and 27..31 cost 255 (-inf) whatever
    their rows hold.  Same dict as ``quantize``."""
    c = np.array(cost, dtype=np.int64)
    if c.ndim != 2 or c.shape[0] != KP:
        raise ValueError("cost must be [32, M]")
    c[K] = 255
    c[27:] = 255
    M = c.shape[1]
    sc = np.maximum(-128, int(bias) - c)
    return {"cost": c.astype(np.uint8), "sc": sc.astype(np.int8), "bias": int(bias),
            "M": M, "tbm": tbm(M)}
