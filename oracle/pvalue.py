"""Oracle conversion of raw filter scores to nats and Gumbel P-values.

Test infrastructure only (see the package docstring); shares nothing with
the library's host helpers.

The paper's kernels record a P-value when a sequence ends (Alg. 2 and
Alg. 7, end-residue branch) but leave the score units and the null
distribution to HMMER3.  The reading used here:

* the filters count in third-bits, s = 3 / ln 2 units per nat;
* an MSV raw score still holds the N->B move and the base level:
  nats = (raw - tjb(L) - base) / s - 3;
* an SSV raw score is relative to -128 and lacks the entry, exit and both
  length moves: nats = (raw + 128 - tbm(M) - 2 tjb(L) - tec) / s - 3;
* the final 3 nats stand for the N/C/J length loops;
* a saturated score (flag 1) is +infinity;
* P(S >= x) under a Gumbel null with location mu and scale lambda (a
  calibration the paper does not give, so the caller supplies it) is
  1 - exp(-exp(-lambda (x - mu))).

Plain Python floats, one score at a time.
"""
from __future__ import annotations

import math

from . import quant as q

UNITS_PER_NAT = 3.0 / math.log(2.0)


def nats(filt: str, raw: int, flag: int, L: int, M: int) -> float:
    """One raw score (uint8 value for MSV, int8 value for SSV) in nats."""
    if flag:
        return math.inf
    if filt == "msv":
        units = raw - q.tjb(int(L)) - q.BASE
    else:
        units = raw + 128 - q.tbm(int(M)) - 2 * q.tjb(int(L)) - q.tec()
    return units / UNITS_PER_NAT - 3.0


def gumbel_p(x: float, mu: float, lam: float) -> float:
    """P(S >= x) for a Gumbel(mu, lambda) score; 0 for x = +inf."""
    if math.isinf(x) and x > 0:
        return 0.0
    return -math.expm1(-math.exp(-lam * (x - mu)))


def pvalues(filt: str, scores, flags, lengths, M: int, mu: float, lam: float):
    """Lists of nats and P-values for arrays of raw scores, flags and lengths."""
    n = [nats(filt, int(s), int(f), int(L), M) for s, f, L in zip(scores, flags, lengths)]
    return n, [gumbel_p(v, mu, lam) for v in n]
