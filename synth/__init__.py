"""Seeded synthetic workloads for the MSV/SSV filters.

This module only draws random inputs: per-node emission probabilities of a
profile, sequence lengths, residue codes, implanted high-scoring segments and
request arrival times.  It holds none of the filters' arithmetic (no log-odds,
no quantization, no dynamic programming), so both the CPU oracle and the GPU
library can be fed from it without sharing any of the method.

The paper measures on Pfam 27.0 query models (lengths 7..2405) against the
env_nr and est_human protein databases (Sec. 4, Table 2).  None of those data
are available here; the workloads below stand in for them with the same kind
of shapes: peaked per-node emission distributions, lognormal protein lengths
with a mean between the two databases' means (197 and 511), and residues drawn
from a standard background composition.

Residue codes: 0..19 are the amino acids in the order ``ALPHABET``; codes
20..31 are non-scoring (invalid) residues.
"""
from __future__ import annotations

import dataclasses
import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
K = 20          # scoring alphabet size
KP = 32         # full code space (20..31 are non-scoring)

# Amino-acid background composition: the BLOSUM62 background frequencies
# (Henikoff & Henikoff, PNAS 1992), three decimals, in ALPHABET order.  They
# sum to exactly 1.000.
BG = np.array([0.074, 0.025, 0.054, 0.054, 0.047, 0.074, 0.026, 0.068, 0.058,
               0.099, 0.025, 0.045, 0.039, 0.034, 0.052, 0.057, 0.051, 0.073,
               0.013, 0.032], dtype=np.float64)
BG = BG / BG.sum()

# Lognormal protein lengths: mean ~350, sd ~300, clipped to [20, 35000].
LOGNORMAL_MU = 5.5825
LOGNORMAL_SIGMA = 0.7422
LEN_MIN, LEN_MAX = 20, 35000

# Order of the spawned child streams of one seed.
_STREAMS = ("profile", "lengths", "residues", "implants", "arrivals")


def streams(seed: int) -> dict:
    """Named, independent generators spawned from one seed."""
    kids = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return {name: np.random.default_rng(s) for name, s in zip(_STREAMS, kids)}


def sample_emissions(rng: np.random.Generator, M: int, conc: float = 0.5) -> np.ndarray:
    """Per-node match emission probabilities, float64 [M, 20].

    Each node is Dirichlet(conc * BG).  The concentrations are small (about
    0.006..0.05), so Gamma draws are taken in log space
    (Gamma(a) = Gamma(a+1) * U**(1/a)) to avoid underflow before normalising.
    Entries can still be exactly 0 after exponentiation; that is a legal
    profile (such a residue can never be emitted by that node).
    """
    a = conc * BG
    g1 = rng.gamma(a + 1.0, size=(M, K))
    u = rng.random(size=(M, K))
    u = np.maximum(u, np.finfo(np.float64).tiny)
    logg = np.log(g1) + np.log(u) / a
    logg -= logg.max(axis=1, keepdims=True)
    e = np.exp(logg)
    e /= e.sum(axis=1, keepdims=True)
    return e


def sample_lengths_uniform(rng, n: int, lo: int, hi: int) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=n, dtype=np.int64)


def sample_lengths_lognormal(rng, n: int) -> np.ndarray:
    L = np.rint(rng.lognormal(LOGNORMAL_MU, LOGNORMAL_SIGMA, size=n))
    return np.clip(L, LEN_MIN, LEN_MAX).astype(np.int64)


def sample_residues(rng, lengths: np.ndarray, chunk: int = 1 << 24):
    """i.i.d. residues from BG.  Returns (codes uint8 [sum L], offsets int64 [n+1])."""
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    res = np.empty(total, dtype=np.uint8)
    cdf = np.cumsum(BG)
    cdf[-1] = 1.0
    for s in range(0, total, chunk):
        e = min(total, s + chunk)
        res[s:e] = np.searchsorted(cdf, rng.random(e - s), side="right").astype(np.uint8)
    np.minimum(res, K - 1, out=res)
    return res, offsets


def implant(rng, res: np.ndarray, offsets: np.ndarray, emis_list, frac: float = 0.01,
            which=None):
    """Overwrite a segment of floor(frac*n) sequences with residues emitted by a profile.

    For a chosen sequence of length L and profile of length M: segment length
    l ~ U{ceil(min(M,L)/2) .. min(M,L)}, start node k0 ~ U{0 .. M-l},
    start position p ~ U{0 .. L-l}; residue t is drawn from node k0+t.
    ``emis_list`` is a list of emission arrays; each implant picks one
    uniformly (or ``which[i]`` if given).  Returns the implanted sequence ids.
    """
    n = len(offsets) - 1
    cnt = int(np.floor(frac * n))
    ids = np.sort(rng.choice(n, size=cnt, replace=False)) if cnt else np.zeros(0, np.int64)
    cdfs = [np.cumsum(e, axis=1) for e in emis_list]
    for t, sid in enumerate(ids):
        pi = int(which[t]) if which is not None else int(rng.integers(len(emis_list)))
        cdf = cdfs[pi]
        M = cdf.shape[0]
        L = int(offsets[sid + 1] - offsets[sid])
        if L == 0:
            continue
        mx = min(M, L)
        lo = (mx + 1) // 2
        ln = int(rng.integers(lo, mx + 1))
        k0 = int(rng.integers(0, M - ln + 1))
        p = int(rng.integers(0, L - ln + 1))
        u = rng.random(ln)
        rows = cdf[k0:k0 + ln]
        codes = (rows < (u[:, None] * rows[:, -1:])).sum(axis=1)
        res[offsets[sid] + p: offsets[sid] + p + ln] = np.minimum(codes, K - 1).astype(np.uint8)
    return ids


def random_cost_table(rng, M: int, dbias: int):
    """A profile given directly as an 8-bit MSV cost table (no emissions).

    Returns (cost uint8 [32, M], consensus uint8 [M]).  Every node has a
    consensus residue scoring dbias - cost in 1..min(dbias, 10), or dbias
    itself (cost 0) at 1.5% of the nodes, so a run of consensus residues along
    a diagonal climbs in small steps with the odd jump.  The other residues
    cost 2 or more above dbias (they score below zero), 5% of them 255.
    Rows 20..31 are 255 (the non-scoring codes).  dbias in 0..255."""
    cost = np.clip(dbias + 2 + np.rint(np.abs(rng.normal(0.0, 8.0, size=(K, M)))),
                   0, 255).astype(np.int64)
    cost[rng.random(size=(K, M)) < 0.05] = 255
    cons = rng.integers(0, K, size=M)
    gain = rng.integers(1, max(1, min(dbias, 10)) + 1, size=M)
    gain[rng.random(M) < 0.015] = dbias
    cost[cons, np.arange(M)] = np.maximum(0, dbias - gain)
    full = np.full((KP, M), 255, dtype=np.uint8)
    full[:K] = cost.astype(np.uint8)
    return full, cons.astype(np.uint8)


def implant_consensus(rng, res, offsets, consensus, frac: float, max_len: int,
                      per_seq=(1, 3)):
    """Overwrite 1..3 segments (``per_seq``) of a fraction of the sequences
    with runs of consensus residues (``random_cost_table``): segment length
    U{1..min(max_len, M, L)}, start node and position uniform.  Returns the
    implanted sequence ids."""
    M = len(consensus)
    ids = np.flatnonzero(rng.random(len(offsets) - 1) < frac)
    for sid in ids:
        a, b = int(offsets[sid]), int(offsets[sid + 1])
        if b == a:
            continue
        for _ in range(int(rng.integers(per_seq[0], per_seq[1] + 1))):
            ln = int(rng.integers(1, min(max_len, M, b - a) + 1))
            k0 = int(rng.integers(0, M - ln + 1))
            p = a + int(rng.integers(0, b - a - ln + 1))
            res[p:p + ln] = consensus[k0:k0 + ln]
    return ids


@dataclasses.dataclass
class Database:
    res: np.ndarray       # uint8 codes, concatenated
    offsets: np.ndarray   # int64 [n+1]

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def residues(self) -> int:
        return int(self.offsets[-1])

    def seq(self, i: int) -> np.ndarray:
        return self.res[self.offsets[i]:self.offsets[i + 1]]

    def subset(self, ids) -> "Database":
        ids = np.asarray(ids, dtype=np.int64)
        lens = self.lengths[ids]
        off = np.zeros(len(ids) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        out = np.empty(int(off[-1]), dtype=np.uint8)
        for t, i in enumerate(ids):
            out[off[t]:off[t + 1]] = self.seq(int(i))
        return Database(out, off)


@dataclasses.dataclass
class Workload:
    name: str
    filters: list         # "msv" / "ssv" per query
    emissions: list       # float64 [M, 20] per query
    db: Database
    implanted: np.ndarray
    seed: int

    @property
    def Ms(self):
        return [int(e.shape[0]) for e in self.emissions]

    def cells(self) -> int:
        return int(sum(self.Ms)) * self.db.residues


def plain_msv_m48(seed: int = 1, nseq: int = 2000) -> Workload:
    """Plain MSV, M=48, lengths U{50..500}, residues i.i.d. from BG."""
    st = streams(seed)
    emis = sample_emissions(st["profile"], 48)
    L = sample_lengths_uniform(st["lengths"], nseq, 50, 500)
    res, off = sample_residues(st["residues"], L)
    return Workload("msv_m48_2k", ["msv"], [emis], Database(res, off),
                    np.zeros(0, np.int64), seed)


def lognormal_db(seed: int, nseq: int, implant_emis=None, frac: float = 0.01, st=None):
    st = st or streams(seed)
    L = sample_lengths_lognormal(st["lengths"], nseq)
    res, off = sample_residues(st["residues"], L)
    ids = np.zeros(0, np.int64)
    if implant_emis:
        ids = implant(st["implants"], res, off, implant_emis, frac)
    return Database(res, off), ids


def plain_msv_m400(seed: int = 2, nseq: int = 500_000) -> Workload:
    """Plain MSV, M=400, lognormal lengths, 1% implants from the query itself."""
    st = streams(seed)
    emis = sample_emissions(st["profile"], 400)
    db, ids = lognormal_db(seed, nseq, [emis], 0.01, st)
    return Workload("msv_m400_500k", ["msv"], [emis], db, ids, seed)


def plain_ssv(seed: int = 3, nseq: int = 500_000, Ms=(100, 400, 1000, 2400),
              db: Database | None = None, implanted=None) -> Workload:
    """Plain SSV queries of several lengths against the 500k lognormal database.

    The database is the M=400 MSV workload's (seed 2) unless one is given."""
    st = streams(seed)
    emis = [sample_emissions(st["profile"], int(m)) for m in Ms]
    if db is None:
        base = plain_msv_m400(nseq=nseq)
        db, implanted = base.db, base.implanted
    return Workload("ssv_500k", ["ssv"] * len(Ms), emis, db,
                    implanted if implanted is not None else np.zeros(0, np.int64), seed)


def batched(seed: int = 4, nseq: int = 1_000_000, nq: int = 64, mlo: int = 30,
            mhi: int = 2400) -> Workload:
    """64 queries, M ~ U{30..2400}, MSV/SSV alternating, 1M-sequence lognormal DB.

    Implants are drawn from the queries, each implant's profile uniform."""
    st = streams(seed)
    Ms = st["profile"].integers(mlo, mhi + 1, size=nq)
    emis = [sample_emissions(st["profile"], int(m)) for m in Ms]
    filt = ["msv" if i % 2 == 0 else "ssv" for i in range(nq)]
    db, ids = lognormal_db(seed, nseq, emis, 0.01, st)
    return Workload("batched_64q_1m", filt, emis, db, ids, seed)


def served_db(seed: int = 5, nseq: int = 2_000_000) -> Database:
    st = streams(seed)
    db, _ = lognormal_db(seed, nseq, None, 0.0, st)
    return db


def request_trace(seed: int, nreq: int, qps: float, mlo: int = 30, mhi: int = 2000):
    """Poisson arrivals.  Returns (arrival times s, M per request, filter per
    request, emissions per request)."""
    kids = np.random.SeedSequence([seed, 0x5E4F]).spawn(2)
    ra = np.random.default_rng(kids[0])
    rp = np.random.default_rng(kids[1])
    gaps = ra.exponential(1.0 / qps, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    Ms = rp.integers(mlo, mhi + 1, size=nreq)
    filt = ["msv" if b else "ssv" for b in (rp.random(nreq) < 0.5)]
    emis = [sample_emissions(rp, int(m)) for m in Ms]
    return t, Ms, filt, emis


def random_db(rng, nseq: int, lo: int, hi: int) -> Database:
    """Small helper for tests: uniform lengths in [lo, hi], i.i.d. residues."""
    L = rng.integers(lo, hi + 1, size=nseq).astype(np.int64)
    res, off = sample_residues(rng, L)
    return Database(res, off)


# ---- gapped (Plan-7) profiles -------------------------------------------
# Transition order per node k (transitions out of node k): M->M, M->I, M->D,
# I->M, I->I, D->M, D->D.  The means below are typical of profile HMMs
# built from curated families (matches dominate, gaps are rare and short);
# they stand in for Pfam models, which are not available.
TRANS_NAMES = ("MM", "MI", "MD", "IM", "II", "DM", "DD")
_TRANS_MEAN_M = np.array([0.90, 0.05, 0.05])
_TRANS_MEAN_I = np.array([0.60, 0.40])
_TRANS_MEAN_D = np.array([0.70, 0.30])


def sample_transitions(rng, M: int, conc: float = 20.0) -> np.ndarray:
    """Per-node transition probabilities, float64 [M, 7] in TRANS_NAMES order.

    Each node's M->{M,I,D}, I->{M,I} and D->{M,D} distributions are
    Dirichlet(conc * mean).  The last node has no successor: its entries
    are whatever was drawn (a profile's users ignore them)."""
    out = np.empty((M, 7), dtype=np.float64)
    out[:, 0:3] = rng.dirichlet(conc * _TRANS_MEAN_M, size=M)
    out[:, 3:5] = rng.dirichlet(conc * _TRANS_MEAN_I, size=M)
    out[:, 5:7] = rng.dirichlet(conc * _TRANS_MEAN_D, size=M)
    return out


def implant_gapped(rng, res, offsets, emis, trans, frac: float, max_len=None):
    """Overwrite a segment of a fraction of the sequences with residues
    emitted along a random path through a gapped profile: start at a random
    node's match state, then follow the node's transition probabilities
    (M->M/I/D, I->M/I, D->M/D), emitting a residue from the match
    emissions at match states and from the background at insert states,
    until the last node or ``max_len`` residues.  Returns the ids."""
    M = emis.shape[0]
    n = len(offsets) - 1
    ids = np.flatnonzero(rng.random(n) < frac)
    bg_cdf = np.cumsum(BG)
    em_cdf = np.cumsum(emis, axis=1)
    for sid in ids:
        a, b = int(offsets[sid]), int(offsets[sid + 1])
        L = b - a
        if L == 0:
            continue
        cap = min(L, max_len or L)
        k = int(rng.integers(0, M))
        state = 0                              # 0 match, 1 insert, 2 delete
        out = []
        while len(out) < cap and k < M:
            if state == 0:
                out.append(int(np.searchsorted(em_cdf[k], rng.random() * em_cdf[k, -1],
                                               side="right")))
                p = trans[k, 0:3]
            elif state == 1:
                out.append(int(np.searchsorted(bg_cdf, rng.random() * bg_cdf[-1],
                                               side="right")))
                p = trans[k, 3:5]
            else:
                p = trans[k, 5:7]
            u = rng.random() * p.sum()
            nxt = int(np.searchsorted(np.cumsum(p), u, side="right"))
            if state == 0:
                state = (0, 1, 2)[min(nxt, 2)]
            elif state == 1:
                state = (0, 1)[min(nxt, 1)]
            else:
                state = (0, 2)[min(nxt, 1)]
            if state != 1:
                k += 1
        ln = len(out)
        if ln == 0:
            continue
        p0 = int(rng.integers(0, L - ln + 1))
        res[a + p0: a + p0 + ln] = np.minimum(np.array(out), K - 1).astype(np.uint8)
    return ids
