"""CPU oracle for the MSV and SSV filters and the gapped P7Viterbi filter.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
implementation that the GPU library's results are compared with.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the library: its own quantizers
(``quant.py`` for MSV/SSV, ``p7.py`` for P7Viterbi, numpy float64) and its
own scalar C filters (``filters.c``, ``p7viterbi.c``, built with gcc at -O2
without auto-vectorisation).

Every function here has been pinned against something other than itself in
``tests/test_oracle_pins.py``: closed-form constants, an unbounded-integer
dynamic programme, enumeration of all segment paths on tiny inputs, the
maximum over all diagonal segments, and special cases with known answers;
P7Viterbi in ``tests/test_oracle_p7_pins.py``: a hand-worked example,
enumeration of every state path on tiny inputs, the no-gap case against an
enumeration of ungapped multi-segment paths, closed forms and saturation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import quant as q
from . import p7

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "filters.c")
_SRCS = [_SRC, os.path.join(_HERE, "p7viterbi.c")]

BASE = q.BASE


def build(force: bool = False) -> str:
    """Compile filters.c and p7viterbi.c into liboracle.so with gcc (scalar,
    no vectorizer)."""
    if force or not os.path.exists(_LIB_PATH) or \
            any(os.path.getmtime(_LIB_PATH) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-tree-vectorize", "-std=c11",
                               "-shared", "-fPIC", "-pthread", "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        lib.oracle_msv_seq.argtypes = [P, i32, i32, i32, i32, i32, P, i64, P, P]
        lib.oracle_ssv_seq.argtypes = [P, i32, P, i64, P, P]
        lib.oracle_batch.argtypes = [i32, P, P, i32, i32, i32, i32, i32, P, P, P, P,
                                     i64, i32, P, P]
        lib.oracle_batch.restype = i32
        lib.oracle_p7_seq.argtypes = [P, P, i32, i32, P, P, i64, P, P]
        lib.oracle_p7_batch.argtypes = [P, P, i32, i32, P, P, P, P, i64, i32, P, P]
        lib.oracle_p7_batch.restype = i32
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def quantize(emis, bg):
    return q.quantize(emis, bg)


def msv_seq(prof: dict, x, L=None):
    """MSV of one sequence (codes uint8).  Returns (score 0..255, flag)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.uint8)
    L = len(x) if L is None else L
    cost = np.ascontiguousarray(prof["cost"])
    s = np.zeros(1, np.uint8)
    f = np.zeros(1, np.uint8)
    tjbm = q.tjb(L) + prof["tbm"]
    lib.oracle_msv_seq(_ptr(cost), prof["M"], prof["bias"], q.BASE, q.tec(), tjbm,
                       _ptr(x), L, _ptr(s), _ptr(f))
    return int(s[0]), int(f[0])


def ssv_seq(prof: dict, x):
    """SSV of one sequence.  Returns (score -128..127, flag)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.uint8)
    sc = np.ascontiguousarray(prof["sc"])
    s = np.zeros(1, np.int8)
    f = np.zeros(1, np.uint8)
    lib.oracle_ssv_seq(_ptr(sc), prof["M"], _ptr(x), len(x), _ptr(s), _ptr(f))
    return int(s[0]), int(f[0])


def score_db(filt: str, prof: dict, res, offsets, ids=None, nthreads=None):
    """Score sequences of a concatenated database.

    ``ids`` restricts the work to those sequence indices (the returned arrays
    still have one entry per database sequence; entries not scored are 0).
    Returns (score array, flag array): uint8/int8 scores, uint8 flags."""
    lib = _load()
    res = np.ascontiguousarray(res, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    tjb = np.ascontiguousarray(q.tjb(np.diff(offsets)), dtype=np.int32).reshape(-1)
    if ids is None:
        order = np.argsort(-np.diff(offsets), kind="stable").astype(np.int64)
    else:
        ids = np.asarray(ids, dtype=np.int64)
        order = ids[np.argsort(-np.diff(offsets)[ids], kind="stable")]
    order = np.ascontiguousarray(order)
    score = np.zeros(n, np.uint8)
    flag = np.zeros(n, np.uint8)
    nthreads = nthreads or max(1, min(16, os.cpu_count() or 1))
    is_msv = 1 if filt == "msv" else 0
    cost = np.ascontiguousarray(prof["cost"])
    sc = np.ascontiguousarray(prof["sc"])
    rc = lib.oracle_batch(is_msv, _ptr(cost), _ptr(sc), prof["M"], prof["bias"],
                          q.BASE, q.tec(), prof["tbm"], _ptr(res), _ptr(offsets),
                          _ptr(tjb), _ptr(order), len(order), nthreads,
                          _ptr(score), _ptr(flag))
    if rc != 0:
        raise RuntimeError("oracle thread start failed")
    if filt == "ssv":
        return score.view(np.int8), flag
    return score, flag


# ---- gapped Plan-7 Viterbi (P7Viterbi, paper Eq. 1) -------------------------
def _p7_lenmodel(L) -> np.ndarray:
    lm = p7.length_model(L)
    return np.array([lm[k] for k in ("NN", "JJ", "CC", "NB", "JB", "CT", "EJ", "EC")],
                    dtype=np.int32)


def p7_seq(prof: dict, x):
    """P7Viterbi score of one sequence: (int16 score, overflow flag)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.uint8)
    msc = np.ascontiguousarray(prof["msc"], dtype=np.int16)
    tr = np.ascontiguousarray(prof["trans"], dtype=np.int16)
    lm = _p7_lenmodel(len(x))
    s = np.zeros(1, np.int16)
    f = np.zeros(1, np.uint8)
    lib.oracle_p7_seq(_ptr(msc), _ptr(tr), prof["M"], prof["tbm"], _ptr(lm), _ptr(x),
                      len(x), _ptr(s), _ptr(f))
    return int(s[0]), int(f[0])


def p7_score_db(prof: dict, res, offsets, ids=None, nthreads=None):
    """P7Viterbi scores of a concatenated database (int16 scores, uint8
    flags, one per sequence; entries outside ``ids`` are 0)."""
    lib = _load()
    res = np.ascontiguousarray(res, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    lens = np.diff(offsets)
    uniq = {int(L): _p7_lenmodel(int(L)) for L in np.unique(lens)}
    lm = np.ascontiguousarray(np.stack([uniq[int(L)] for L in lens])
                              if n else np.zeros((0, 8), np.int32), dtype=np.int32)
    if ids is None:
        order = np.argsort(-lens, kind="stable").astype(np.int64)
    else:
        ids = np.asarray(ids, dtype=np.int64)
        order = ids[np.argsort(-lens[ids], kind="stable")]
    order = np.ascontiguousarray(order)
    score = np.zeros(n, np.int16)
    flag = np.zeros(n, np.uint8)
    msc = np.ascontiguousarray(prof["msc"], dtype=np.int16)
    tr = np.ascontiguousarray(prof["trans"], dtype=np.int16)
    nthreads = nthreads or max(1, min(16, os.cpu_count() or 1))
    rc = lib.oracle_p7_batch(_ptr(msc), _ptr(tr), prof["M"], prof["tbm"], _ptr(lm),
                             _ptr(res), _ptr(offsets), _ptr(order), len(order), nthreads,
                             _ptr(score), _ptr(flag))
    if rc != 0:
        raise RuntimeError("oracle thread start failed")
    return score, flag
