"""MSV / SSV profile-HMM filters on AMD Instinct MI355X (gfx950).

A thin ctypes binding over ``libhmsv.so`` (C ABI in ``include/hmsv.h``).
This module only marshals arguments: quantization, database packing and both
filters run in the native library and its HIP kernels.  PyTorch supplies
device memory (output and table tensors) and streams.

If ``libhmsv.so`` has not been built, importing this package raises
ImportError: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
from typing import NamedTuple
import os

import numpy as np
import torch  # must load before libhmsv so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmsv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_1707_09683_amd/build.py` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
K = 20
KP = 32
BASE = 190
TEC = 3
MAX_M = 3839
MAX_BIAS = 64


class HmsvError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.hmsv_strerror(status).decode()
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


class _CProfile(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("dbias", ctypes.c_int32),
                ("cost", ctypes.c_void_p), ("sc", ctypes.c_void_p)]


class Plan(ctypes.Structure):
    """Launch plan (hmsv_plan): group width G, registers per lane Q,
    waves per block, blocks (0 = persistent)."""
    _fields_ = [("G", ctypes.c_int32), ("Q", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("blocks", ctypes.c_int32)]

    def __repr__(self):
        return (f"Plan(G={self.G}, Q={self.Q}, waves_per_block={self.waves_per_block}, "
                f"blocks={self.blocks})")

    def as_tuple(self):
        return (self.G, self.Q, self.waves_per_block, self.blocks)


_P = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64
_lib.hmsv_strerror.restype = ctypes.c_char_p
_lib.hmsv_strerror.argtypes = [ctypes.c_int]
_lib.hmsv_tbm.restype = _i32
_lib.hmsv_tbm.argtypes = [_i32]
_lib.hmsv_tjb.restype = _i32
_lib.hmsv_tjb.argtypes = [_i64]
_lib.hmsv_quantize.restype = ctypes.c_int
_lib.hmsv_quantize.argtypes = [_P, _P, _i32, _P, _P, ctypes.POINTER(_i32)]
_lib.hmsv_db_create.restype = ctypes.c_int
_lib.hmsv_db_create.argtypes = [_P, _P, _i64, ctypes.POINTER(_P)]
_lib.hmsv_db_destroy.restype = None
_lib.hmsv_db_destroy.argtypes = [_P]
for _f in ("hmsv_db_nseq", "hmsv_db_residues", "hmsv_db_padded_rows"):
    getattr(_lib, _f).restype = _i64
    getattr(_lib, _f).argtypes = [_P]
class Alg1Stats(ctypes.Structure):
    """hmsv_alg1_stats: the padding and balance of Alg. 1's blocks."""
    _fields_ = [("real", _i64), ("ending", _i64), ("padding", _i64), ("max_height", _i64),
                ("mean_height", ctypes.c_double), ("sd_height", ctypes.c_double),
                ("mean_ending", ctypes.c_double), ("sd_ending", ctypes.c_double),
                ("prr", ctypes.c_double), ("efficiency", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.hmsv_alg1_pack.restype = ctypes.c_int
_lib.hmsv_alg1_pack.argtypes = [_P, _i64, _i32, _i32, _P, _P, ctypes.POINTER(Alg1Stats)]
_lib.hmsv_fasta_parse.restype = ctypes.c_int
_lib.hmsv_fasta_parse.argtypes = [ctypes.c_char_p, _i64, _P, _P, _P, ctypes.POINTER(_i64),
                                  ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
_lib.hmsv_db_table_rows.restype = _i32
_lib.hmsv_db_table_rows.argtypes = [_P]
_lib.hmsv_db_default_plan.restype = ctypes.c_int
_lib.hmsv_db_default_plan.argtypes = [_P, _i32, _i32, ctypes.POINTER(Plan)]
_lib.hmsv_default_plan.restype = ctypes.c_int
_lib.hmsv_default_plan.argtypes = [_i32, _i32, ctypes.POINTER(Plan)]
_lib.hmsv_workspace_bytes.restype = ctypes.c_size_t
_lib.hmsv_workspace_bytes.argtypes = [_i64]
_lib.hmsv_plan_lds_bytes.restype = ctypes.c_size_t
_lib.hmsv_plan_lds_bytes.argtypes = [_i32, _i32]
for _f in ("hmsv_msv_score", "hmsv_ssv_score"):
    getattr(_lib, _f).restype = ctypes.c_int
    getattr(_lib, _f).argtypes = [ctypes.POINTER(_CProfile), _P, _P, _P, _P,
                                  ctypes.POINTER(Plan), _P]
_lib.hmsv_msv_score_noalloc.restype = ctypes.c_int
_lib.hmsv_msv_score_noalloc.argtypes = [ctypes.POINTER(_CProfile), _P, _P, _P,
                                        ctypes.POINTER(Plan), _P]
for _f in ("hmsv_msv_score_range", "hmsv_ssv_score_range"):
    getattr(_lib, _f).restype = ctypes.c_int
    getattr(_lib, _f).argtypes = [ctypes.POINTER(_CProfile), _P, _i64, _i64, _P, _P, _P,
                                  ctypes.POINTER(Plan), _P]
_lib.hmsv_db_order.restype = ctypes.c_int
_lib.hmsv_db_order.argtypes = [_P, _P]
_lib.hmsv_score_nats.restype = ctypes.c_int
_lib.hmsv_score_nats.argtypes = [_i32, _i32, _P, _P, _P, _i64, _P]
_lib.hmsv_gumbel_pvalue.restype = ctypes.c_int
_lib.hmsv_gumbel_pvalue.argtypes = [_P, _i64, ctypes.c_double, ctypes.c_double, _P]
_lib.hmsv_split_info.restype = ctypes.c_int
_lib.hmsv_split_info.argtypes = [_P, _i64, _i64, _i32, _i32, ctypes.POINTER(Plan),
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]

class _CP7Profile(ctypes.Structure):
    _fields_ = [("M", _i32), ("tbm", _i32), ("msc", _P), ("trans", _P)]


_lib.hmsv_p7_quantize.restype = ctypes.c_int
_lib.hmsv_p7_quantize.argtypes = [_P, _P, _P, _i32, _P, _P, ctypes.POINTER(_i32)]
_lib.hmsv_p7_length_model.restype = ctypes.c_int
_lib.hmsv_p7_length_model.argtypes = [_i64, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.hmsv_p7_lds_bytes.restype = ctypes.c_size_t
_lib.hmsv_p7_lds_bytes.argtypes = [_i32, _i32]
_lib.hmsv_p7_default_plan.restype = ctypes.c_int
_lib.hmsv_p7_default_plan.argtypes = [_i32, ctypes.POINTER(Plan)]
_lib.hmsv_p7_score.restype = ctypes.c_int
_lib.hmsv_p7_score.argtypes = [ctypes.POINTER(_CP7Profile), _P, _P, _P, _P,
                               ctypes.POINTER(Plan), _P]
_lib.hmsv_select.restype = ctypes.c_int
_lib.hmsv_select.argtypes = [_P, _P, _P, _i32, _i32, _P, _P, _P, _P]
_lib.hmsv_p7_score_selected.restype = ctypes.c_int
_lib.hmsv_p7_score_selected.argtypes = [ctypes.POINTER(_CP7Profile), _P, _P, _P, _P, _P, _P,
                                        ctypes.POINTER(Plan), _P]

EXPORTED = ("hmsv_strerror", "hmsv_tbm", "hmsv_tjb", "hmsv_quantize", "hmsv_db_create",
            "hmsv_db_destroy", "hmsv_db_nseq", "hmsv_db_residues", "hmsv_db_padded_rows",
            "hmsv_default_plan", "hmsv_plan_lds_bytes", "hmsv_workspace_bytes",
            "hmsv_msv_score", "hmsv_ssv_score",
            "hmsv_batch_create", "hmsv_batch_launch", "hmsv_batch_destroy",
            "hmsv_msv_score_range", "hmsv_ssv_score_range", "hmsv_db_order",
            "hmsv_split_info", "hmsv_score_nats", "hmsv_gumbel_pvalue",
            "hmsv_msv_score_noalloc", "hmsv_db_table_rows", "hmsv_db_default_plan",
            "hmsv_fasta_parse", "hmsv_alg1_pack",
            "hmsv_p7_quantize", "hmsv_p7_length_model",
            "hmsv_p7_lds_bytes", "hmsv_p7_default_plan", "hmsv_p7_score",
            "hmsv_select", "hmsv_p7_score_selected")


def _check(rc: int, what: str):
    if rc != OK:
        raise HmsvError(rc, what)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def tbm(M: int) -> int:
    return int(_lib.hmsv_tbm(int(M)))


def tjb(L: int) -> int:
    return int(_lib.hmsv_tjb(int(L)))


def quantize(emissions, bg):
    """Host quantization (hmsv_quantize).  Returns dict(cost uint8 [32, M],
    sc int8 [32, M], dbias, M)."""
    e = np.ascontiguousarray(emissions, dtype=np.float64)
    b = np.ascontiguousarray(bg, dtype=np.float64)
    if e.ndim != 2 or e.shape[1] != K or b.shape != (K,):
        raise ValueError("emissions must be [M, 20] and bg [20]")
    M = e.shape[0]
    cost = np.empty((KP, M), np.uint8)
    sc = np.empty((KP, M), np.int8)
    dbias = _i32(0)
    _check(_lib.hmsv_quantize(_np_ptr(e), _np_ptr(b), M, _np_ptr(cost), _np_ptr(sc),
                              ctypes.byref(dbias)), "hmsv_quantize")
    return {"cost": cost, "sc": sc, "dbias": int(dbias.value), "M": M}


class Profile:
    """A quantized profile with its tables in device memory (torch tensors)."""

    def __init__(self, cost: torch.Tensor, sc: torch.Tensor, dbias: int):
        if cost.dtype != torch.uint8 or sc.dtype != torch.int8:
            raise TypeError("cost must be uint8 and sc int8")
        if cost.shape != sc.shape or cost.shape[0] != KP:
            raise ValueError("tables must both be [32, M]")
        self.cost = cost.contiguous()
        self.sc = sc.contiguous()
        self.M = int(cost.shape[1])
        self.dbias = int(dbias)
        self.device = self.cost.device
        self._c = _CProfile(self.M, self.dbias, self.cost.data_ptr(), self.sc.data_ptr())

    @classmethod
    def from_emissions(cls, emissions, bg, device="cuda"):
        q = quantize(emissions, bg)
        return cls(torch.from_numpy(q["cost"]).to(device), torch.from_numpy(q["sc"]).to(device),
                   q["dbias"])


class Database:
    """Packed, device-resident sequence database (hmsv_db)."""

    def __init__(self, residues, offsets, device="cuda"):
        res = np.ascontiguousarray(residues, dtype=np.uint8)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        if off.ndim != 1 or len(off) < 1:
            raise ValueError("offsets must be [nseq + 1]")
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.hmsv_db_create(_np_ptr(res) if res.size else None, _np_ptr(off),
                                       len(off) - 1, ctypes.byref(h)), "hmsv_db_create")
        self._h = h
        self.lengths = np.diff(off)
        self.nseq = int(_lib.hmsv_db_nseq(h))
        self.residues = int(_lib.hmsv_db_residues(h))
        self.padded_rows = int(_lib.hmsv_db_padded_rows(h))
        # LDS table rows of its scoring calls: 27 with degenerate codes, else 21
        self.table_rows = int(_lib.hmsv_db_table_rows(h))

    def order(self) -> np.ndarray:
        """Processing order: original index of each position (longest first)."""
        ids = np.empty(self.nseq, np.int64)
        _check(_lib.hmsv_db_order(self._h, _np_ptr(ids)), "hmsv_db_order")
        return ids

    def close(self):
        if getattr(self, "_h", None):
            _lib.hmsv_db_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_plan(filt: str, M: int) -> Plan:
    p = Plan()
    _check(_lib.hmsv_default_plan(1 if filt == "msv" else 0, int(M), ctypes.byref(p)),
           "hmsv_default_plan")
    return p


def alg1_pack(lengths, nblocks: int, width: int):
    """The paper's warp-based blocks (Alg. 1) for these sequence lengths:
    (container per sequence, block heights, stats dict)."""
    L = np.ascontiguousarray(lengths, dtype=np.int64)
    cont = np.empty(max(1, L.size), np.int32)
    heights = np.empty(int(nblocks), np.int64)
    st = Alg1Stats()
    _check(_lib.hmsv_alg1_pack(_np_ptr(L), L.size, int(nblocks), int(width), _np_ptr(cont),
                               _np_ptr(heights), ctypes.byref(st)), "hmsv_alg1_pack")
    return cont[:L.size], heights, st.as_dict()


def parse_fasta(text: bytes):
    """Protein FASTA bytes -> (headers list[str], residues uint8 [n],
    offsets int64 [nseq + 1]), parsed by the library (hmsv_fasta_parse)."""
    if isinstance(text, str):
        text = text.encode()
    nres, nseq, err = _i64(0), _i64(0), _i64(-1)
    rc = _lib.hmsv_fasta_parse(text, len(text), None, None, None, ctypes.byref(nres),
                               ctypes.byref(nseq), ctypes.byref(err))
    if rc != OK:
        raise HmsvError(rc, f"hmsv_fasta_parse (byte {err.value})")
    res = np.empty(max(1, nres.value), np.uint8)
    off = np.empty(nseq.value + 1, np.int64)
    names = np.empty((max(1, nseq.value), 2), np.int64)
    _check(_lib.hmsv_fasta_parse(text, len(text), _np_ptr(res), _np_ptr(off), _np_ptr(names),
                                 ctypes.byref(nres), ctypes.byref(nseq), ctypes.byref(err)),
           "hmsv_fasta_parse")
    heads = [text[a:a + n].decode(errors="replace") for a, n in names[:nseq.value]]
    return heads, res[:nres.value], off


def read_fasta(path):
    """A protein FASTA file -> (headers, residues, offsets); see parse_fasta."""
    with open(path, "rb") as f:
        return parse_fasta(f.read())


def db_default_plan(db, filt: str, M: int) -> Plan:
    """The plan a call with plan=None uses on this database (the default
    plan, or one whose image fits the LDS with the degenerate rows)."""
    p = Plan()
    _check(_lib.hmsv_db_default_plan(db._h, 1 if filt == "msv" else 0, int(M), ctypes.byref(p)),
           "hmsv_db_default_plan")
    return p


def make_plan(G, Q, waves_per_block=4, blocks=0) -> Plan:
    return Plan(int(G), int(Q), int(waves_per_block), int(blocks))


def plan_for(filt: str, M: int) -> Plan:
    """The library's default plan: the autotuned one (hmsv_default_plan)."""
    return default_plan(filt, M)


def plan_lds_bytes(G, Q) -> int:
    """LDS bytes per workgroup of a plan's kernels (0 for an invalid shape)."""
    return int(_lib.hmsv_plan_lds_bytes(int(G), int(Q)))


def workspace_bytes(nseq: int) -> int:
    """Workspace bytes for scoring calls on a database of nseq sequences."""
    return int(_lib.hmsv_workspace_bytes(int(nseq)))


def new_workspace(device="cuda", nseq: int = 0) -> torch.Tensor:
    return torch.zeros(workspace_bytes(nseq), dtype=torch.uint8, device=device)


def _score(filt, profile: Profile, db: Database, score, flags, workspace, plan, stream,
           rng=None):
    dev = profile.device
    n = db.nseq
    sdt = torch.uint8 if filt == "msv" else torch.int8
    if score is None:
        score = torch.empty(n, dtype=sdt, device=dev)
    if flags is None:
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
    if workspace is None:
        workspace = new_workspace(dev, n)
    if score.dtype != sdt or flags.dtype != torch.uint8:
        raise TypeError("score/flags dtype")
    if score.numel() < n or flags.numel() < n or not score.is_contiguous() \
            or not flags.is_contiguous():
        raise ValueError("score/flags must be contiguous with >= nseq entries")
    if workspace.numel() * workspace.element_size() < workspace_bytes(n):
        raise ValueError("workspace too small")
    for t in (score, flags, workspace):
        if t.device != dev:
            raise ValueError("all tensors must be on the profile's device")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    if plan is None:
        plan = db_default_plan(db, filt, profile.M)
    pl = ctypes.byref(plan) if plan is not None else None
    with torch.cuda.device(dev):
        if rng is None:
            fn = _lib.hmsv_msv_score if filt == "msv" else _lib.hmsv_ssv_score
            _check(fn(ctypes.byref(profile._c), db._h, score.data_ptr(), flags.data_ptr(),
                      workspace.data_ptr(), pl, ctypes.c_void_p(stream.cuda_stream)),
                   f"hmsv_{filt}_score")
        else:
            fn = _lib.hmsv_msv_score_range if filt == "msv" else _lib.hmsv_ssv_score_range
            _check(fn(ctypes.byref(profile._c), db._h, int(rng[0]), int(rng[1]),
                      score.data_ptr(), flags.data_ptr(), workspace.data_ptr(), pl,
                      ctypes.c_void_p(stream.cuda_stream)), f"hmsv_{filt}_score_range")
    return score, flags


def msv_score(profile, db, score=None, flags=None, workspace=None, plan=None, stream=None):
    """MSV filter (paper Alg. 2): uint8 scores and overflow flags per sequence."""
    return _score("msv", profile, db, score, flags, workspace, plan, stream)


NOALLOC_MAX_SEQ = 1 << 20


def msv_score_noalloc(profile, db, score, flags, plan=None, stream=None):
    """MSV filter with the library's own device workspace (no allocation;
    see hmsv_msv_score_noalloc): score and flags are caller-owned uint8
    device tensors of >= nseq entries.  Calls that overlap on one GPU race."""
    dev = profile.device
    n = db.nseq
    if score.dtype != torch.uint8 or flags.dtype != torch.uint8:
        raise TypeError("score/flags dtype")
    if score.numel() < n or flags.numel() < n or not score.is_contiguous() \
            or not flags.is_contiguous() or score.device != dev or flags.device != dev:
        raise ValueError("score/flags must be contiguous on the profile's device with >= nseq "
                         "entries")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    pl = ctypes.byref(plan) if plan is not None else None
    with torch.cuda.device(dev):
        _check(_lib.hmsv_msv_score_noalloc(ctypes.byref(profile._c), db._h, score.data_ptr(),
                                           flags.data_ptr(), pl,
                                           ctypes.c_void_p(stream.cuda_stream)),
               "hmsv_msv_score_noalloc")
    return score, flags


def ssv_score(profile, db, score=None, flags=None, workspace=None, plan=None, stream=None):
    """SSV filter (paper Alg. 7): int8 scores and overflow flags per sequence."""
    return _score("ssv", profile, db, score, flags, workspace, plan, stream)


# ---- P7Viterbi (gapped Viterbi filter, paper Sec. 2.1, Eq. 1) ---------------

P7_UNITS = 32
P7_MAX_M = 2815
P7_TRANSITIONS = ("MM", "MI", "MD", "IM", "II", "DM", "DD")


def p7_quantize(emissions, transitions, bg):
    """Host quantization of a gapped profile (hmsv_p7_quantize): emissions
    [M, 20], transitions [M, 7] (order P7_TRANSITIONS), bg [20] probabilities
    -> dict(msc int16 [32, M], trans int16 [7, M], tbm, M)."""
    e = np.ascontiguousarray(emissions, dtype=np.float64)
    t = np.ascontiguousarray(transitions, dtype=np.float64)
    b = np.ascontiguousarray(bg, dtype=np.float64)
    if e.ndim != 2 or e.shape[1] != K or b.shape != (K,) or t.shape != (e.shape[0], 7):
        raise ValueError("emissions must be [M, 20], transitions [M, 7] and bg [20]")
    M = e.shape[0]
    msc = np.empty((KP, M), np.int16)
    trans = np.empty((7, M), np.int16)
    tb = _i32(0)
    _check(_lib.hmsv_p7_quantize(_np_ptr(e), _np_ptr(t), _np_ptr(b), M, _np_ptr(msc),
                                 _np_ptr(trans), ctypes.byref(tb)), "hmsv_p7_quantize")
    return {"msc": msc, "trans": trans, "tbm": int(tb.value), "M": M}


def p7_length_model(L: int):
    """(loop, move) of the P7 length model for a target of L residues."""
    lo, mv = _i32(0), _i32(0)
    _check(_lib.hmsv_p7_length_model(int(L), ctypes.byref(lo), ctypes.byref(mv)),
           "hmsv_p7_length_model")
    return int(lo.value), int(mv.value)


def p7_lds_bytes(G, Q) -> int:
    """LDS bytes per workgroup of the P7 kernel (G, Q); 0 if invalid."""
    return int(_lib.hmsv_p7_lds_bytes(int(G), int(Q)))


def p7_default_plan(M: int) -> Plan:
    p = Plan()
    _check(_lib.hmsv_p7_default_plan(int(M), ctypes.byref(p)), "hmsv_p7_default_plan")
    return p


class P7Profile:
    """A quantized gapped profile with its tables in device memory."""

    def __init__(self, msc: torch.Tensor, trans: torch.Tensor, tbm: int):
        if msc.dtype != torch.int16 or trans.dtype != torch.int16:
            raise TypeError("msc and trans must be int16")
        if msc.dim() != 2 or msc.shape[0] != KP or trans.shape != (7, msc.shape[1]):
            raise ValueError("msc must be [32, M] and trans [7, M]")
        if msc.device != trans.device:
            raise ValueError("tables must be on one device")
        self.msc = msc.contiguous()
        self.trans = trans.contiguous()
        self.M = int(msc.shape[1])
        self.tbm = int(tbm)
        self.device = self.msc.device
        self._c = _CP7Profile(self.M, self.tbm, self.msc.data_ptr(), self.trans.data_ptr())

    @classmethod
    def from_probabilities(cls, emissions, transitions, bg, device="cuda"):
        q = p7_quantize(emissions, transitions, bg)
        return cls(torch.from_numpy(q["msc"]).to(device), torch.from_numpy(q["trans"]).to(device),
                   q["tbm"])


def p7_score(profile: P7Profile, db: Database, score=None, flags=None, workspace=None,
             plan=None, stream=None):
    """P7Viterbi filter: int16 scores (1/32 bit) and saturation flags per
    sequence, in the database's original order."""
    dev = profile.device
    n = db.nseq
    if score is None:
        score = torch.empty(n, dtype=torch.int16, device=dev)
    if flags is None:
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
    if workspace is None:
        workspace = new_workspace(dev, n)
    if score.dtype != torch.int16 or flags.dtype != torch.uint8:
        raise TypeError("score must be int16 and flags uint8")
    if score.numel() < n or flags.numel() < n or not score.is_contiguous() \
            or not flags.is_contiguous():
        raise ValueError("score/flags must be contiguous with >= nseq entries")
    if workspace.numel() * workspace.element_size() < workspace_bytes(n):
        raise ValueError("workspace too small")
    for t in (score, flags, workspace):
        if t.device != dev:
            raise ValueError("all tensors must be on the profile's device")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    pl = ctypes.byref(plan) if plan is not None else None
    with torch.cuda.device(dev):
        _check(_lib.hmsv_p7_score(ctypes.byref(profile._c), db._h, score.data_ptr(),
                                  flags.data_ptr(), workspace.data_ptr(), pl,
                                  ctypes.c_void_p(stream.cuda_stream)), "hmsv_p7_score")
    return score, flags


def _device_tensor(t, dtype, n, dev, what):
    if t.dtype != dtype or t.numel() < n or not t.is_contiguous() or t.device != dev:
        raise ValueError(f"{what} must be a contiguous {dtype} tensor of >= {n} entries "
                         f"on {dev}")


def select(db: Database, score, flags, filt, threshold, positions=None, count=None,
           workspace=None, stream=None):
    """Survivors of a filter stage (see hmsv_select): the processing-order
    positions of the sequences whose score reaches `threshold` or whose flag
    is set, longest first, and their number, both left on the device."""
    if filt not in ("msv", "ssv"):
        raise ValueError("filt must be 'msv' or 'ssv'")
    dev = score.device
    n = db.nseq
    _device_tensor(score, torch.uint8 if filt == "msv" else torch.int8, n, dev, "score")
    _device_tensor(flags, torch.uint8, n, dev, "flags")
    if positions is None:
        positions = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if count is None:
        count = torch.empty(1, dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = new_workspace(dev, n)
    _device_tensor(positions, torch.int32, n, dev, "positions")
    _device_tensor(count, torch.int32, 1, dev, "count")
    if workspace.device != dev or workspace.numel() * workspace.element_size() \
            < workspace_bytes(n):
        raise ValueError("workspace too small or on another device")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        _check(_lib.hmsv_select(db._h, score.data_ptr(), flags.data_ptr(),
                                1 if filt == "msv" else 0, int(threshold), positions.data_ptr(),
                                count.data_ptr(), workspace.data_ptr(),
                                ctypes.c_void_p(stream.cuda_stream)), "hmsv_select")
    return positions, count


def p7_score_selected(profile: P7Profile, db: Database, positions, count, score, flags,
                      workspace=None, plan=None, stream=None):
    """P7Viterbi on the records at positions[0 .. count) only (see
    hmsv_p7_score_selected): their entries of score/flags (original order)
    are written, every other entry keeps its value."""
    dev = profile.device
    n = db.nseq
    _device_tensor(positions, torch.int32, n, dev, "positions")
    _device_tensor(count, torch.int32, 1, dev, "count")
    _device_tensor(score, torch.int16, n, dev, "score")
    _device_tensor(flags, torch.uint8, n, dev, "flags")
    if workspace is None:
        workspace = new_workspace(dev, n)
    if workspace.device != dev or workspace.numel() * workspace.element_size() \
            < workspace_bytes(n):
        raise ValueError("workspace too small or on another device")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    pl = ctypes.byref(plan) if plan is not None else None
    with torch.cuda.device(dev):
        _check(_lib.hmsv_p7_score_selected(ctypes.byref(profile._c), db._h,
                                           positions.data_ptr(), count.data_ptr(),
                                           score.data_ptr(), flags.data_ptr(),
                                           workspace.data_ptr(), pl,
                                           ctypes.c_void_p(stream.cuda_stream)),
               "hmsv_p7_score_selected")
    return score, flags


class PipelineResult(NamedTuple):
    filter_score: "torch.Tensor"   # uint8 (MSV) / int8 (SSV), original order
    filter_flags: "torch.Tensor"
    positions: "torch.Tensor"      # int32 processing-order positions of the survivors
    count: "torch.Tensor"          # int32 [1]: how many survivors
    p7_score: "torch.Tensor"       # int16, original order; -32768 where not run
    p7_flags: "torch.Tensor"       # uint8; 0 where not run


def pipeline(filt, profile: Profile, p7_profile: P7Profile, db: Database, threshold,
             workspace=None, plan=None, p7_plan=None, stream=None) -> PipelineResult:
    """The filter stage (MSV or SSV) over the whole database, the survivors
    selected on the device, then P7Viterbi on those only: three calls on
    one stream sharing one workspace, no host synchronisation."""
    if filt not in ("msv", "ssv"):
        raise ValueError("filt must be 'msv' or 'ssv'")
    if p7_profile.device != profile.device:
        raise ValueError("profiles on different devices")
    dev = profile.device
    n = db.nseq
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    # outputs allocated on the stream that writes them (the caching
    # allocator reuses a block only after that stream's work on it)
    with torch.cuda.stream(stream):
        if workspace is None:
            workspace = new_workspace(dev, n)
        fs = torch.empty(n, dtype=torch.uint8 if filt == "msv" else torch.int8, device=dev)
        ff = torch.empty(n, dtype=torch.uint8, device=dev)
        pos = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        cnt = torch.empty(1, dtype=torch.int32, device=dev)
        ps = torch.full((n,), -32768, dtype=torch.int16, device=dev)
        pf = torch.zeros(n, dtype=torch.uint8, device=dev)
    fn = msv_score if filt == "msv" else ssv_score
    fn(profile, db, fs, ff, workspace=workspace, plan=plan, stream=stream)
    select(db, fs, ff, filt, threshold, pos, cnt, workspace=workspace, stream=stream)
    p7_score_selected(p7_profile, db, pos, cnt, ps, pf, workspace=workspace, plan=p7_plan,
                      stream=stream)
    return PipelineResult(fs, ff, pos, cnt, ps, pf)


def score_nats(filt, M, score, flags, lengths):
    """Raw scores as log-odds in nats (overflow: +inf); host arrays, one
    entry per sequence, lengths in residues (see hmsv_score_nats)."""
    sc = np.ascontiguousarray(score)
    if sc.dtype.itemsize != 1:
        raise TypeError("scores are one byte each")
    sc = sc.view(np.uint8 if filt == "msv" else np.int8)
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    ln = np.ascontiguousarray(lengths, dtype=np.int64)
    if not (sc.size == fl.size == ln.size):
        raise ValueError("score, flags and lengths must have one entry per sequence")
    out = np.empty(sc.size, dtype=np.float64)
    _check(_lib.hmsv_score_nats(1 if filt == "msv" else 0, int(M), _np_ptr(sc), _np_ptr(fl),
                                _np_ptr(ln), sc.size, _np_ptr(out)), "hmsv_score_nats")
    return out


def gumbel_pvalue(nats, mu, lam):
    """P-values of scores in nats under a Gumbel null with caller-supplied
    location mu and scale lam (see hmsv_gumbel_pvalue)."""
    x = np.ascontiguousarray(nats, dtype=np.float64)
    out = np.empty(x.size, dtype=np.float64)
    _check(_lib.hmsv_gumbel_pvalue(_np_ptr(x), x.size, float(mu), float(lam), _np_ptr(out)),
           "hmsv_gumbel_pvalue")
    return out


def split_info(filt, M, db, plan=None, first=0, count=-1):
    """(split sequences, segments, rows per segment) of a scoring call with
    this filter, profile length and plan on positions [first, first+count)
    of the processing order (count -1: the whole database)."""
    ns, nseg, T = _i32(), _i32(), _i32()
    pl = ctypes.byref(plan) if plan is not None else None
    _check(_lib.hmsv_split_info(db._h, int(first), int(count), 1 if filt == "msv" else 0,
                                int(M), pl, ctypes.byref(ns), ctypes.byref(nseg),
                                ctypes.byref(T)), "hmsv_split_info")
    return ns.value, nseg.value, T.value


def score_range(filt, profile, db, first, count, score, flags, workspace=None, plan=None,
                stream=None):
    """Score positions [first, first+count) of the processing order (see
    Database.order) into the full-size score/flags tensors."""
    return _score(filt, profile, db, score, flags, workspace, plan, stream, (first, count))

