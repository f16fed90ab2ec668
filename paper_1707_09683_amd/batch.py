"""Batched launches: many profiles against one resident database in one graph launch.

Thin wrapper over ``hmsv_batch_create`` / ``hmsv_batch_launch``: the C
library captures every query's (prep, filter) kernels, each with its own
plan, into one hipGraph with independent branches; one launch runs the
whole batch.  Output buffers and workspaces are torch tensors owned here.
"""
from __future__ import annotations

import ctypes

import torch

from . import (_CProfile, Plan, Profile, Database, _lib, _check, workspace_bytes,
               db_default_plan)


class _CQuery(ctypes.Structure):
    _fields_ = [("is_msv", ctypes.c_int32), ("prof", _CProfile),
                ("score", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("plan", Plan)]


_lib.hmsv_batch_create.restype = ctypes.c_int
_lib.hmsv_batch_create.argtypes = [ctypes.POINTER(_CQuery), ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
_lib.hmsv_batch_launch.restype = ctypes.c_int
_lib.hmsv_batch_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.hmsv_batch_destroy.restype = None
_lib.hmsv_batch_destroy.argtypes = [ctypes.c_void_p]


class Batch:
    """``queries``: list of (filter, Profile) with filter "msv" or "ssv".

    ``plans``: optional list of Plan (None entries = tuned/default plan).
    After ``launch()`` and a stream sync, ``scores[i]`` / ``flags[i]`` hold
    query i's results in the database's original sequence order."""

    def __init__(self, queries, db: Database, branches: int = 4, plans=None):
        if not queries:
            raise ValueError("empty batch")
        dev = queries[0][1].device
        n = db.nseq
        self.db = db
        self.queries = list(queries)
        self.scores, self.flags, self.workspaces, self.plans = [], [], [], []
        arr = (_CQuery * len(queries))()
        for i, (filt, prof) in enumerate(queries):
            if filt not in ("msv", "ssv"):
                raise ValueError(f"filter {filt!r}")
            if prof.device != dev:
                raise ValueError("all profiles must be on one device")
            sdt = torch.uint8 if filt == "msv" else torch.int8
            s = torch.empty(n, dtype=sdt, device=dev)
            f = torch.empty(n, dtype=torch.uint8, device=dev)
            ws = torch.zeros(workspace_bytes(n), dtype=torch.uint8, device=dev)
            p = plans[i] if plans is not None and plans[i] is not None \
                else db_default_plan(db, filt, prof.M)
            self.scores.append(s)
            self.flags.append(f)
            self.workspaces.append(ws)
            self.plans.append(p)
            arr[i].is_msv = 1 if filt == "msv" else 0
            arr[i].prof = prof._c
            arr[i].score = s.data_ptr()
            arr[i].flags = f.data_ptr()
            arr[i].workspace = ws.data_ptr()
            arr[i].plan = p if p is not None else Plan()
        self._arr = arr
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(_lib.hmsv_batch_create(arr, len(queries), db._h, int(branches),
                                          ctypes.byref(h)), "hmsv_batch_create")
        self._h = h
        self.device = dev

    def launch(self, stream=None):
        stream = stream or torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            _check(_lib.hmsv_batch_launch(self._h, ctypes.c_void_p(stream.cuda_stream)),
                   "hmsv_batch_launch")

    def cells(self) -> int:
        return sum(p.M for _, p in self.queries) * self.db.residues

    def close(self):
        if getattr(self, "_h", None):
            _lib.hmsv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
