"""Continuous-batching search server over a database resident in HBM.

Requests (a profile of any length, MSV or SSV) arrive at any time.  Each
admitted request owns a slot: output buffers, a workspace, pinned host
buffers and its own stream, all taken from a pool sized by an HBM budget
at start-up (no allocation on the request path besides the profile's
small tables).  A request's search is split into chunks: contiguous ranges
of the database's longest-first processing order holding about
``chunk_cells`` cells each.  The scheduler keeps up to ``depth`` chunks on
the GPU; whenever one finishes it issues the next chunk of the admitted
request with the earliest key "arrival + aging x remaining work / rate"
(FIFO at aging 0, shortest-remaining-work first as aging grows; its own
stream, so chunks of one
request stay ordered and chunks of different requests overlap on the
device), provided the LDS images of the chunks then in flight fit one CU's
LDS together (``lds_budget``) so they can actually co-reside.  Requests
arriving while others run are admitted as soon as a slot frees and join
the rotation at the next chunk boundary.  A finished request's scores are
copied to pinned host memory on its stream and its future is completed.

``Server(..., max_inflight=1, depth=1, chunk_cells=inf)`` is the plain
one-request-per-launch FIFO path used as the comparison baseline.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import math
import threading
import time

import numpy as np
import torch

from . import Profile, Database, db_default_plan, score_range, workspace_bytes, quantize
from .autotune import lds_bytes


def chunk_ranges(cum, nseq, M, chunk_cells):
    """Split the processing order into ranges of about chunk_cells cells for
    a profile of M nodes.  cum[t] = residues of the first t sequences of the
    processing order.  Returns [(first, count), ...] covering 0..nseq."""
    if not math.isfinite(chunk_cells) or cum is None or nseq == 0:
        return [(0, nseq)]
    per = max(1, int(chunk_cells // max(1, M)))            # residues per chunk
    total = int(cum[-1])
    k = max(1, int(math.ceil(total / per)))
    cuts = np.searchsorted(cum, np.linspace(0, total, k + 1)[1:-1])
    edges = [0] + sorted(set(int(c) for c in cuts if 0 < c < nseq)) + [nseq]
    return [(a, b - a) for a, b in zip(edges[:-1], edges[1:])]


def pick_next(active, running_lds, lds_budget, aging, rate):
    """The admitted request whose next chunk goes to the GPU, or None.

    active: requests with chunks left (attributes rid, t_arrival, remaining,
    lds).  running_lds: {request id: LDS bytes} of requests with chunks on
    the GPU.  A request is eligible if it already runs (its chunks stay in
    order on its stream), if nothing runs, or if its LDS image fits beside
    the running ones.  Among eligible requests the earliest
    t_arrival + aging * remaining / rate wins (ties: lowest rid)."""
    used = sum(running_lds.values())
    cands = sorted(active, key=lambda r: (r.t_arrival + aging * r.remaining / rate, r.rid))
    return next((c for c in cands if not running_lds or id(c) in running_lds
                 or used + c.lds <= lds_budget), None)


def slots_for_budget(hbm_budget, bytes_per_slot, max_inflight):
    """Slots the HBM budget allows (at least one)."""
    return max(1, min(max_inflight, int(hbm_budget // bytes_per_slot)))


class Request:
    __slots__ = ("rid", "filt", "profile", "plan", "t_arrival", "t_admit", "t_done",
                 "future", "chunks", "next_chunk", "remaining", "slot", "event", "lds",
                 "cells")

    def __init__(self, rid, filt, profile, plan, t_arrival, table_rows=21):
        self.rid = rid
        self.filt = filt
        self.profile = profile
        self.plan = plan
        self.t_arrival = t_arrival
        self.t_admit = None
        self.t_done = None
        self.future = cf.Future()
        self.future.rid = rid             # lets a caller find the request's record
        self.chunks = []
        self.next_chunk = 0
        self.remaining = 0
        self.slot = None
        self.event = None
        # the image has table_rows rows (27 with degenerate codes) of the
        # 21-row figure's size each
        self.lds = lds_bytes(plan.G, plan.Q) * table_rows // 21
        self.cells = 0


class _Slot:
    def __init__(self, n, device):
        self.score = torch.empty(n, dtype=torch.uint8, device=device)
        self.flags = torch.empty(n, dtype=torch.uint8, device=device)
        self.ws = torch.zeros(workspace_bytes(n), dtype=torch.uint8, device=device)
        self.h_score = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        self.h_flags = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        self.stream = torch.cuda.Stream(device)
        self.busy = False

    @staticmethod
    def bytes_for(n):
        return 2 * n + workspace_bytes(n)


class Server:
    def __init__(self, db: Database, bg, device="cuda", max_inflight=8, depth=2,
                 chunk_cells=2e11, hbm_budget=2 << 30, lds_budget=160 * 1024,
                 poll_s=100e-6, aging=1.0, rate=3.0e13, keep_completed=256):
        self.db = db
        self.bg = np.asarray(bg, dtype=np.float64)
        self.device = torch.device(device)
        n = db.nseq
        self.max_inflight = slots_for_budget(hbm_budget, _Slot.bytes_for(n), max_inflight)
        self.depth = depth
        self.chunk_cells = chunk_cells
        self.lds_budget = lds_budget
        self.poll_s = poll_s
        # priority key = arrival time + aging * remaining cells / rate: aging 0
        # is FIFO, large aging is shortest-remaining-work first; in between,
        # short requests overtake long ones only while the long ones have not
        # waited longer than their own remaining run time (scaled by aging).
        # rate (cells/s) should be the device's measured throughput.
        self.aging = aging
        self.rate = rate
        order = db.order()
        self._order = order
        self._cum = None
        self.set_lengths(db.lengths)
        with torch.cuda.device(self.device):
            self.slots = [_Slot(n, self.device) for _ in range(self.max_inflight)]
        self._queue = collections.deque()      # submitted, not admitted
        self._active = []                      # admitted, chunks left to issue
        self._inflight = []                    # (request, chunk index, event) on the GPU
        self._finishing = []                   # all chunks issued, waiting for D2H
        self._cv = threading.Condition()
        self._stop = False
        self._rid = 0
        # the last keep_completed finished requests (timing fields and the
        # future); their device tables are released at completion
        self.completed = collections.deque(maxlen=keep_completed)
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    # ---- public ------------------------------------------------------------
    def set_lengths(self, lengths):
        """Residues per sequence (original order), used to size chunks."""
        ls = np.asarray(lengths, dtype=np.int64)[self._order]
        self._cum = np.concatenate(([0], np.cumsum(np.maximum(ls, 1))))

    def submit(self, filt: str, emissions, t_arrival=None) -> cf.Future:
        if filt not in ("msv", "ssv"):
            raise ValueError(filt)
        q = quantize(emissions, self.bg)
        prof = Profile(torch.from_numpy(q["cost"]).to(self.device, non_blocking=False),
                       torch.from_numpy(q["sc"]).to(self.device, non_blocking=False), q["dbias"])
        plan = db_default_plan(self.db, filt, prof.M)
        with self._cv:
            self._rid += 1
            r = Request(self._rid, filt, prof, plan,
                        time.perf_counter() if t_arrival is None else t_arrival,
                        self.db.table_rows)
            self._queue.append(r)
            self._cv.notify()
        return r.future

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify()
        self._thread.join()

    # ---- scheduler -----------------------------------------------------------
    def _chunks_for(self, M):
        return chunk_ranges(self._cum, self.db.nseq, M, self.chunk_cells)

    def _admit(self):
        while self._queue:
            slot = next((s for s in self.slots if not s.busy), None)
            if slot is None:
                return
            r = self._queue.popleft()
            slot.busy = True
            r.slot = slot
            r.t_admit = time.perf_counter()
            r.chunks = self._chunks_for(r.profile.M)
            r.cells = r.profile.M * self.db.residues
            r.remaining = r.cells
            self._active.append(r)

    def _chunk_cells(self, r, ci):
        first, count = r.chunks[ci]
        if self._cum is None:
            return r.cells * count // max(1, self.db.nseq)
        return r.profile.M * int(self._cum[first + count] - self._cum[first])

    def _issue(self):
        while len(self._inflight) < self.depth and self._active:
            # LDS of the distinct requests with chunks on the GPU (chunks of one
            # request run in order on its stream and never co-reside)
            running = {id(r): r.lds for r, _, _ in self._inflight}
            r = pick_next(self._active, running, self.lds_budget, self.aging, self.rate)
            if r is None:
                return
            ci = r.next_chunk
            first, count = r.chunks[ci]
            s = r.slot
            score = s.score if r.filt == "msv" else s.score.view(torch.int8)
            with torch.cuda.stream(s.stream):
                score_range(r.filt, r.profile, self.db, first, count, score, s.flags, s.ws,
                            r.plan, s.stream)
                ev = torch.cuda.Event()
                ev.record(s.stream)
            r.next_chunk += 1
            r.remaining -= self._chunk_cells(r, ci)
            self._inflight.append((r, ci, ev))
            if r.next_chunk == len(r.chunks):
                self._active.remove(r)
                with torch.cuda.stream(s.stream):
                    s.h_score.copy_(s.score, non_blocking=True)
                    s.h_flags.copy_(s.flags, non_blocking=True)
                    r.event = torch.cuda.Event()
                    r.event.record(s.stream)
                self._finishing.append(r)

    def _reap(self):
        self._inflight = [(r, ci, ev) for r, ci, ev in self._inflight if not ev.query()]
        done = [r for r in self._finishing if r.event.query()]
        for r in done:
            self._finishing.remove(r)
            r.t_done = time.perf_counter()
            sc = r.slot.h_score.numpy().copy()
            if r.filt == "ssv":
                sc = sc.view(np.int8)
            fl = r.slot.h_flags.numpy().copy()
            r.slot.busy = False
            r.slot = None
            r.profile = None                  # the request's device tables
            self.completed.append(r)
            r.future.set_result((sc, fl))

    def _loop(self):
        with torch.cuda.device(self.device):
            while True:
                with self._cv:
                    if self._stop and not (self._queue or self._active or self._inflight
                                           or self._finishing):
                        return
                    if not (self._queue or self._active or self._inflight or self._finishing):
                        self._cv.wait(timeout=0.05)
                        continue
                    self._admit()
                try:
                    self._issue()
                    self._reap()
                except Exception as e:            # fail every pending request loudly
                    for r in list(self._active) + list(self._finishing) + list(self._queue):
                        if not r.future.done():
                            r.future.set_exception(e)
                    raise
                time.sleep(self.poll_s)


def latency_stats(reqs):
    lat = np.array([r.t_done - r.t_arrival for r in reqs])
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_ms": round(float(lat.mean()) * 1e3, 2), "n": len(reqs)}


def replay(server: Server, arrivals, filters, emissions):
    """Submit each request at its arrival time (seconds from now); wait for all.
    Returns the list of completed Request objects in submission order and
    the wall time from the first arrival to the last completion."""
    t0 = time.perf_counter()
    futs = []
    for t, f, e in zip(arrivals, filters, emissions):
        dt = t0 + t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        futs.append(server.submit(f, e, t_arrival=t0 + t))
    for fu in futs:
        fu.result()
    done = {r.rid: r for r in server.completed}
    if any(fu.rid not in done for fu in futs):
        raise RuntimeError("replay longer than the server keeps completed requests")
    reqs = [done[fu.rid] for fu in futs]
    span = max(r.t_done for r in reqs) - t0
    return reqs, span
