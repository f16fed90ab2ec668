#!/usr/bin/env python3
"""Throughput of the MSV/SSV filters on one MI355X, plus batched and served forms.

Headline workload (value): the MSV filter of one M=400 profile
(Dirichlet(0.5*bg) emissions) against 500,000 synthetic protein sequences
(lognormal lengths, mean ~350, clipped to 20..35000, residues i.i.d. from
the background, 1% carrying a segment emitted by the profile), seed 2.  A
step is one full MSV pass of the profile over the database (the prep kernel
that builds the profile's LDS image and the filter kernel), with the packed
database already resident in HBM.  GCUPS = M x real residues / step time.

The same line also reports:
* ssv: the SSV filter of profiles with M = 100, 400, 1000 and 2400 (seed 3)
  on the same database, each checked in full against the oracle;
* batched: 64 profiles with M ~ U{30..2400}, MSV/SSV alternating, against a
  1,000,000-sequence lognormal database (seed 4), one hipGraph launch vs 64
  sequential plain launches with the same plans (outputs must be identical;
  a sample of sequences per query is checked against the oracle);
* p7: the P7Viterbi filter (the gapped stage, Sec. 2.1, Eq. 1) of
  profiles with M = 100, 400, 1000 and 2400 (seed 3 emissions and
  transitions) on the same database, checked against the oracle on every
  sequence at M = 400 and on a seeded sample of 5,000 sequences at the
  others;
* served: a resident 2,000,000-sequence database (seed 5) and a Poisson
  stream of searches (M ~ U{30..2000}, MSV or SSV), replayed through the
  continuous-batching server and through the plain one-request-per-launch
  FIFO path; QPS = 0.7 x the plain path's measured capacity; p50/p99
  latency (arrival -> results in host memory) and GCUPS for both.

Every output of the timed headline runs is compared bit for bit with the
CPU oracle, which is also timed on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ALU roofline.  MI355X issues one VALU instruction per lane per clock on
# each of 256 CUs x 64 lanes at the 2.4 GHz peak engine clock.  The fewest
# VALU instructions a cell can cost on gfx950's packed 16-bit datapath (two
# cells per instruction): one saturating (clamped) add of the per-node score
# per cell pair, plus half of a three-way max into scE -> 1.5 per pair for
# both filters.  (MSV's max with scB folds into the cell representation
# while scB is fixed: cells are kept relative to scB.)
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
PEAK_INSTR = CUS * LANES * CLOCK_HZ              # 39.3e12 lane-instructions/s
INSTR_PER_CELL = {"msv": 0.75, "ssv": 0.75, "p7": 7.0}
# The same peak counted in the paper's per-cell operations (Alg. 2: four
# 8-bit operations per MSV cell; Alg. 7: two per SSV cell) at two 16-bit
# lanes per packed instruction: 19.7e12 MSV and 39.3e12 SSV cells/s.  The
# kernels exceed this ceiling because gfx950 folds several of those
# operations into one instruction (the clamp modifier saturates the add,
# a three-way max takes two cells into scE, and MSV cells kept relative to
# scB drop the max with scB), so the issue-rate fraction above is the
# meaningful one; this one is reported beside it.
# P7Viterbi (Eq. 1 and the E state): per cell eight saturating adds (the
# three transitions and the emission into M, two into I, two into D) and six
# maxima (three for M, one each for I, D and E), 14 operations; two cells
# per packed int16 instruction gives the 7 instructions per cell above (the
# lazy completion of the D chains comes on top of that floor).
OPS_PER_CELL = {"msv": 4, "ssv": 2, "p7": 14}
OPS_CEILING = {f: PEAK_INSTR * 2 / n for f, n in OPS_PER_CELL.items()}

# HBM bytes per dispatch of the headline kernel come from rocprofv3
# FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB device copy measured the same
# way (profiles/traffic_*.json).  A record is used only if it was taken on
# the current library sources (kernel and database layout) and the same plan
# and workload.
PROFILES = os.path.join(ROOT, "profiles")


def library_source_sha1():
    import glob
    import hashlib
    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1707_09683_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_for(workload, plan):
    import glob
    sha = library_source_sha1()
    for f in glob.glob(os.path.join(PROFILES, "traffic_*.json")):
        rec = json.load(open(f))
        if rec.get("library_source_sha1") == sha and rec.get("workload") == workload \
                and list(rec.get("plan", [])) == list(plan):
            return rec["bytes_per_launch"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nseq", type=int, default=500_000)
    ap.add_argument("--filter", choices=["msv", "ssv", "p7"], default="msv")
    ap.add_argument("--M", type=int, default=400)
    ap.add_argument("--plan", type=str, default="",
                    help="G,Q,waves_per_block,blocks (default: tuned plan)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only (no SSV, batched or served legs)")
    ap.add_argument("--batch-nseq", type=int, default=1_000_000)
    ap.add_argument("--serve-nseq", type=int, default=2_000_000)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--reps", type=int, default=5,
                    help="timed runs of the batched and sequential forms (median)")
    ap.add_argument("--replays", type=int, default=3,
                    help="replays of the served trace per path (median and spread)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


def calibrate_copy(mib: int):
    """One plain copy kernel of known size, so that HBM byte counters
    (FETCH_SIZE / WRITE_SIZE) can be scaled to bytes."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "read_bytes": n, "write_bytes": n}))


def cpu_share():
    """Host threads this process may use: the thread budget the environment
    declares (OMP_NUM_THREADS, a host's share of cores per GPU), else the
    cores in this process's affinity mask."""
    try:
        v = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        v = 0
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else \
        (os.cpu_count() or 1)
    return max(1, min(v, aff) if v > 0 else aff)


def nthreads(a):
    return a.cpu_threads or cpu_share()


def progress(msg):
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_plain(hm, torch, filt, prof, gdb, plan, steps, warmup):
    """Mean wall time per step (back-to-back), mean and median HIP-event time
    per step."""
    dev = prof.device
    fn = {"msv": hm.msv_score, "ssv": hm.ssv_score, "p7": hm.p7_score}[filt]
    sdt = {"msv": torch.uint8, "ssv": torch.int8, "p7": torch.int16}[filt]
    score = torch.empty(gdb.nseq, dtype=sdt, device=dev)
    flags = torch.empty(gdb.nseq, dtype=torch.uint8, device=dev)
    ws = hm.new_workspace(dev, gdb.nseq)
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        fn(prof, gdb, score, flags, ws, plan, stream)
    torch.cuda.synchronize()
    # no collector pauses while the calls are enqueued: a host stall longer
    # than the queued GPU work would show up as idle time between events
    import gc
    gc.collect()
    gc.disable()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t1 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        fn(prof, gdb, score, flags, ws, plan, stream)
        e.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t1) / steps
    gc.enable()
    times = [s.elapsed_time(e) for s, e in ev]
    kern = float(np.mean(times)) * 1e-3
    kern_median = float(np.median(times)) * 1e-3
    return wall, kern, kern_median, score, flags


def layout_leg(hm, h):
    """Padding of the database layouts on the headline database: this
    library's records (each sequence's rows rounded up to the kernel's
    16-row step, or 8 for groups of 16+ lanes) against the paper's
    warp-based blocks (Alg. 1) at the paper's K40 shape (15 SMX x 32 warps,
    128 columns) and at this GPU's (the headline plan's resident wavefronts,
    64/G sequences each).  Host arithmetic only."""
    L = np.asarray(h["db"].lengths, dtype=np.int64)
    G, Q, wpb = h["plan"].G, h["plan"].Q, h["plan"].waves_per_block
    step = 16 if G < 16 else 8
    rows = np.maximum(4, (L + 3) // 4 * 4)
    run = int(((rows + step - 1) // step * step).sum())
    real = int(L.sum())
    out = {"this_layout": {"rows_run": run, "real": real,
                           "padding_to_real": round((run - real) / real, 6),
                           "balance": "dynamic queue; sequences above 1.5x the mean work "
                                      "per lane group are split into segments"}}
    nwaves = 256 * 4 * (4 if G < 64 else 2)
    for name, nb, width in (("alg1_k40_shape", 15 * 32, 128),
                            ("alg1_mi355x_shape", nwaves, 64 // G)):
        _, _, st = hm.alg1_pack(L, nb, width)
        out[name] = {"blocks": nb, "width": width, "prr": round(st["prr"], 7),
                     "mean_height": round(st["mean_height"], 1),
                     "sd_height": round(st["sd_height"], 1),
                     "max_height": st["max_height"],
                     "efficiency": round(st["efficiency"], 4),
                     "mean_ending": round(st["mean_ending"], 1),
                     "sd_ending": round(st["sd_ending"], 2)}
    return out


def headline(a, hm, torch, synth):
    t0 = time.time()
    w = synth.plain_msv_m400(nseq=a.nseq)
    db = w.db
    trans = None
    if a.filter == "msv" and a.M == 400:
        emis = w.emissions[0]
        wname = f"msv_m400_{a.nseq // 1000}k_lognormal"
    elif a.filter == "p7":
        emis, trans = p7_profile(synth, a.M)
        wname = f"p7_m{a.M}_{a.nseq // 1000}k_lognormal"
    else:
        emis = synth.sample_emissions(synth.streams(3)["profile"], a.M)
        wname = f"{a.filter}_m{a.M}_{a.nseq // 1000}k_lognormal"
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    gdb = hm.Database(db.res, db.offsets, dev)
    if a.filter == "p7":
        prof = hm.P7Profile.from_probabilities(emis, trans, synth.BG, dev)
        plan = hm.p7_default_plan(a.M)
    else:
        prof = hm.Profile.from_emissions(emis, synth.BG, dev)
        plan = hm.plan_for(a.filter, a.M)
    if a.plan:
        plan = hm.make_plan(*[int(v) for v in a.plan.split(",")])
    wall, kern, kern_median, score, flags = time_plain(hm, torch, a.filter, prof, gdb, plan,
                                                       a.steps, a.warmup)
    cells = a.M * db.residues
    return {"workload": wname, "db": db, "gdb": gdb, "emis": emis, "trans": trans, "plan": plan,
            "wall": wall, "kern": kern, "kern_median": kern_median, "cells": cells,
            "gen_s": gen_s,
            "score": score.cpu().numpy(), "flags": flags.cpu().numpy()}


def p7_profile(synth, M):
    """Gapped profile of length M: seed-3 emissions, then transitions."""
    rng = synth.streams(3)["profile"]
    emis = synth.sample_emissions(rng, M)
    return emis, synth.sample_transitions(rng, M)


def oracle_check(a, filt, emis, db, gs, gf, synth, ids=None, trans=None):
    import oracle
    from oracle import quant as oq
    from oracle import p7 as op7
    t = time.perf_counter()
    if filt == "p7":
        es, ef = oracle.p7_score_db(op7.quantize(emis, trans, synth.BG), db.res, db.offsets,
                                    ids=ids, nthreads=nthreads(a))
    else:
        es, ef = oracle.score_db(filt, oq.quantize(emis, synth.BG), db.res, db.offsets,
                                 ids=ids, nthreads=nthreads(a))
    dt = time.perf_counter() - t
    if ids is None:
        bad = int(((gs != es) | (gf != ef)).sum())
    else:
        bad = int(((gs[ids] != es[ids]) | (gf[ids] != ef[ids])).sum())
    return bad, dt


def ssv_leg(a, hm, torch, synth, h):
    """SSV on the same 500k database for the four profile lengths of the SSV
    workload (seed 3): throughput, roofline fraction and full oracle parity."""
    w = synth.plain_ssv(db=h["db"])
    out = []
    for emis in w.emissions:
        M = emis.shape[0]
        prof = hm.Profile.from_emissions(emis, synth.BG, h["gdb"].device)
        plan = hm.plan_for("ssv", M)
        wall, kern, kern_med, score, flags = time_plain(hm, torch, "ssv", prof, h["gdb"], plan,
                                                         10, 5)
        cells = M * h["db"].residues
        bad, _ = oracle_check(a, "ssv", emis, h["db"], score.cpu().numpy(),
                              flags.cpu().numpy(), synth)
        out.append({"M": M, "value": round(cells / wall / 1e9, 1), "unit": "GCUPS",
                    "kernel_ms": round(kern * 1e3, 4),
                    "kernel_ms_median": round(kern_med * 1e3, 4),
                    "frac": round(cells / kern * INSTR_PER_CELL["ssv"] / PEAK_INSTR, 4),
                    "ops_frac": round(cells / kern / OPS_CEILING["ssv"], 4),
                    "plan": list(plan.as_tuple()),
                    "parity": "bit-exact" if bad == 0 else f"{bad} mismatches"})
    return {"workload": "ssv_500k_lognormal", "per_M": out}


def p7_leg(a, hm, torch, synth, h):
    """P7Viterbi on the same 500k database for four profile lengths:
    throughput, roofline fraction (7 packed instructions per cell) and oracle
    parity: every sequence at M = 400, a seeded sample of 5,000 sequences at
    the other lengths."""
    out = []
    sub = np.sort(np.random.default_rng(7).choice(h["db"].n, 5000, replace=False))
    for M in (100, 400, 1000, 2400):
        emis, trans = p7_profile(synth, M)
        prof = hm.P7Profile.from_probabilities(emis, trans, synth.BG, h["gdb"].device)
        plan = hm.p7_default_plan(M)
        wall, kern, kern_med, score, flags = time_plain(hm, torch, "p7", prof, h["gdb"], plan,
                                                         5, 2)
        cells = M * h["db"].residues
        full = M == 400
        bad, osec = oracle_check(a, "p7", emis, h["db"], score.cpu().numpy(),
                                 flags.cpu().numpy(), synth, ids=None if full else sub,
                                 trans=trans)
        out.append({"M": M, "value": round(cells / wall / 1e9, 1), "unit": "GCUPS",
                    "kernel_ms": round(kern * 1e3, 4),
                    "kernel_ms_median": round(kern_med * 1e3, 4),
                    "frac": round(cells / kern * INSTR_PER_CELL["p7"] / PEAK_INSTR, 4),
                    "plan": list(plan.as_tuple()),
                    "parity": ("bit-exact" if bad == 0 else f"{bad} mismatches")
                    + (f" (all {h['db'].n} sequences, oracle {osec:.1f} s)" if full
                       else " (5,000-sequence sample, seed 7)")})
    return {"workload": "p7_500k_lognormal", "per_M": out}


def pipeline_leg(a, hm, torch, synth, h, rate=0.022, steps=5, warmup=2):
    """The pipeline of Sec. 2.1 on the headline database: MSV over every
    sequence, the survivors selected on the device (threshold at the score
    that passes about 2.2% of the sequences, the paper's MSV pass rate),
    P7Viterbi on the survivors only; three stages on one stream, one
    workspace, no host synchronisation.  Times each stage with HIP events;
    checks the selection against its definition and the survivors' P7
    scores against the oracle."""
    import oracle
    from oracle import p7 as op7
    M = 400
    emis = h["emis"]
    trans = synth.sample_transitions(np.random.default_rng(400), M)
    dev = h["gdb"].device
    gdb = h["gdb"]
    n = gdb.nseq
    prof = hm.Profile.from_emissions(emis, synth.BG, dev)
    p7 = hm.P7Profile.from_probabilities(emis, trans, synth.BG, dev)
    sc = h["score"].astype(np.int64)
    thr = int(np.ceil(np.quantile(sc, 1.0 - rate)))
    ws = hm.new_workspace(dev, n)
    fs = torch.empty(n, dtype=torch.uint8, device=dev)
    ff = torch.empty(n, dtype=torch.uint8, device=dev)
    pos = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    ps = torch.empty(n, dtype=torch.int16, device=dev)
    pf = torch.empty(n, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    mplan = hm.plan_for("msv", M)
    out = {"workload": "msv_select_p7_m400_500k_lognormal", "M": M, "threshold": thr,
           "per_plan": []}
    # the selected call's own default (64-lane groups), then the full-database
    # default plan and a 32-lane one
    plans = [None, hm.p7_default_plan(M), hm.make_plan(32, 7, 8)]
    for pplan in plans:
        ev = []
        for i in range(warmup + steps):
            e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
            e0.record(stream)
            hm.msv_score(prof, gdb, fs, ff, ws, mplan, stream)
            e1.record(stream)
            hm.select(gdb, fs, ff, "msv", thr, pos, cnt, ws, stream)
            e2.record(stream)
            hm.p7_score_selected(p7, gdb, pos, cnt, ps, pf, ws, pplan, stream)
            e3.record(stream)
            if i >= warmup:
                ev.append((e0, e1, e2, e3))
        torch.cuda.synchronize()
        t = np.array([[x.elapsed_time(y) for x, y in ((e0, e1), (e1, e2), (e2, e3), (e0, e3))]
                      for e0, e1, e2, e3 in ev]) * 1e-3
        ms = np.median(t, axis=0)
        c = int(cnt.cpu()[0])
        sel = pos[:c].cpu().numpy()
        order = gdb.order()
        fsn, ffn = fs.cpu().numpy(), ff.cpu().numpy()
        keep = np.nonzero((ffn[order] != 0) | (fsn[order].astype(np.int64) >= thr))[0]
        sel_ok = np.array_equal(sel, keep)
        ids = order[sel]
        ps_o, pf_o = oracle.p7_score_db(op7.quantize(emis, trans, synth.BG), h["db"].res,
                                        h["db"].offsets, ids=ids, nthreads=nthreads(a))
        psn, pfn = ps.cpu().numpy(), pf.cpu().numpy()
        bad = int(((psn[ids] != ps_o[ids]) | (pfn[ids] != pf_o[ids])).sum())
        surv_res = int(np.asarray(h["db"].lengths)[ids].sum())
        q64 = (M + 128) // 128
        plan_used = (pplan.as_tuple() if pplan is not None
                     else (64, q64, 16 if q64 <= 18 or q64 == 20 else 8, 0))
        out["per_plan"].append({
            "p7_plan": list(plan_used), "survivors": c, "survivor_frac": round(c / n, 5),
            "survivor_residues": surv_res,
            "ms": {"msv": round(ms[0] * 1e3, 4), "select": round(ms[1] * 1e3, 4),
                   "p7": round(ms[2] * 1e3, 4), "total": round(ms[3] * 1e3, 4)},
            "msv_gcups": round(M * h["db"].residues / ms[0] / 1e9, 1),
            "p7_gcups_on_survivors": round(M * surv_res / ms[2] / 1e9, 1),
            "pipeline_gcups": round(M * h["db"].residues / ms[3] / 1e9, 1),
            "selection": "matches its definition" if sel_ok else "MISMATCH",
            "parity": "bit-exact" if bad == 0 else f"{bad} mismatches"})
    out["overlap"] = pipeline_overlap(hm, torch, synth, h, emis, trans, thr)
    return out


def pipeline_overlap(hm, torch, synth, h, emis, trans, thr, nprof=4, reps=3):
    """Several queries through the pipeline: one stream after another, then
    spread over two and three streams, so that one query's P7 stage (bound by its
    longest survivors, a few waves) runs beside the next query's MSV stage.
    Each query owns its buffers and workspace; the scores of both forms must
    be identical."""
    dev = h["gdb"].device
    gdb = h["gdb"]
    rng = np.random.default_rng(401)
    profs = [(emis, trans)] + [(synth.sample_emissions(rng, 400),
                                synth.sample_transitions(rng, 400)) for _ in range(nprof - 1)]
    qs = [(hm.Profile.from_emissions(e, synth.BG, dev),
           hm.P7Profile.from_probabilities(e, t, synth.BG, dev), hm.new_workspace(dev, gdb.nseq))
          for e, t in profs]
    streams = [torch.cuda.current_stream(dev), torch.cuda.Stream(dev), torch.cuda.Stream(dev)]

    def run(nstreams):
        outs = []
        for i, (mp, pp, ws) in enumerate(qs):
            outs.append(hm.pipeline("msv", mp, pp, gdb, thr, workspace=ws,
                                    stream=streams[i % nstreams]))
        return outs

    res = {}
    for ns in (1, 2, 3):
        run(ns)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            outs = run(ns)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[ns] = (float(np.median(ts)), [(o.p7_score.cpu(), o.count.cpu()) for o in outs])
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
               for ns in (2, 3) for a, b in zip(res[1][1], res[ns][1]))
    return {"queries": nprof, "M": 400, "threshold": thr,
            "survivors": [int(c[0]) for _, c in res[1][1]],
            "ms_one_stream": round(res[1][0] * 1e3, 3),
            "ms_two_streams": round(res[2][0] * 1e3, 3),
            "ms_three_streams": round(res[3][0] * 1e3, 3),
            "wall_per_query_ms": round(min(res[2][0], res[3][0]) * 1e3 / nprof, 3),
            "identical_one_vs_two_streams": same}


def _median_spread(xs):
    xs = sorted(xs)
    return {"median": round(float(np.median(xs)), 4), "min": round(xs[0], 4),
            "max": round(xs[-1], 4), "runs": len(xs)}


def batched_leg(a, hm, torch, synth):
    """64 queries against the 1M-sequence database: one graph launch vs 64
    sequential plain launches with the same plans, each timed as the median
    of ``a.reps`` runs; the 8 shortest-profile queries checked against the
    oracle on every sequence, the others on a seeded sample."""
    import paper_1707_09683_amd.batch as hb
    t0 = time.time()
    w = synth.batched(nseq=a.batch_nseq)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    gdb = hm.Database(w.db.res, w.db.offsets, dev)
    profs = [hm.Profile.from_emissions(e, synth.BG, dev) for e in w.emissions]
    queries = list(zip(w.filters, profs))
    b = hb.Batch(queries, gdb, branches=4)
    cells = b.cells()
    b.launch()                                        # warm-up
    torch.cuda.synchronize()
    t_batch = []
    for _ in range(a.reps):
        t = time.perf_counter()
        b.launch()
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - t)
    # 64 sequential plain launches, same plans, one stream
    outs = []
    ws = hm.new_workspace(dev, gdb.nseq)
    for f, p in queries:
        sdt = torch.uint8 if f == "msv" else torch.int8
        outs.append((torch.empty(gdb.nseq, dtype=sdt, device=dev),
                     torch.empty(gdb.nseq, dtype=torch.uint8, device=dev)))

    def sequential():
        for (f, p), plan, (s, fl) in zip(queries, b.plans, outs):
            (hm.msv_score if f == "msv" else hm.ssv_score)(p, gdb, s, fl, ws, plan)

    sequential()                                      # warm-up
    torch.cuda.synchronize()
    t_seq = []
    for _ in range(a.reps):
        t = time.perf_counter()
        sequential()
        torch.cuda.synchronize()
        t_seq.append(time.perf_counter() - t)
    same = all(torch.equal(s, b.scores[i]) and torch.equal(fl, b.flags[i])
               for i, (s, fl) in enumerate(outs))
    # oracle: the 8 shortest profiles on every sequence, the rest on a sample
    Ms = np.array([e.shape[0] for e in w.emissions])
    full = set(np.argsort(Ms, kind="stable")[:8].tolist())
    rng = np.random.default_rng(44)
    ids = np.sort(rng.choice(w.db.n, size=min(10_000, w.db.n), replace=False))
    bad_full = bad_sample = 0
    t_or = time.perf_counter()
    for i, (f, _) in enumerate(queries):
        b2, _ = oracle_check(a, f, w.emissions[i], w.db, b.scores[i].cpu().numpy(),
                             b.flags[i].cpu().numpy(), synth, None if i in full else ids)
        if i in full:
            bad_full += b2
        else:
            bad_sample += b2
    t_or = time.perf_counter() - t_or
    b.close()
    gdb.close()
    tb, ts = float(np.median(t_batch)), float(np.median(t_seq))
    return {"workload": f"batched_64q_{a.batch_nseq // 1000}k_lognormal",
            "queries": len(queries), "cells": cells,
            "batched_gcups": round(cells / tb / 1e9, 1),
            "sequential_plain_gcups": round(cells / ts / 1e9, 1),
            "batched_s": _median_spread(t_batch), "sequential_s": _median_spread(t_seq),
            "speedup": round(ts / tb, 3),
            "identical_to_plain": bool(same),
            "oracle_full": f"{len(full)} queries (M = {sorted(int(Ms[i]) for i in full)}) x "
                           f"all {w.db.n} sequences, "
                           + ("bit-exact" if bad_full == 0 else f"{bad_full} mismatches"),
            "oracle_sample": f"{len(ids)} sequences x {len(queries) - len(full)} queries, "
                             + ("bit-exact" if bad_sample == 0 else f"{bad_sample} mismatches"),
            "oracle_s": round(t_or, 1), "gen_s": round(gen_s, 1)}


def served_leg(a, hm, torch, synth):
    """Poisson trace at 0.7x the plain path's capacity, replayed ``a.replays``
    times through the server and through the plain FIFO path (median and
    spread of p50/p99); a saturated replay (every request at t = 0) of both
    for capacity; the 8 shortest-profile MSV and 8 shortest-profile SSV
    requests checked against the oracle on every sequence."""
    import paper_1707_09683_amd.serve as sv
    t0 = time.time()
    db = synth.served_db(nseq=a.serve_nseq)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    gdb = hm.Database(db.res, db.offsets, dev)
    # capacity of the plain path: mean service time of back-to-back requests
    cal = synth.request_trace(5 + 1000, 8, 1e6)
    plain = sv.Server(gdb, synth.BG, max_inflight=1, depth=1, chunk_cells=float("inf"))
    reqs, span = sv.replay(plain, np.zeros(len(cal[0])), cal[2], cal[3])
    service = span / len(reqs)
    rate = float(np.sum(cal[1])) * db.residues / span          # cells/s, back to back
    qps = 0.7 / service
    arr, Ms, filt, emis = synth.request_trace(5, a.serve_requests, qps)
    cells = int(np.sum(Ms)) * db.residues
    srv = sv.Server(gdb, synth.BG, max_inflight=8, depth=2, chunk_cells=2e11, aging=1.0,
                    rate=rate)
    runs = {"served": [], "plain": []}
    first = {}
    for rep in range(a.replays):
        for name, server in (("plain", plain), ("served", srv)):
            rq, sp = sv.replay(server, arr, filt, emis)
            runs[name].append({**sv.latency_stats(rq), "gcups": cells / sp / 1e9})
            if rep == 0:
                first[name] = [r.future.result() for r in rq]
    # saturated: every request arrives at once; capacity = cells / span
    cap = {}
    for name, server in (("plain", plain), ("served", srv)):
        rq, sp = sv.replay(server, np.zeros(len(arr)), filt, emis)
        cap[name] = round(cells / sp / 1e9, 1)
    plain.close()
    srv.close()
    same = all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
               for x, y in zip(first["plain"], first["served"]))
    # oracle on every sequence for the shortest profiles of each filter
    chosen = []
    for f in ("msv", "ssv"):
        idx = [i for i in range(len(filt)) if filt[i] == f]
        chosen += sorted(idx, key=lambda i: (int(Ms[i]), i))[:8]
    bad = 0
    t_or = time.perf_counter()
    for i in chosen:
        gs, gf = first["served"][i]
        # the oracle's scores: uint8 for MSV, int8 for SSV
        gs = np.asarray(gs).view(np.uint8 if filt[i] == "msv" else np.int8)
        b2, _ = oracle_check(a, filt[i], emis[i], db, gs, np.asarray(gf), synth)
        bad += b2
    t_or = time.perf_counter() - t_or
    gdb.close()

    def summary(rs):
        return {k: _median_spread([r[k] for r in rs]) for k in ("p50_ms", "p99_ms", "gcups")}

    ps, ss = summary(runs["plain"]), summary(runs["served"])
    return {"workload": f"served_{a.serve_nseq // 1000}k_resident",
            "requests": len(arr), "qps": round(qps, 2), "replays": a.replays,
            "plain_service_ms": round(service * 1e3, 2),
            "served": ss, "plain": ps,
            "p50_speedup": round(ps["p50_ms"]["median"] / ss["p50_ms"]["median"], 3),
            "p99_speedup": round(ps["p99_ms"]["median"] / ss["p99_ms"]["median"], 3),
            "saturated_capacity_gcups": cap,
            "identical_alone_vs_mix": bool(same),
            "oracle_full": f"{len(chosen)} requests (8 MSV + 8 SSV, shortest M: "
                           f"{sorted(int(Ms[i]) for i in chosen)}) x all {db.n} sequences, "
                           + ("bit-exact" if bad == 0 else f"{bad} mismatches"),
            "oracle_s": round(t_or, 1), "gen_s": round(gen_s, 1)}


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (the filters shard by "
                          "database sequences with no exchange between GPUs)"}))
        sys.exit(2)
    import torch
    import synth
    import paper_1707_09683_amd as hm

    h = headline(a, hm, torch, synth)
    cells, kern, wall = h["cells"], h["kern"], h["wall"]
    achieved = cells / kern * INSTR_PER_CELL[a.filter]
    cpu = None
    parity = "not checked"
    if not a.no_cpu_baseline:
        progress("oracle on the whole headline workload")
        bad, cpu_s = oracle_check(a, a.filter, h["emis"], h["db"], h["score"], h["flags"],
                                  synth, trans=h["trans"])
        parity = "bit-exact" if bad == 0 else f"{bad} mismatches"
        # one thread on a fixed seeded subset of the same database
        sub = np.sort(np.random.default_rng(2024).choice(h["db"].n, 5000, replace=False))
        sub_cells = a.M * int(h["db"].lengths[sub].sum())
        a1 = argparse.Namespace(**{**vars(a), "cpu_threads": 1})
        bad1, one_s = oracle_check(a1, a.filter, h["emis"], h["db"], h["score"], h["flags"],
                                   synth, ids=sub, trans=h["trans"])
        if bad1:
            parity = f"{bad1} mismatches (single-thread subset)"
        cpu = {"value": round(cells / cpu_s / 1e9, 3), "unit": "GCUPS", "cores": nthreads(a),
               "kind": "oracle",
               "sample": f"all {h['db'].n} sequences of the workload ({cells:.3e} cells), "
                         f"{cpu_s:.1f} s wall on {nthreads(a)} threads",
               "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
               "cpu_share": cpu_share(),
               "single_core_gcups": round(sub_cells / one_s / 1e9, 3),
               "single_core_sample": f"5000 sequences drawn with seed 2024 "
                                     f"({sub_cells:.3e} cells), {one_s:.2f} s"}
    extra = {}
    if not a.no_extra:
        progress("ssv leg")
        extra["ssv"] = ssv_leg(a, hm, torch, synth, h)
        progress("p7 leg")
        extra["p7"] = p7_leg(a, hm, torch, synth, h)
        extra["layout"] = layout_leg(hm, h)
        if a.filter == "msv" and a.M == 400:
            progress("pipeline leg")
            extra["pipeline"] = pipeline_leg(a, hm, torch, synth, h)
    h["gdb"].close()
    if not a.no_extra:
        progress("batched leg")
        extra["batched"] = batched_leg(a, hm, torch, synth)
        progress("served leg")
        extra["served"] = served_leg(a, hm, torch, synth)

    out = {
        # the default line carries the SSV and served legs beside the MSV value
        "metric": ("MSV/SSV GCUPS at M=400 (bit-exact) + served p50/p99 latency vs plain launch"
                   if (a.filter, a.M, a.no_extra) == ("msv", 400, False)
                   else f"{a.filter.upper()} GCUPS at M={a.M} (bit-exact)"),
        "value": round(cells / wall / 1e9, 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("s16x2 (int16 saturating)" if a.filter == "p7"
                  else "f16x2 (exact u8/s8 saturating semantics)"),
        "data": "synthetic",
        "config": {"workload": h["workload"], "filter": a.filter, "M": a.M,
                   "nseq": h["db"].n, "residues": h["db"].residues, "cells": cells,
                   "plan": list(h["plan"].as_tuple()), "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": round(PEAK_INSTR / 1e12, 2),
                     "unit": "T VALU lane-instr/s",
                     "frac": round(achieved / PEAK_INSTR, 4),
                     "traffic": traffic_for(h["workload"], h["plan"].as_tuple()),
                     "kernel_ms": round(kern * 1e3, 4),
                     "kernel_ms_median": round(h["kern_median"] * 1e3, 4),
                     "instr_per_cell": INSTR_PER_CELL[a.filter],
                     "cell_ceiling_gcups": round(PEAK_INSTR / INSTR_PER_CELL[a.filter] / 1e9),
                     "ops_per_cell": OPS_PER_CELL[a.filter],
                     "ops_ceiling_gcups": round(OPS_CEILING[a.filter] / 1e9),
                     "ops_frac": round(cells / kern / OPS_CEILING[a.filter], 4)},
        "cpu_baseline": cpu,
        "parity": parity,
        **extra,
        "context": {"paper_k40_gcups": {"msv": 283.9, "ssv": 471.7},
                    "workload_gen_s": round(h["gen_s"], 1)},
    }
    print(json.dumps(out), flush=True)
    bad_legs = [k for k, v in extra.items()
                if ("parity" in v and v["parity"] != "bit-exact")
                or v.get("identical_to_plain") is False
                or v.get("identical_alone_vs_mix") is False
                or ("oracle_sample" in v and "mismatch" in v["oracle_sample"])
                or ("oracle_full" in v and "mismatch" in v["oracle_full"])
                or any(not m.get("parity", "bit-exact").startswith("bit-exact")
                       for m in v.get("per_M", []))
                or any(m["parity"] != "bit-exact" or m["selection"] != "matches its definition"
                       for m in v.get("per_plan", []))
                or v.get("overlap", {}).get("identical_one_vs_two_streams") is False]
    if parity not in ("bit-exact", "not checked") or bad_legs:
        sys.exit(1)


if __name__ == "__main__":
    main()
