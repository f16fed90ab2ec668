#!/usr/bin/env python3
"""Throughput of the MSV filter at M = 400 on one MI355X.

Workload: one M=400 profile (Dirichlet(0.5*bg) emissions) against 500,000
synthetic protein sequences (lognormal lengths, mean ~350, clipped to
20..35000, residues i.i.d. from the background, 1% carrying a segment
emitted by the profile), seed 2.  A step is one full MSV pass of the
profile over the database: the work-queue reset plus the filter kernel,
with the packed database and profile already resident in HBM.

Prints one JSON line: GCUPS (model nodes x real residues / s), the ALU
roofline of the filter kernel (HIP events on its own stream), and the CPU
oracle's throughput on the machine's host cores.  Every output of the timed
runs is compared with the oracle (bit-exact) before the line is printed.
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
# cells per instruction): MSV = max(gamma, scB) + saturating add of
# (dbias - cost) + half of a three-way max into scE -> 2.5 per cell pair;
# SSV = saturating add + half a three-way max -> 1.5 per pair.
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
PEAK_INSTR = CUS * LANES * CLOCK_HZ              # 39.3e12 lane-instructions/s
INSTR_PER_CELL = {"msv": 1.25, "ssv": 0.75}
PAPER_OPS_PER_CELL = {"msv": 4, "ssv": 2}        # 8-bit SIMD ops per cell in the K40 listings


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nseq", type=int, default=500_000)
    ap.add_argument("--filter", choices=["msv", "ssv"], default="msv")
    ap.add_argument("--M", type=int, default=400)
    ap.add_argument("--plan", type=str, default="",
                    help="G,Q,waves_per_block,blocks,tile (default: library's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
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


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the filter shards "
                          "by database sequences with no exchange, see DESIGN.md"}))
        sys.exit(2)
    import torch
    import synth
    import paper_1707_09683_amd as hm

    t0 = time.time()
    if a.filter == "msv" and a.M == 400:
        w = synth.plain_msv_m400(nseq=a.nseq)
        emis, db = w.emissions[0], w.db
        wname = f"msv_m400_{a.nseq // 1000}k_lognormal"
    else:
        base = synth.plain_msv_m400(nseq=a.nseq)
        st = synth.streams(3)
        emis = synth.sample_emissions(st["profile"], a.M)
        db = base.db
        wname = f"{a.filter}_m{a.M}_{a.nseq // 1000}k_lognormal"
    gen_s = time.time() - t0

    dev = torch.device("cuda:0")
    prof = hm.Profile.from_emissions(emis, synth.BG, dev)
    gdb = hm.Database(db.res, db.offsets, dev)
    plan = hm.default_plan(a.filter, a.M) if not a.plan else \
        hm.make_plan(*[int(v) for v in a.plan.split(",")])
    fn = hm.msv_score if a.filter == "msv" else hm.ssv_score
    sdt = torch.uint8 if a.filter == "msv" else torch.int8
    score = torch.empty(gdb.nseq, dtype=sdt, device=dev)
    flags = torch.empty(gdb.nseq, dtype=torch.uint8, device=dev)
    ws = hm.new_workspace(dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(a.warmup):
        fn(prof, gdb, score, flags, ws, plan, stream)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        fn(prof, gdb, score, flags, ws, plan, stream)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    step_ms = [s.elapsed_time(e) for s, e in ev]
    kern_ms = float(np.mean(step_ms))

    cells = a.M * db.residues
    gcups = cells / (wall / a.steps) / 1e9
    achieved = cells / (kern_ms * 1e-3) * INSTR_PER_CELL[a.filter]

    # bit-exact check of the timed outputs against the oracle, and the oracle's
    # own throughput on this host (every sequence of the workload).
    gs, gf = score.cpu().numpy(), flags.cpu().numpy()
    cpu = None
    parity = "not checked"
    if not a.no_cpu_baseline:
        import oracle
        from oracle import quant as oq
        oprof = oq.quantize(emis, synth.BG)
        nthr = a.cpu_threads or max(1, min(16, os.cpu_count() or 1))
        t2 = time.perf_counter()
        es, ef = oracle.score_db(a.filter, oprof, db.res, db.offsets, nthreads=nthr)
        cpu_s = time.perf_counter() - t2
        bad = int(((gs != es) | (gf != ef)).sum())
        parity = "bit-exact" if bad == 0 else f"{bad} mismatches"
        cpu = {"value": round(cells / cpu_s / 1e9, 3), "unit": "GCUPS", "cores": nthr,
               "kind": "oracle",
               "sample": f"all {db.n} sequences of the workload ({cells:.3e} cells), "
                         f"{cpu_s:.1f} s wall"}

    out = {
        "metric": f"{a.filter.upper()} GCUPS at M={a.M} (bit-exact)",
        "value": round(gcups, 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x2 (exact u8/s8 saturating semantics)",
        "data": "synthetic",
        "config": {"workload": wname, "filter": a.filter, "M": a.M, "nseq": db.n,
                   "residues": db.residues, "cells": cells,
                   "plan": list(plan.as_tuple()), "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": round(PEAK_INSTR / 1e12, 2),
                     "unit": "T VALU lane-instr/s",
                     "frac": round(achieved / PEAK_INSTR, 4), "traffic": None,
                     "kernel_ms": round(kern_ms, 4),
                     "instr_per_cell": INSTR_PER_CELL[a.filter],
                     "cell_ceiling_gcups": round(PEAK_INSTR / INSTR_PER_CELL[a.filter] / 1e9)},
        "cpu_baseline": cpu,
        "parity": parity,
        "context": {"paper_k40_gcups": {"msv": 283.9, "ssv": 471.7},
                    "workload_gen_s": round(gen_s, 1)},
    }
    print(json.dumps(out), flush=True)
    gdb.close()
    if parity not in ("bit-exact", "not checked"):
        sys.exit(1)


if __name__ == "__main__":
    main()
