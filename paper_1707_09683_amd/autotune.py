"""Autotuner for launch plans: group width and waves per block.

For each filter and each profile length of a grid of M-bins, every valid
plan is timed on a lognormal database sample with HIP events (mean of
back-to-back launches after one warm-up launch) and the fastest is kept.  All candidates must return identical outputs; a plan
that disagrees with the first one fails the run.  Results are written to
``tuned_plans.json`` keyed by the device (architecture and CU count); the
package's ``plan_for()`` reads them.

Run on the GPU:  python -m paper_1707_09683_amd.autotune [--nseq N]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_plans.json")

M_BINS = (30, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 400, 512, 640, 768, 1024,
          1280, 1536, 2048, 2400, 3072, 3839)
GROUPS = (1, 2, 4, 8, 16, 32, 64)
WAVES = (2, 3, 4, 5, 6, 8)
QMAX = 32
LDS_LIMIT = 160 * 1024


def lds_bytes(G, Q):
    """Bytes of a plan's LDS image, as the library computes it."""
    from . import plan_lds_bytes
    return plan_lds_bytes(G, Q)


def q_for(G, M):
    return (M + 1 + 2 * G - 1) // (2 * G)


def candidates(filt, M):
    for G in GROUPS:
        Q = q_for(G, M)
        if Q > QMAX or lds_bytes(G, Q) > LDS_LIMIT:
            continue
        for wpb in WAVES + ((12, 16) if G >= 32 else ()):
            yield (G, Q, wpb, 0, 64)


def device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}:{p.multi_processor_count}cu"


def load_table():
    if not os.path.exists(TABLE):
        return {}
    with open(TABLE) as fh:
        return json.load(fh)


def lookup(table, key, filt, M):
    """Plan tuple for M from the nearest M-bin (log distance) whose group
    width still fits M; None if the table has nothing usable."""
    ent = table.get(key, {}).get(filt)
    if not ent:
        return None
    bins = sorted(int(k) for k in ent)
    for b in sorted(bins, key=lambda b: abs(math.log(b) - math.log(M))):
        G, _, wpb, blocks, tile = ent[str(b)]
        Q = q_for(G, M)
        if Q <= QMAX and lds_bytes(G, Q) <= LDS_LIMIT:
            return (G, Q, wpb, blocks, tile)
    return None


def tune(nseq=500_000, bins=M_BINS, filters=("msv", "ssv"), reps=4, seed=2, log=print):
    import torch
    import synth
    from . import Profile, Database, msv_score, ssv_score, new_workspace, make_plan

    dev = torch.device("cuda:0")
    st = synth.streams(seed)
    db_np, _ = synth.lognormal_db(seed, nseq, None, 0.0, st)
    db = Database(db_np.res, db_np.offsets, dev)
    ws = new_workspace(dev, db.nseq)
    out = {}
    for filt in filters:
        fn = msv_score if filt == "msv" else ssv_score
        sdt = torch.uint8 if filt == "msv" else torch.int8
        s = torch.empty(db.nseq, dtype=sdt, device=dev)
        f = torch.empty(db.nseq, dtype=torch.uint8, device=dev)
        res = {}
        for M in bins:
            emis = synth.sample_emissions(st["profile"], M)
            prof = Profile.from_emissions(emis, synth.BG, dev)
            ref = None
            best = None
            for cand in candidates(filt, M):
                plan = make_plan(*cand)
                fn(prof, db, s, f, ws, plan)
                torch.cuda.synchronize()
                if ref is None:
                    ref = (s.clone(), f.clone())
                elif not (torch.equal(s, ref[0]) and torch.equal(f, ref[1])):
                    raise RuntimeError(f"plan {cand} disagrees with {best} at {filt} M={M}")
                # back-to-back launches so host enqueue time stays hidden
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fn(prof, db, s, f, ws, plan)
                e1.record()
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) / reps
                if best is None or t < best[0]:
                    best = (t, cand)
            gcups = M * db.residues / (best[0] * 1e-3) / 1e9
            log(f"{filt} M={M}: best {best[1]} {best[0]:.3f} ms {gcups:.0f} GCUPS", flush=True)
            res[str(M)] = list(best[1])
        out[filt] = res
    db.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nseq", type=int, default=500_000)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    t0 = time.time()
    res = tune(a.nseq, reps=a.reps)
    table = load_table() if os.path.exists(a.out) else {}
    table[device_key()] = res
    table.setdefault("_meta", {})[device_key()] = {
        "nseq": a.nseq, "seconds": round(time.time() - t0, 1),
        "note": "fastest plan per (filter, M-bin) on a lognormal database sample"}
    with open(a.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
