"""Build libhmsv.so for gfx950 with hipcc (in-tree).

The kernel template is compiled once per (group width G, range of Q) so the
instantiations build in parallel; the host code is one more translation
unit.  Usage: ``python paper_1707_09683_amd/build.py [--jobs N] [--incremental]``
(run as a file: importing the package needs the library this script builds).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhmsv.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# The atomic optimizer rewrites the work-queue atomic into a wave reduction
# that reads its result back at once; the kernels defer that read to the
# next sequence switch, so the rewrite is turned off.
COMMON = ["-O3", f"--offload-arch={ARCH}", "-std=c++20", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
          "-I", CSRC, "-I", INCLUDE, "-Wno-unused-command-line-argument"]

# (G, largest Q).  The LDS table is 21 rows x G x Q dwords and must fit in
# 160 KiB, which caps G = 64 at Q = 30 (profiles up to 3840 nodes).
GROUPS = ((1, 32), (2, 32), (4, 32), (8, 32), (16, 32), (32, 32), (64, 30))
QCHUNK = 4
# P7Viterbi kernels: (G, largest Q); 28 table rows cap G = 64 at Q = 22.
P7_GROUPS = ((4, 16), (8, 16), (16, 16), (32, 16), (64, 22))


def kernel_units():
    units = []
    for G, qmax in GROUPS:
        for lo in range(1, qmax + 1, QCHUNK):
            hi = min(qmax, lo + QCHUNK - 1)
            units.append((G, lo, hi))
    return units


def _deps_hash(extra):
    h = hashlib.sha1()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    with open(os.path.join(INCLUDE, "hmsv.h"), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join(COMMON + extra).encode())
    return h.hexdigest()


def _compile(cmd, out, stamp, incremental):
    if incremental and os.path.exists(out) and os.path.exists(out + ".stamp"):
        if open(out + ".stamp").read() == stamp:
            return out, 0.0, ""
    import time
    t0 = time.time()
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{p.stderr}")
    with open(out + ".stamp", "w") as fh:
        fh.write(stamp)
    return out, time.time() - t0, p.stderr


def write_tuned_header() -> str:
    """csrc/tuned_plans.inc from tuned_plans.json (autotune.py, loaded by
    path: importing the package needs the library being built)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("hmsv_autotune",
                                                  os.path.join(HERE, "autotune.py"))
    at = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(at)
    return at.write_header()


def build(jobs: int | None = None, incremental: bool = False, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    write_tuned_header()
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    tasks = []
    host_obj = os.path.join(OBJ, "hmsv_host.o")
    host_cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, "hmsv_host.cpp"),
                "-o", host_obj]
    tasks.append((host_cmd, host_obj, _deps_hash(["host"])))
    for G, qmax in P7_GROUPS:
        for lo in range(1, qmax + 1, QCHUNK):
            hi = min(qmax, lo + QCHUNK - 1)
            obj = os.path.join(OBJ, f"p7_g{G}_q{lo}_{hi}.o")
            defs = [f"-DHMSV_G={G}", f"-DHMSV_QLO={lo}", f"-DHMSV_QHI={hi}"]
            cmd = [HIPCC, *COMMON, *defs, "-c", os.path.join(CSRC, "p7.hip"), "-o", obj]
            tasks.append((cmd, obj, _deps_hash(["p7", *defs])))
    exact_obj = os.path.join(OBJ, "exact.o")
    tasks.append(([HIPCC, *COMMON, "-c", os.path.join(CSRC, "exact.hip"), "-o", exact_obj],
                  exact_obj, _deps_hash(["exact"])))
    select_obj = os.path.join(OBJ, "select.o")
    tasks.append(([HIPCC, *COMMON, "-c", os.path.join(CSRC, "select.hip"), "-o", select_obj],
                  select_obj, _deps_hash(["select"])))
    for G, lo, hi in kernel_units():
        obj = os.path.join(OBJ, f"kernels_g{G}_q{lo}_{hi}.o")
        defs = [f"-DHMSV_G={G}", f"-DHMSV_QLO={lo}", f"-DHMSV_QHI={hi}"]
        cmd = [HIPCC, *COMMON, *defs, "-c", os.path.join(CSRC, "kernels.hip"), "-o", obj]
        tasks.append((cmd, obj, _deps_hash(defs)))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, c, o, s, incremental) for c, o, s in tasks]
        for f in futs:
            o, dt, err = f.result()
            objs.append(o)
            if verbose:
                print(f"  {os.path.basename(o)}: {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
                           *objs])
    os.replace(tmp, LIB)
    return LIB


def resources(jobs: int | None = None) -> str:
    """Compiler resource usage of the tuned plans' filter kernels (and the
    exact pass and the default P7Viterbi plans), as a
    markdown table: VGPRs, SGPRs, scratch and the occupancy the compiler
    reports, the LDS image, and the wavefronts per SIMD the launch gets
    (VGPRs, LDS and waves per block together).  Compiles the kernel units
    again with -Rpass-analysis=kernel-resource-usage (no library is built)."""
    import json
    import re
    import tempfile
    table = json.load(open(os.path.join(HERE, "tuned_plans.json")))
    key = next(k for k in table if not k.startswith("_"))
    want = {}
    for filt in ("msv", "ssv"):
        for M, (G, Q, wpb, _b) in table[key][filt].items():
            want.setdefault((filt, G, Q), []).append((int(M), wpb))
    units = sorted({(G, lo, hi) for _f, G, Q in want for (GG, lo, hi) in kernel_units()
                    if GG == G and lo <= Q <= hi})
    rx = re.compile(r"remark:\s+(Function Name|VGPRs|TotalSGPRs|ScratchSize \[bytes/lane\]|"
                    r"Occupancy \[waves/SIMD\]): (\S+)")
    usage = {}

    def one(unit):
        G, lo, hi = unit
        with tempfile.TemporaryDirectory() as td:
            cmd = [HIPCC, *COMMON, f"-DHMSV_G={G}", f"-DHMSV_QLO={lo}", f"-DHMSV_QHI={hi}",
                   "--cuda-device-only", "-c", os.path.join(CSRC, "kernels.hip"),
                   "-o", os.path.join(td, "k.o"), "-Rpass-analysis=kernel-resource-usage"]
            return subprocess.run(cmd, capture_output=True, text=True).stderr

    def exact_unit():
        with tempfile.TemporaryDirectory() as td:
            cmd = [HIPCC, *COMMON, "--cuda-device-only", "-c", os.path.join(CSRC, "exact.hip"),
                   "-o", os.path.join(td, "x.o"), "-Rpass-analysis=kernel-resource-usage"]
            return subprocess.run(cmd, capture_output=True, text=True).stderr

    exact = {}
    cur = None
    for m in rx.finditer(exact_unit()):
        k, v = m.group(1), m.group(2)
        if k == "Function Name":
            mm = re.search(r"exact_kernelILi(\d+)ELi(\d+)E", v)
            cur = int(mm.group(1)) if mm else None
            if cur:
                exact[cur] = {}
        elif cur:
            exact[cur][k] = int(v)
    with cf.ThreadPoolExecutor(max_workers=jobs or 8) as ex:
        for err in ex.map(one, units):
            cur = None
            for m in rx.finditer(err):
                k, v = m.group(1), m.group(2)
                if k == "Function Name":
                    mm = re.search(r"filter_kernelILi(\d+)ELi(\d+)ELi(\d)ELi(\d+)E", v)
                    cur = (("msv" if mm.group(3) == "1" else "ssv"), int(mm.group(1)),
                           int(mm.group(2)), int(mm.group(4))) if mm else None
                    if cur:
                        usage[cur] = {}
                elif cur:
                    usage[cur][k] = int(v)
    sys.path.insert(0, ROOT)
    from paper_1707_09683_amd import plan_lds_bytes
    lines = ["| filter | M-bins | G | Q | waves/block | VGPRs | SGPRs | scratch B/lane | "
             "waves/SIMD (VGPRs) | LDS KiB/block | waves/SIMD (launch) |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for (filt, G, Q), uses in sorted(want.items(), key=lambda t: (t[0][0], min(t[1])[0])):
        lds = plan_lds_bytes(G, Q)
        for wpb in sorted({w for _m, w in uses}):
            u = usage.get((filt, G, Q, 1024 if wpb > 8 else 512), {})
            bins = ",".join(str(m) for m, w in sorted(uses) if w == wpb)
            occ_v = u.get("Occupancy [waves/SIMD]", 0)
            blocks = min(160 * 1024 // lds, (4 * occ_v) // wpb) if lds else 0
            lines.append(f"| {filt} | {bins} | {G} | {Q} | {wpb} | {u.get('VGPRs')} | "
                         f"{u.get('TotalSGPRs')} | {u.get('ScratchSize [bytes/lane]')} | "
                         f"{occ_v} | {lds / 1024:.1f} | {blocks * wpb / 4:g} |")
    lines += ["", "MSV exact pass (`exact_kernel<QX>`, 64-lane groups, blocks of 4 wavefronts; "
              "QX = ceil((M + 1) / 128)):", "",
              "| QX | M up to | VGPRs | SGPRs | scratch B/lane | waves/SIMD (VGPRs) | "
              "LDS KiB/block |", "|---|---|---|---|---|---|---|"]
    for qx in sorted(exact):
        u = exact[qx]
        lines.append(f"| {qx} | {128 * qx - 1} | {u.get('VGPRs')} | {u.get('TotalSGPRs')} | "
                     f"{u.get('ScratchSize [bytes/lane]')} | {u.get('Occupancy [waves/SIMD]')} | "
                     f"{plan_lds_bytes(64, qx) / 1024:.1f} |")
    # P7Viterbi: the default plans at the measured profile lengths
    from paper_1707_09683_amd import p7_default_plan, p7_lds_bytes
    p7_bins = (30, 64, 100, 200, 400, 700, 1000, 1100, 1500, 2047, 2200, 2400, 2815)
    p7_plans = {}
    for M in p7_bins:
        pl = p7_default_plan(M)
        p7_plans.setdefault((pl.G, pl.Q, pl.waves_per_block), []).append(M)

    def p7_unit(gq):
        G, Q = gq
        with tempfile.TemporaryDirectory() as td:
            cmd = [HIPCC, *COMMON, f"-DHMSV_G={G}", f"-DHMSV_QLO={Q}", f"-DHMSV_QHI={Q}",
                   "--cuda-device-only", "-c", os.path.join(CSRC, "p7.hip"),
                   "-o", os.path.join(td, "p.o"), "-Rpass-analysis=kernel-resource-usage"]
            return gq, subprocess.run(cmd, capture_output=True, text=True).stderr

    p7_use = {}
    with cf.ThreadPoolExecutor(max_workers=jobs or 8) as ex:
        for (G, Q), err in ex.map(p7_unit, sorted({(g, q) for g, q, _w in p7_plans})):
            cur = None
            for m in rx.finditer(err):
                k, v = m.group(1), m.group(2)
                if k == "Function Name":
                    mm = re.search(r"p7_kernelILi\d+ELi\d+ELi(\d+)E", v)
                    cur = (G, Q, int(mm.group(1))) if mm else None
                    if cur:
                        p7_use[cur] = {}
                elif cur:
                    p7_use[cur][k] = int(v)
    lines += ["", "P7Viterbi (`p7_kernel<G, Q, threads>`, default plans at the measured lengths; "
              "blocks of 16 wavefronts are 1024-thread kernels):",
              "", "| M-bins | G | Q | waves/block | VGPRs | SGPRs | scratch B/lane | "
              "waves/SIMD (VGPRs) | LDS KiB/block | waves/SIMD (launch) |",
              "|---|---|---|---|---|---|---|---|---|---|"]
    for (G, Q, wpb), Ms in sorted(p7_plans.items(), key=lambda t: min(t[1])):
        u = p7_use.get((G, Q, 1024 if wpb > 8 else 512), {})
        lds = p7_lds_bytes(G, Q)
        occ_v = u.get("Occupancy [waves/SIMD]", 0)
        blocks = min(160 * 1024 // lds, (4 * occ_v) // wpb) if lds else 0
        lines.append(f"| {','.join(map(str, Ms))} | {G} | {Q} | {wpb} | {u.get('VGPRs')} | "
                     f"{u.get('TotalSGPRs')} | {u.get('ScratchSize [bytes/lane]')} | {occ_v} | "
                     f"{lds / 1024:.1f} | {blocks * wpb / 4:g} |")
    return "\n".join(lines)


def clean():
    shutil.rmtree(OBJ, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--resources", action="store_true",
                    help="print the tuned plans' compiler resource usage instead of building")
    a = ap.parse_args()
    if a.resources:
        print(resources(a.jobs))
        sys.exit(0)
    print(build(a.jobs, a.incremental, a.verbose))
    sys.exit(0)
