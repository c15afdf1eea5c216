#!/usr/bin/env python3
"""Operating points of the mixed-code workload: for each of its 45 codes
(N in {256..4096} x rate in {1/3, 1/2, 0.84} x L in {2, 8, 32}, CRC inside
K, int8 LLRs), the Eb/N0 on a 0.05 dB grid at which the frame error rate
reaches 1e-3, found by bisection with 200,000 device-made frames per probe
(Philox payloads and noise, see pscl_generate) decoded by the library.

The point kept for a code is the lowest grid value whose measured FER is at
most 1e-3.  Writes c4_points.json next to this file (bench.py's mixed-launch
leg reads it).  Needs the GPU:

    python c4_points.py [--frames 200000] [--target 1e-3]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(ROOT, "c4_points.json")
GRID = 0.05


def fer(pk, torch, gen, plan, ebn0, frames, seed, chunk=65536):
    errs = done = 0
    llr = info = None
    while done < frames:
        F = min(chunk, frames - done)
        llr, info = gen.generate(F, ebn0, seed, first_frame=done,
                                 llr=None if llr is None else llr[:F],
                                 info=None if info is None else info[:F])
        u, _, _ = plan.decode(llr[:F])
        errs += int((u != info[:F]).any(dim=1).sum().item())
        done += F
    return errs / frames


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--frames", type=int, default=200000)
    ap.add_argument("--target", type=float, default=1e-3)
    ap.add_argument("--lo", type=float, default=-1.0)
    ap.add_argument("--hi", type=float, default=7.0)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()

    import torch

    import paper_1505_01466_amd as pk
    import synth
    from bench import c4_codes

    torch.cuda.set_device(0)
    rows = []
    t0 = time.time()
    for i, (code, L, design) in enumerate(c4_codes(synth)):
        gen = pk.Generator(code.N, code.K, code.frozen, code.poly, code.r, "i8")
        plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, L, "i8")
        seed = 0x43340000 + i
        # grid indices: lo_i fails the target (or is the range's bottom),
        # hi_i meets it
        lo_i, hi_i = 0, int(round((a.hi - a.lo) / GRID))
        at = lambda j: round(a.lo + j * GRID, 4)  # noqa: E731
        probes = {}
        f_hi = fer(pk, torch, gen, plan, at(hi_i), a.frames, seed)
        probes[at(hi_i)] = f_hi
        if f_hi > a.target:
            raise SystemExit(f"code {i}: FER {f_hi} above the target at {at(hi_i)} dB")
        while hi_i - lo_i > 1:
            mid = (lo_i + hi_i) // 2
            f = fer(pk, torch, gen, plan, at(mid), a.frames, seed)
            probes[at(mid)] = f
            if f <= a.target:
                hi_i = mid
            else:
                lo_i = mid
        row = {"N": code.N, "K": code.K, "crc": code.r, "L": L, "rate": round(code.K / code.N, 4),
               "design_ebn0_db": design, "ebn0_db": at(hi_i), "fer": probes[at(hi_i)],
               "frames_per_probe": a.frames,
               "probes": {str(k): v for k, v in sorted(probes.items())}}
        rows.append(row)
        print(f"[{i + 1}/45] N={code.N} K={code.K} L={L}: {row['ebn0_db']} dB, FER {row['fer']:.2e} "
              f"({len(probes)} probes, {time.time() - t0:.0f} s)", flush=True)
        gen.close()
        plan.close()
    with open(a.out, "w") as fh:
        json.dump({"what": "Eb/N0 (dB) at FER <= target per code of the mixed workload, int8 LLRs",
                   "target_fer": a.target, "grid_db": GRID, "frames_per_probe": a.frames,
                   "codes": rows}, fh, indent=1)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
