#!/usr/bin/env python3
"""Information throughput of CRC-aided list decoding on one MI355X.

Workload: the (2048, 1723) polar code with a 32-bit CRC (0x04C11DB7) inside K
(1691 payload bits), Bhattacharyya construction at 4.0 dB, list size L = 32,
the Rate-0 / Rate-1 / repetition / SPC-4 decoding tree, BPSK-AWGN frames at
Eb/N0 = 4.0 dB.  One step decodes one batch of frames already resident in
device memory; the value is payload bits decoded per second.

Prints one JSON line (see the keys below).  Extra legs:
  roofline      the decode kernel's algorithmic element rate against the
                VALU issue peak, timed with HIP events on the launch stream;
  cpu_baseline  the oracle timed on a bounded sample of the same frames on
                this host's cores.
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

PAYLOAD = 1723 - 32

# Algorithmic work per frame of this workload (decoding tree at L = 32): F
# outputs, G outputs, leaf-node input reads and scored candidates, summed over
# active paths.  Recomputed from the schedule at run time and checked.
PEAK_ELEM_OPS = 256 * 64 * 2.4e9  # one 32-bit VALU lane-op per element: 39.3e12/s


def work_per_frame(pk, code, L):
    ops = pk.schedule(code.N, code.frozen, L)
    P = 1
    f = g = reads = cands = 0
    cand_per = {"R0": 1, "REP": 2, "SPC": 8 if L != 2 else 2}
    for t, k, _side, paths in ops.tolist():
        name = pk.OP_NAMES[t]
        if name == "F":
            f += P * (1 << (k - 1))
        elif name == "G":
            g += P * (1 << (k - 1))
        elif name != "COMB":
            reads += P * (1 << k)
            c = cand_per.get(name, 2 if k == 0 else 4)
            cands += P * c
            P = paths
    return {"F": int(f), "G": int(g), "leaf_reads": int(reads), "candidates": int(cands),
            "total": int(f + g + reads + cands)}


def cpu_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f32", choices=["f32", "i16", "i8"])
    ap.add_argument("--frames", type=int, default=65536, help="frames per step")
    ap.add_argument("--ebn0", type=float, default=4.0)
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="frames the oracle decodes for the CPU baseline (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: frames are independent, so more GPUs would "
              "split the batch with no exchange; --gpus above 1 is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1505_01466_amd as pk
    import synth

    torch.cuda.set_device(0)
    N, K, r, L = 2048, 1723, 32, 32
    code = synth.make_code(N, K, r, synth.CRC32_POLY, 4.0)
    print(f"[bench] generating {args.frames} frames ({args.dtype}, {args.ebn0} dB)", file=sys.stderr,
          flush=True)
    b = synth.make_batch(code, args.frames, args.ebn0, (20481723, int(args.ebn0 * 100)), args.dtype)
    llr = torch.from_numpy(b.llr).cuda()
    plan = pk.Plan(N, K, code.frozen, code.poly, r, L, args.dtype)
    u_hat = torch.empty((args.frames, K), dtype=torch.uint8, device="cuda")
    crc_ok = torch.empty(args.frames, dtype=torch.uint8, device="cuda")
    pm = torch.empty(args.frames, dtype=torch.float32 if args.dtype == "f32" else torch.int32,
                     device="cuda")

    for _ in range(args.warmup):
        plan.decode(llr, u_hat, crc_ok, pm)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        plan.decode(llr, u_hat, crc_ok, pm)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kernel_ms = float(np.mean([a.elapsed_time(bb) for a, bb in ev]))
    value = args.frames * PAYLOAD / (ms_per_step * 1e-3) / 1e9

    u = u_hat.cpu().numpy()
    fer = float((u != b.info).any(axis=1).mean())

    wk = work_per_frame(pk, code, L)
    achieved = wk["total"] * args.frames / (kernel_ms * 1e-3) / 1e12
    peak = PEAK_ELEM_OPS / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(peak, 2),
            "unit": "Telem-op/s", "frac": round(achieved / peak, 5), "traffic": None,
            "kernel": "pscl::decode_kernel", "kernel_ms": round(kernel_ms, 4),
            "elem_ops_per_frame": wk["total"], "frames_per_launch": args.frames}

    cpu = None
    if args.cpu_sample > 0:
        import oracle

        S = min(args.cpu_sample, args.frames)
        th = cpu_threads()
        print(f"[bench] cpu baseline: oracle on {S} frames, {th} threads", file=sys.stderr, flush=True)
        ts = time.perf_counter()
        ref = oracle.decode_tree(N, K, code.frozen, code.poly, r, L, b.llr[:S], args.dtype,
                                 threads=th)
        te = time.perf_counter()
        agree = int(((ref[0] == u[:S]).all(axis=1) & (ref[1] == crc_ok[:S].cpu().numpy())).sum())
        cpu = {"value": round(S * PAYLOAD / (te - ts) / 1e9, 6), "unit": "Gbps", "cores": th,
               "kind": "oracle",
               "sample": f"first {S} frames of the timed batch, decoder A (tree, L=32, {args.dtype})",
               "seconds": round(te - ts, 3), "gpu_agrees_on_sample": f"{agree}/{S}"}

    info = plan.info()
    out = {
        "metric": "info Gbps @ (2048,1723) CRC32 L=32",
        "value": round(value, 4),
        "unit": "Gbps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic: uniform payloads, CRC-32 inside K, BPSK-AWGN",
        "config": {"workload": "polar (2048,1723) CRC-32 (0x04C11DB7) inside K, Bhattacharyya 4.0 dB, "
                               "L=32, Dec-SPC-4 tree",
                   "frames_per_step": args.frames, "ebn0_db": args.ebn0, "payload_bits": PAYLOAD,
                   "fer": fer, "launch": info},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
