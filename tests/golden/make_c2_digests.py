"""Writes tests/golden/c2_oracle_digests.jsonl: for every sub-chunk of the
full-scale (2048,1723) CRC-32 L=32 parity workload (tests/scale_parity.py),
the oracle's (decoder A) output digest, its frame errors against the sent
bits, its CRC failures and its near-tie count.  Calls only the oracle and the
input generator.  Resumable: sub-chunks already in the file are skipped, one
line is appended per finished sub-chunk.

    python tests/golden/make_c2_digests.py [--workers W] [--subs S]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import scale_parity as sp  # noqa: E402


def _task(args):
    import numpy as np

    import oracle

    pi, sub = args
    c = sp.code()
    info, llr = sp.frames(pi, sub)
    out = []
    for dt in sp.DTYPES:
        t = time.time()
        u, ok, pm, nt = oracle.decode_tree(c.N, c.K, c.frozen, c.poly, c.r, sp.L, llr[dt], dt,
                                           threads=1)
        out.append({"key": sp.key(dt, pi, sub), "frames": int(u.shape[0]),
                    "digest": sp.digest(u, ok, pm, dt),
                    "errors": int((u != info).any(axis=1).sum()),
                    "crc_fail": int((ok == 0).sum()), "near_tie": int(nt.sum()),
                    "seconds": round(time.time() - t, 1)})
        del u, ok, pm, nt
    del info, llr
    np.random.default_rng()  # keep the worker's imports warm
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--subs", type=int, default=sp.SUBS)
    ap.add_argument("--out", default=sp.DIGESTS)
    a = ap.parse_args()
    done = sp.load_digests(a.out)
    todo = [(pi, s) for s in range(a.subs) for pi in range(len(sp.POINTS))
            if any(sp.key(dt, pi, s) not in done for dt in sp.DTYPES)]
    print(f"{len(todo)} sub-chunks to decode with {a.workers} workers", flush=True)
    with Pool(a.workers, maxtasksperchild=4) as pool, open(a.out, "a") as fh:
        for recs in pool.imap_unordered(_task, todo):
            for rec in recs:
                fh.write(json.dumps(rec, sort_keys=True) + "\n")
            fh.flush()
            print(" ".join(f"{r['key']} err={r['errors']} nt={r['near_tie']} {r['seconds']}s"
                           for r in recs), flush=True)


if __name__ == "__main__":
    main()
