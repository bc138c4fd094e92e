"""Method choice for an accuracy target on one GPU.

    python -m paper_1710_01839_amd.select_study [--n 4096] [--bits 24 48 ...]

For FP64 and double-double inputs and each target of `bits` (normwise:
max |C - AB| <= 2^-bits l max|A| max|B|), the library times every method
whose a-priori bound meets the target (DD / QD block, Winograd-Strassen
depths, the split INT8 product with its slice count: all digit pairs, the
triangle, the residue form) and keeps the fastest.
Printed per target (one JSON line): the choice, the bits its bound
guarantees, its time, the wall time of the choice itself, and the time of
the plain choice (the DD block kernel when its bound meets the target, else
the QD block kernel) with the speedup over it.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

ALGO = {1: "simple", 2: "block", 3: "strassen", 4: "split INT8", 5: "split INT8, residue form of the DD parts"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--bits", type=int, nargs="+", default=[24, 48, 72, 90, 120, 160, 190])
    ap.add_argument("--inputs", type=int, nargs="+", default=[1, 2], help="input limbs: 1 FP64, 2 DD, 4 QD")
    args = ap.parse_args()

    from paper_1710_01839_amd import mpgemm as M

    ctx = M.Context(0)
    T = M.Tuner(ctx)
    n = args.n
    plain = {}
    for prec in (2, 4):
        plain[prec] = T.time(prec, n, n, n, "block", None, reps=3)
    for kind in args.inputs:
        for bits in args.bits:
            t0 = time.perf_counter()
            r = T.select(n, n, n, bits, kind)
            secs = time.perf_counter() - t0
            dd_ok = M.method_bound(kind, 2, "block", None, "all", n, n, n) <= 2.0 ** -bits
            base = plain[2] if dd_ok else plain[4]
            what = ALGO[r["algo"]] + (f" depth {r['tile']['depth']}" if r["algo"] == 3 else "")
            if r["algo"] == 4:
                what += f", {r['tile']['slices']} slices, " + \
                    ("residue form" if r["pairs"] == "crt" else f"{r['pairs']} pairs")
            print(json.dumps({"n": n, "in_limbs": kind, "bits": bits,
                              "choice": f"{'DD' if r['precision'] == 2 else 'QD'} {what}",
                              "bound_bits": round(r["bound_bits"], 1), "ms": round(r["ms"], 3),
                              "select_s": round(secs, 2),
                              "plain": "DD block" if dd_ok else "QD block", "plain_ms": round(base, 3),
                              "speedup": round(base / r["ms"], 2)}), flush=True)
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
