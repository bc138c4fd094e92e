"""Exact long-integer (fixed-point) matrix product on one GPU: the analog of
the paper's 128- to 2048-bit runs.

    python -m paper_1710_01839_amd.int_study [--n 1024] [--bits 128 256 512 1024 2048]

For each operand size (uniformly random two's complement words, both
operands the same size) at n x n x n and each candidate plan (chunk width,
Karatsuba depth): wall time per product, the INT8 product launches' total
time and the other launches' (residue planes, chunk sums, reconstruction),
the count of INT8 products of n^3 (chunk pairs x moduli) and their rate, and
exact multiply-adds per second (n^3 / t).  One JSON line per size and plan.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

INT8_PEAK_TOPS = 5000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--bits", type=int, nargs="+", default=[128, 256, 512, 1024, 2048])
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()

    import numpy as np
    import torch
    from paper_1710_01839_amd import mpgemm as M

    ctx = M.Context(0)
    g = np.random.default_rng(2048)
    n = args.n
    for bits in args.bits:
        w = bits // 32
        A = torch.as_tensor(g.integers(0, 1 << 32, size=(w, n, n), dtype=np.uint64).astype(np.uint32)
                            .view(np.int32)).cuda()
        B = torch.as_tensor(g.integers(0, 1 << 32, size=(w, n, n), dtype=np.uint64).astype(np.uint32)
                            .view(np.int32)).cuda()
        wc = M.int_words_needed(w, w, n)
        C = torch.empty((wc, n, n), dtype=torch.int32, device="cuda")
        for plan in M.int_candidates(w, w, n):
            M.int_gemm(ctx, A, B, C, plan)
            torch.cuda.synchronize()
            ctx.prof_enable(True)
            t0 = time.perf_counter()
            for _ in range(args.reps):
                M.int_gemm(ctx, A, B, C, plan)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.reps * 1e3
            gms, gn = ctx.prof_read(M.MPG_KCLASS_GEMM)
            ams, _ = ctx.prof_read(M.MPG_KCLASS_AUX)
            ctx.prof_enable(False)
            moduli = int(M._lib.mpg_ozaki_last_moduli(ctx.handle))
            products = M.int_products(w, w, n, plan)
            gemm_ms = gms / args.reps
            tops = products * 2.0 * n ** 3 / (gemm_ms * 1e-3) / 1e12
            print(json.dumps({"bits": bits, "n": n, "plan": plan, "words_out": wc, "moduli": moduli,
                              "int8_products": products, "wall_ms": round(wall, 3), "int8_ms": round(gemm_ms, 3),
                              "other_ms": round(ams / args.reps, 3), "int8_tops": round(tops, 1),
                              "frac_int8_peak": round(tops / INT8_PEAK_TOPS, 4),
                              "exact_madds_per_s": float(f"{n ** 3 / (wall * 1e-3):.4g}")}), flush=True)
        del A, B, C
        torch.cuda.empty_cache()
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
