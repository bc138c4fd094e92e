"""Quad-double GEMM and the batched double-double workload on one GPU.

    python -m paper_1710_01839_amd.gemm_study [--qd 512 1024 2048] [--batch 512]

QD: every built QD tile alone, then Winograd-Strassen depth 1 and 2 over
the default tile, and the residue form of the split INT8 product (three
products of the operands' double-double parts), on square n x n products
of QD operands (limb 0 ~
U[-1, 1], each next limb inside the previous limb's half-ulp).  Per run:
wall time, the multiply-add launch time, QD Gflop/s (2 n^3 / wall) and the
fraction of the FP64 issue peak the multiply-add launch reaches (124 FP64
operations per QD multiply-add, 39.32 T lane-operations/s at 2.4 GHz).

Batch: `count` independent DD products with m, n, l log-uniform in
[16, 512], run as separate block-kernel launches, as one persistent
grouped launch, and as the replay of a captured batch plan (HIP graph).
Per tile variant: the three times and DD Gflop/s (sum of 2 m n l / t).
One JSON line per measurement.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

FP64_ISSUE_PEAK_TOPS = 39.3216
QD_OPS_PER_MADD = 124.0
DD_OPS_PER_MADD = 10.75


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--qd", type=int, nargs="*", default=[512, 1024, 2048])
    ap.add_argument("--batch", type=int, default=512, help="problems in the batch (0: skip)")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()

    import torch
    from paper_1710_01839_amd import inputs, mpgemm as M

    ctx = M.Context(0)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps * 1e3
        gms, gn = ctx.prof_read(M.MPG_KCLASS_GEMM)
        ctx.prof_enable(False)
        return wall, gms / max(gn, 1)

    for n in args.qd:
        A, B = M.to_device(inputs.qd_uniform(n, n, 20)), M.to_device(inputs.qd_uniform(n, n, 21))
        C = M.empty_like_limbs(n, n, 4)
        runs = [("block", v) for v in M.variants(4)]
        runs += [("strassen", {"depth": d}) for d in (1, 2) if n >= 64 << d]
        runs += [("ozaki_crt", None)]
        for algo, tile in runs:
            wall, kms = timed(lambda: M.mpgemm_qd(ctx, A, B, C, algo=algo, tile=tile), args.reps)
            rec = {"kind": "qd", "n": n, "algo": algo, "tile": tile, "wall_ms": round(wall, 3),
                   "launch_ms": round(kms, 3), "qd_gflops": round(2.0 * n ** 3 / wall / 1e6, 1)}
            if algo == "ozaki_crt":
                # three residue-form products of the double-double parts; launch_ms is the
                # mean INT8 product launch (one per part product)
                rec.update({"slices": M.ozaki_last_slices(ctx), "moduli_all_products": M.ozaki_last_moduli(ctx)})
            else:
                d = tile.get("depth", 0) if algo == "strassen" else 0
                rec["frac_fp64_issue_peak"] = round(
                    (7 / 8) ** d * n ** 3 * QD_OPS_PER_MADD / (kms * 1e-3) / (FP64_ISSUE_PEAK_TOPS * 1e12), 4)
            print(json.dumps(rec), flush=True)
        del A, B, C
        torch.cuda.empty_cache()

    if args.batch > 0:
        shapes = inputs.batch_shapes(args.batch)
        flops = sum(2.0 * m * n * l for m, n, l in shapes)
        madds = sum(float(m) * n * l for m, n, l in shapes)
        probs = []
        for i, (m, n, l) in enumerate(shapes):
            probs.append((M.to_device(inputs.dd_uniform(m, l, 3 * i)), M.to_device(inputs.dd_uniform(l, n, 3 * i + 1)),
                          M.empty_like_limbs(m, n, 2)))

        def wall_of(fn, reps):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps * 1e3

        for v, tile in enumerate(M.variants(2)):
            t_sep = wall_of(lambda: [M.mpgemm_dd(ctx, a, b, c, algo="block", tile=tile) for a, b, c in probs],
                            args.reps)
            t_bat = wall_of(lambda: M.mpgemm_dd_batched(ctx, probs, tile), args.reps)
            plan = M.BatchPlan(ctx, probs, tile)
            t_graph = wall_of(lambda: plan.launch(), 5 * args.reps)
            plan.close()
            print(json.dumps({"kind": "batch", "problems": len(shapes), "variant": v, "tile": tile,
                              "separate_ms": round(t_sep, 3), "persistent_ms": round(t_bat, 3),
                              "graph_ms": round(t_graph, 3),
                              "graph_dd_gflops": round(flops / t_graph / 1e6, 1),
                              "graph_frac_fp64_issue_peak":
                                  round(madds * DD_OPS_PER_MADD / (t_graph * 1e-3) / (FP64_ISSUE_PEAK_TOPS * 1e12), 4)}),
                  flush=True)
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
