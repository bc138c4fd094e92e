"""Split-precision (Ozaki, INT8 MFMA) product against the double-double
kernels on the same FP64 operands, on one GPU.

    python -m paper_1710_01839_amd.ozaki_study [--n 4096 ...] [--dist uniform|wide]

For each size: the exact slice count (every digit product kept, so the
result is the product rounded to double-double up to the final
accumulation, the accuracy class of the DD kernels), a few smaller slice
counts, and the DD block and Strassen (depth 2) kernels on the same
operands with zero low parts (or the double-double operands themselves).  Printed per run (one JSON line): wall time
per product, the INT8 MFMA launch time and its rate against the 5.0 POP/s
dense INT8 peak, the splitting/scan time, and DD-equivalent Gflop/s
(2 n^3 / t).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

INT8_PEAK_TOPS = 5000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[2048, 4096])
    ap.add_argument("--dist", choices=("uniform", "wide", "dd"), default="uniform",
                    help="FP64 operands U[-1,1] or with wide exponents, or double-double operands "
                         "(the DD GEMM workload: hi ~ U[-1,1], lo inside hi's half-ulp)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--slices", type=int, nargs="*", default=[8, 12, 15])
    ap.add_argument("--triangle", action="store_true",
                    help="also time each slice count with only the pairs s + t <= S + 1")
    ap.add_argument("--crt", action="store_true",
                    help="also time the residue (CRT) form at each slice count up to 20 (one INT8 "
                         "product per modulus)")
    ap.add_argument("--auto", action="store_true",
                    help="with --dist dd: also time MPG_AUTO with the residue form (exact slice count) in the "
                         "tuning table, whose slice and moduli counts are decided on the device")
    args = ap.parse_args()

    import torch
    from paper_1710_01839_amd import inputs, mpgemm as M

    ctx = M.Context(0)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.reps):
            fn()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.reps * 1e3
        gms, gn = ctx.prof_read(M.MPG_KCLASS_GEMM)
        ams, _ = ctx.prof_read(M.MPG_KCLASS_AUX)
        ctx.prof_enable(False)
        return wall, gms / max(gn, 1), ams / args.reps

    for n in args.n:
        dd = args.dist == "dd"
        if dd:
            Ad, Bd = M.to_device(inputs.dd_uniform(n, n, 20)), M.to_device(inputs.dd_uniform(n, n, 21))
            A, B = Ad[0], Bd[0]
        elif args.dist == "uniform":
            A = torch.as_tensor(inputs.dd_uniform(n, n, 40)[0]).cuda()
            B = torch.as_tensor(inputs.dd_uniform(n, n, 41)[0]).cuda()
        else:
            A = torch.as_tensor(inputs.fp64_wide(n, n, 40)).cuda()
            B = torch.as_tensor(inputs.fp64_wide(n, n, 41)).cuda()
        C = M.empty_like_limbs(n, n, 2)

        def product(S, mode="all"):
            if dd:
                M.mpgemm_dd_ozaki(ctx, Ad, Bd, C, S, mode)
            else:
                M.mpgemm_ozaki_dd(ctx, A, B, C, S, mode)

        product(0)
        s_exact = M.ozaki_last_slices(ctx)
        runs = [(S, "all") for S in [0] + [s for s in args.slices if s < s_exact]]
        if args.triangle:
            runs += [(S, "triangle") for S in [s_exact] + [s for s in args.slices if s < s_exact]]
        if args.crt:
            runs += [(S, "crt") for S in [0] + [s for s in args.slices if s < s_exact]
                     if (S or s_exact) <= 20]
        for S, mode in runs:
            wall, kms, aux = timed(lambda: product(S, mode))
            used = M.ozaki_last_slices(ctx)
            npairs = {"all": used * used, "triangle": used * (used + 1) // 2,
                      "crt": M.ozaki_last_moduli(ctx)}[mode]
            tops = npairs * 2.0 * n ** 3 / (kms * 1e-3) / 1e12
            print(json.dumps({"kind": "ozaki", "n": n, "dist": args.dist, "slices": used, "pairs": mode,
                              "int8_products": npairs,
                              "exact": S == 0, "wall_ms": round(wall, 3), "mfma_launch_ms": round(kms, 3),
                              "aux_ms": round(aux, 3), "int8_tops": round(tops, 1),
                              "frac_int8_peak": round(tops / INT8_PEAK_TOPS, 4),
                              "dd_equiv_gflops": round(2.0 * n ** 3 / wall / 1e6, 1)}), flush=True)
        if dd and args.auto:
            M.Tuner(ctx).table_set("dd", n, n, n, "ozaki_crt", {"slices": 0})
            wall, kms, aux = timed(lambda: M.mpgemm_dd(ctx, Ad, Bd, C, algo="auto"))
            print(json.dumps({"kind": "ozaki_auto", "n": n, "dist": args.dist, "pairs": "crt",
                              "wall_ms": round(wall, 3), "aux_ms": round(aux, 3)}), flush=True)
        if not dd:
            Ad, Bd = (A, torch.zeros_like(A)), (B, torch.zeros_like(B))
        for algo, tile in (("block", None), ("strassen", {"depth": 2})):
            wall, kms, aux = timed(lambda: M.mpgemm_dd(ctx, Ad, Bd, C, algo=algo, tile=tile))
            print(json.dumps({"kind": "dd", "n": n, "algo": algo, "tile": tile, "wall_ms": round(wall, 3),
                              "launch_ms": round(kms, 3), "aux_ms": round(aux, 3),
                              "dd_gflops": round(2.0 * n ** 3 / wall / 1e6, 1)}), flush=True)
        del A, B, C, Ad, Bd
        torch.cuda.empty_cache()
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
