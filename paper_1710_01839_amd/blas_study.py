"""Cost of the BLAS-style form (transposes, alpha / beta, complex DD) on one GPU.

    python -m paper_1710_01839_amd.blas_study [--dd 4096] [--qd 1024] [--z 2048]

Real DD and QD: the plain product C := A B next to alpha op(A) op(B) + beta C
with both operands transposed, over the same product algorithm (Strassen
depth 2 over the default tile for DD, depth 1 for QD).  Complex DD: the
embedding product (m x 2k times 2k x 2n real DD) by the block kernel, by
Strassen depth 2 and by the split product with the exact slice count.

Per run: wall time per call, the product launch time, the time of the
packing and scaling kernels, and Gflop/s counted as 2 m n k real (8 m n k
complex) multiply-adds per call.  One JSON line per measurement.
"""
from __future__ import annotations

import argparse
import json
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dd", type=int, nargs="*", default=[4096])
    ap.add_argument("--qd", type=int, nargs="*", default=[1024])
    ap.add_argument("--z", type=int, nargs="*", default=[2048])
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
        ams, _ = ctx.prof_read(M.MPG_KCLASS_AUX)
        ctx.prof_enable(False)
        return wall, gms / reps, ams / reps

    def emit(rec):
        print(json.dumps(rec), flush=True)

    for limbs, sizes, depth in ((2, args.dd, 2), (4, args.qd, 1)):
        gen = inputs.dd_uniform if limbs == 2 else inputs.qd_uniform
        alpha = (-1.25, 2.0 ** -62, 0.0, 0.0)[:limbs]
        beta = (0.5, 0.0, 0.0, 0.0)[:limbs]
        for n in sizes:
            A, B = M.to_device(gen(n, n, 50)), M.to_device(gen(n, n, 51))
            C = M.to_device(gen(n, n, 52))
            tile = {"depth": depth}
            for ta, tb, a, b in (("N", "N", 1.0, 0.0), ("T", "T", 1.0, 0.0),
                                 ("N", "N", alpha, beta), ("T", "T", alpha, beta)):
                wall, g, aux = timed(lambda: M.rgemm(ctx, A, B, C, a, b, ta, tb, "strassen", tile),
                                     args.reps)
                emit({"form": "real", "limbs": limbs, "n": n, "op": ta + tb,
                      "alpha_beta": a != 1.0 or b != 0.0, "algo": f"strassen{depth}",
                      "wall_ms": round(wall, 3), "product_ms": round(g, 3), "aux_ms": round(aux, 3),
                      "gflops": round(2 * n ** 3 / wall / 1e6, 2)})
            del A, B, C
            torch.cuda.empty_cache()

    for n in args.z:
        A = M.to_device(inputs.dd_uniform(n, n, 60) + inputs.dd_uniform(n, n, 61))
        B = M.to_device(inputs.dd_uniform(n, n, 62) + inputs.dd_uniform(n, n, 63))
        C = M.to_device(inputs.dd_uniform(n, n, 64) + inputs.dd_uniform(n, n, 65))
        alpha, beta = (0.75, 0.0, -0.5, 0.0), (0.0, 0.0, 1.0, 0.0)
        for algo, tile in (("block", None), ("strassen", {"depth": 2}), ("ozaki", {"slices": 0})):
            wall, g, aux = timed(lambda: M.zgemm_dd(ctx, A, B, C, alpha, beta, "C", "N", algo, tile),
                                 args.reps)
            emit({"form": "complex", "limbs": 2, "n": n, "op": "CN", "alpha_beta": True,
                  "algo": algo, "wall_ms": round(wall, 3), "product_ms": round(g, 3),
                  "aux_ms": round(aux, 3), "gflops": round(8 * n ** 3 / wall / 1e6, 2)})
        del A, B, C
        torch.cuda.empty_cache()
    ctx.close()


if __name__ == "__main__":
    main()
