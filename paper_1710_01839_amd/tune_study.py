"""Tuning study on one GPU: how well the prediction of Section 3 works in
its printed form and in the GPU form, and what the run-time MLP gains over
the paper's procedure and over exhaustive search.

    python -m paper_1710_01839_amd.tune_study [--out FILE.jsonl]

1. Prediction accuracy: for DD n in {2048, 4096} and QD n = 1024 and the
   first four tile variants, the real full-size block time against the
   prediction from slabs (GPU rule: slabs of one and two waves of resident
   workgroups, extrapolated linearly in waves; printed rule: two block rows
   scaled linearly).
2. Training data: exhaustive tuning of training shapes (every candidate
   timed) into a JSONL timing database; the MLP is trained on it on the GPU.
3. Held-out shapes: exhaustive, paper and MLP-pruned (the default top-k) tuning; each
   pick is re-timed (median of 5) and its regret against the exhaustive pick
   reported with the wall-clock tuning time of each mode.

Prints one JSON object per line and a summary line at the end.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

TRAIN = ([("dd", n, n, n) for n in (192, 256, 384, 512, 768, 1024, 1536, 2048, 3072)]
         + [("dd", 512, 2048, 1024), ("dd", 2048, 512, 768), ("dd", 1024, 1024, 4096),
            ("dd", 3072, 1024, 2048)]
         + [("qd", n, n, n) for n in (192, 256, 384, 512, 768, 1024, 1536)]
         + [("qd", 512, 1024, 768)])
HELD_OUT = [("dd", 640, 640, 640), ("dd", 1280, 1280, 1280), ("dd", 1792, 1792, 1792),
            ("dd", 2560, 2560, 2560), ("dd", 4096, 4096, 4096), ("dd", 768, 1536, 1024),
            ("qd", 640, 640, 640), ("qd", 1280, 1280, 1280), ("qd", 2048, 2048, 2048)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="also write the records to this JSONL file")
    ap.add_argument("--epochs", type=int, default=3000)
    args = ap.parse_args()

    from paper_1710_01839_amd import mpgemm as M
    ctx = M.Context(0)
    T = M.Tuner(ctx)
    recs = []

    def emit(r):
        recs.append(r)
        print(json.dumps(r), flush=True)

    for prec, n in (("dd", 2048), ("dd", 4096), ("qd", 1024)):
        for v in M.variants(2 if prec == "dd" else 4)[:4]:
            real = T.time(prec, n, n, n, "block", v, reps=3)
            p0, s0 = T.predict_block(prec, n, n, n, v, 0)
            p1, s1 = T.predict_block(prec, n, n, n, v, 1)
            emit({"kind": "prediction", "prec": prec, "n": n, "tile": v, "real_ms": real,
                  "gpu_rule_ms": p0, "gpu_rule_slab_ms": s0, "gpu_rule_err": abs(p0 - real) / real,
                  "paper_rule_ms": p1, "paper_rule_slab_ms": s1,
                  "paper_rule_err": abs(p1 - real) / real})

    db = os.path.join(tempfile.mkdtemp(), "timings.jsonl")
    T.set_db(db)
    t0 = time.time()
    for prec, m, n, l in TRAIN:
        r = T.tune(prec, m, n, l, "exhaustive")
        emit({"kind": "train", "prec": prec, "shape": [m, n, l], **r})
    sweep = time.time() - t0
    T.set_db(None)
    mlp = M.MLP(ctx)
    t0 = time.time()
    loss, rows = mlp.train_db(db, args.epochs, 3e-3)
    emit({"kind": "mlp_training", "rows": rows, "epochs": args.epochs, "final_loss": loss,
          "seconds": time.time() - t0, "exhaustive_sweep_seconds": sweep})

    summary = {"paper": [], "mlp": [], "paper_time": [], "mlp_time": []}
    for prec, m, n, l in HELD_OUT:
        res = {mode: T.tune(prec, m, n, l, mode, 0) for mode in ("exhaustive", "paper", "mlp")}
        ret = {mode: T.time(prec, m, n, l, r["algo"], r["tile"], reps=5) for mode, r in res.items()}
        rec = {"kind": "held_out", "prec": prec, "shape": [m, n, l]}
        for mode in res:
            rec[mode] = {"algo": res[mode]["algo"], "tile": res[mode]["tile"], "ms": ret[mode],
                         "regret": ret[mode] / ret["exhaustive"] - 1.0,
                         "tuning_seconds": res[mode]["seconds"], "trials": res[mode]["trials"],
                         "time_fraction": res[mode]["seconds"] / res["exhaustive"]["seconds"]}
        for mode in ("paper", "mlp"):
            summary[mode].append(rec[mode]["regret"])
            summary[mode + "_time"].append(rec[mode]["time_fraction"])
        emit(rec)
    emit({"kind": "summary",
          "paper_max_regret": max(summary["paper"]), "paper_mean_time_fraction":
              sum(summary["paper_time"]) / len(summary["paper_time"]),
          "mlp_max_regret": max(summary["mlp"]), "mlp_mean_time_fraction":
              sum(summary["mlp_time"]) / len(summary["mlp_time"]),
          "mlp_max_time_fraction": max(summary["mlp_time"])})
    if args.out:
        with open(args.out, "w") as f:
            for r in recs:
                f.write(json.dumps(r) + "\n")
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
