"""Prediction of block-algorithm run time and the three-step tuning procedure
(Section 3 of the paper), written out plainly.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

Reading of the missing Fig. 1: the product of a slab of A -- the first
2 * n_min rows (two block rows) -- with the full B is timed and the time is
scaled linearly in the number of rows.  Every row of the paper's Tables 1
and 3 satisfies predicted = cost * n / (2 n_min), and for n_min >= n / 2 the
slab is the whole matrix and the prediction costs as much as the product.
"""
from __future__ import annotations


def slab_rows(n: int, n_min: int) -> int:
    """Rows of A used for the prediction (capped at n)."""
    return min(n, 2 * n_min)


def predict_full_time(t_slab: float, n: int, n_min: int) -> float:
    """Full-size block time predicted from the time of the slab product."""
    return t_slab * n / slab_rows(n, n_min)


def rel_diff(predicted: float, real: float) -> float:
    return abs(predicted - real) / real


def tune(n: int, n_min_candidates, time_block_slab, time_full):
    """The paper's tuning program.

    (1) For every candidate block size, time the slab product and predict
        the full-size block time; keep the block size with the smallest
        prediction.
    (2) Time the simple algorithm, the block algorithm with that block size
        and the Strassen algorithm at full size.
    (3) Return the fastest of the three.

    time_block_slab(n_min, rows) -> seconds; time_full(algo, n_min) ->
    seconds with algo in {'simple', 'block', 'strassen'}.  Returns
    (algo, n_min, timings) where timings lists every measurement made, in
    order, as (kind, n_min, seconds)."""
    log = []
    best_nmin, best_pred = None, None
    for nm in n_min_candidates:
        rows = slab_rows(n, nm)
        t = time_block_slab(nm, rows)
        log.append(("slab", nm, t))
        pred = predict_full_time(t, n, nm)
        if best_pred is None or pred < best_pred:
            best_nmin, best_pred = nm, pred
    full = {}
    for algo in ("simple", "block", "strassen"):
        t = time_full(algo, best_nmin)
        log.append((algo, best_nmin, t))
        full[algo] = t
    algo = min(full, key=full.get)
    return algo, best_nmin, log
