"""Write c5_targets.json: per-problem targets of the 64 unseen uneven problems
(m log-uniform in [1e4, 2e5], n in [128, 4096], column-scale spread up to
1e3; logistic, lambda = 1e-5, b = 64) from the FP64 oracle only.

For each problem: the plain-SGD step size (s = 1) with the lowest held-out
loss after half an epoch, over eta = 2^k / mean ||a_i||^2, k = -4 .. 12 (the
column scales spread the row norms over orders of magnitude, so the grid is
placed relative to them); then plain SGD with it
for four epochs, the held-out test loss after every 1/16 epoch, and
L* = the mean of those losses over the last two epochs (the plateau level of
constant-step SGD). A method reaches the target at the first snapshot where
the mean test loss of the trailing half epoch of snapshots is <= L* (1 + 1e-3).

    OMP_NUM_THREADS=8 python tests/golden/make_c5_targets.py
"""
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import reference as R  # noqa: E402
from workloads import uneven_problem, uneven_problem_specs  # noqa: E402

B, LAM, SEED, EPOCHS, SNAPS_PER_EPOCH = 64, 1e-5, 42, 4, 16
EVAL_SEED, COUNT = 202, 64
RANGES = dict(m_range=(1e4, 2e5), n_range=(128, 4096), spread_range=(1.0, 1e3))
KS = range(-4, 13)


def main():
    out = []
    t0 = time.time()
    for i, spec in enumerate(uneven_problem_specs(COUNT, EVAL_SEED, **RANGES)):
        p = uneven_problem(spec)
        per_epoch = p.m // B
        r2 = float(np.mean(np.sum(p.X.astype(np.float64) ** 2, axis=1)))
        best = None
        for eta in [2.0 ** k / r2 for k in KS]:
            x = R.sgd(p.X, p.y, np.zeros(p.n), eta, LAM, B, SEED, 0, per_epoch // 2)
            loss = R.logloss(p.X_test, p.y_test, x)
            if math.isfinite(loss) and (best is None or loss < best[0]):
                best = (loss, eta)
        eta = best[1]
        every = max(1, per_epoch // SNAPS_PER_EPOCH)
        nsnap = EPOCHS * SNAPS_PER_EPOCH
        x = np.zeros(p.n)
        losses = []
        for k in range(nsnap):
            x = R.sgd(p.X, p.y, x, eta, LAM, B, SEED, k * every, every)
            losses.append(R.logloss(p.X_test, p.y_test, x))
        L_star = float(np.mean(losses[nsnap // 2:]))
        out.append(dict(spec=spec, eta=eta, mean_row_norm2=r2, steps_per_snapshot=every,
                        snapshots=nsnap,
                        test_loss=losses, L_star=L_star))
        print(f"{i}: m={p.m} n={p.n} eta={eta:.4g} (x r2 = {eta * r2:g}) L*={L_star:.6f} "
              f"({time.time() - t0:.0f}s)",
              flush=True)
    doc = dict(workload="64 unseen uneven dense logistic problems (uneven_problem_specs(64, 202)),"
                        " lambda=1e-5, b=64, seed 42",
               rule="L* = mean oracle plain-SGD test loss over epochs 3-4 (16 snapshots per "
                    "epoch); target L* (1 + 1e-3) on the trailing half-epoch mean",
               source="oracle.reference.sgd / logloss (FP64), tests/golden/make_c5_targets.py",
               problems=out)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_targets.json"),
              "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
