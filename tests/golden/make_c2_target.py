"""Write c2_target.json: the FP64 oracle's plain mini-batch SGD (s = 1) on the
dense 2^20 x 2048 FP32 workload for its full budget of 20 epochs, with the
held-out test loss after every epoch.

L* is the plateau level of constant-step SGD: the mean of the per-epoch test
losses over the second half of the budget (epochs 11-20). A method reaches
the target at the first snapshot where the mean test loss of the trailing
half epoch of snapshots is <= L* (1 + 1e-3). Only the oracle and the input
generators are used. Runtime: a few minutes on 4-8 cores.

    OMP_NUM_THREADS=4 python tests/golden/make_c2_target.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import reference as R  # noqa: E402
from workloads import dense_c2  # noqa: E402

ETA, LAM, B, SEED, EPOCHS = 2.0, 1e-5, 64, 42, 20


def main():
    t0 = time.time()
    p = dense_c2(SEED)
    print(f"generated in {time.time() - t0:.1f}s", flush=True)
    steps_per_epoch = p.m // B
    x = np.zeros(p.n)
    losses = []
    for ep in range(EPOCHS):
        t = time.time()
        x = R.sgd(p.X, p.y, x, ETA, LAM, B, SEED, ep * steps_per_epoch, steps_per_epoch)
        losses.append(R.logloss(p.X_test, p.y_test, x))
        print(f"epoch {ep + 1}: test loss {losses[-1]:.9f} ({time.time() - t:.1f}s)", flush=True)
    out = dict(workload="dense 2^20x2048 FP32, N(0,1/2048), 205 columns x10, 5% flips, "
                        "seed 42, 2^18 test rows",
               eta=ETA, lam=LAM, b=B, seed=SEED, epochs=EPOCHS,
               steps=EPOCHS * steps_per_epoch, test_loss_by_epoch=losses,
               L_star=float(np.mean(losses[EPOCHS // 2:])), L_final=losses[-1],
               rule="L* = mean oracle test loss over epochs 11-20; target L* (1 + 1e-3) on the "
                    "trailing half-epoch mean of a method's snapshot losses",
               source="oracle.reference.sgd (FP64), tests/golden/make_c2_target.py")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_target.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
