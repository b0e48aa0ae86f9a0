"""Write the stored expected values under tests/golden/ (calls only the oracle).

    python tests/golden/make_golden.py

finger_h4_c4_fixed_point.npz: the local/global fixed point of the 4-chamber
finger at 4 mm voxels (alpha = 2, self-collision on), iterated by the FP64
oracle from the rest shape until r_k <= 1e-11 with an unchanged active set.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2203_02054_amd import meshgen as mg  # noqa: E402
import oracle  # noqa: E402


def finger_fixed_point():
    wl = mg.finger(4.0, 4, 2.0)
    prob = oracle.Problem.from_workload(wl)
    x, A, st = oracle.solve(prob, wl.alpha, tol=1e-11, max_iter=20000)
    assert st["converged"], st
    rows, tg = A.listing(prob)
    np.savez_compressed(os.path.join(HERE, "finger_h4_c4_fixed_point.npz"), x=x, contacts=rows, targets=tg,
                        iters=st["iters"], residual=st["residual"])
    print("finger fixed point:", st["iters"], "iterations, residual", st["residual"], "contacts", len(rows))


if __name__ == "__main__":
    finger_fixed_point()
