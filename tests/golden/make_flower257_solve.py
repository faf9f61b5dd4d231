"""Writes flower257_fp64_solve.json: the oracle's whole solve of the 257^3
flower (u = exp(x+y+z), FP64 V(2,1) from u = 0 to ||r|| <= 1e-10 ||r0||):
its cycle count, residual history, checksums of the final u over the
unknowns, and the final u at 4096 seeded sample nodes.  It calls only the
oracle (and the seeded input generator).

    python tests/golden/make_flower257_solve.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2207_14208_amd import workloads as W  # noqa: E402


def main():
    N, tol = 256, 1e-10
    c = W.flower3d(N)
    O = oracle.Problem(3, N, c.phi)
    og = O.ghosts(0)
    O.set_rhs(c.f, W.points_eval(c.g, og["q"], 3))
    cls = O.classes(0)
    u = np.where(cls == oracle.BOXDIR, c.gB, 0.0)
    it, hist = O.solve(u, tol, 200)
    assert it > 0
    m = (cls == oracle.INSIDE) | (cls == oracle.GHOST)
    idx = np.nonzero(m)[0]
    rng = np.random.Generator(np.random.PCG64(257))
    sample = np.sort(rng.choice(idx, size=4096, replace=False))
    out = {
        "what": "oracle solve of the 257^3 flower, FP64 V(2,1) from u = 0, tol 1e-10 (written by make_flower257_solve.py)",
        "N": N, "tol": tol, "cycles": int(it), "history": [float(v) for v in hist],
        "n_unknowns": int(m.sum()),
        "u_sum": float(u[m].sum()), "u_abs_sum": float(np.abs(u[m]).sum()), "u_max": float(np.abs(u[m]).max()),
        "sample_idx": [int(i) for i in sample], "sample_u": [float(u[i]) for i in sample],
    }
    with open(os.path.join(HERE, "flower257_fp64_solve.json"), "w") as fh:
        json.dump(out, fh)
    print("cycles", it)


if __name__ == "__main__":
    main()
