"""Writes c3_residual_floor.txt: the true relative residual ||f - K x|| / ||f||
(FP64, scipy sparse product) of the oracle's own FP64 solution of the
elasticity workload C3 (48^3 Q1, 216 uneven subdomains, stiff inclusions).

The solution is the oracle's PCG with its multilevel BDDC preconditioner
(initial constraints c+e, no adaptive ones: the same solution, fewer
operations) run to a recursive residual of 1e-13, well below the floor, so
that its true residual is what FP64 attains on this system as measured by
this formula.  Calls only the oracle and the workload generator.

    python tests/golden/c3_residual_floor.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402
from oracle import fem  # noqa: E402


def main():
    t0 = time.perf_counter()
    prob = W.CONFIGS["c3"](0)
    H = O.setup_hierarchy(prob, adaptive=False)
    K = H.levels[0].Kglob
    f = prob.rhs[:, 0]
    x, its, al, be, hist = O.pcg(K, f, lambda v: O.bddc_apply(H, v), rtol=1e-13, maxit=3000)
    Kf = fem.assemble_global(prob)
    res = float(np.linalg.norm(f - Kf @ x) / np.linalg.norm(f))
    best = min(hist)
    out = os.path.join(HERE, "c3_residual_floor.txt")
    with open(out, "w") as fh:
        fh.write("# true relative residual of the oracle's FP64 PCG solution of C3 (seed 0)\n")
        fh.write(f"# written by tests/golden/c3_residual_floor.py; PCG iterations {its}, "
                 f"last recursive residual {hist[-1]:.3e}, {time.perf_counter() - t0:.0f} s\n")
        fh.write(f"{res:.6e}\n")
    print(out, res)


if __name__ == "__main__":
    main()
