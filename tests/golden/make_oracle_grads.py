"""Writes the FP64 oracle's exact gradients of the benchmark-size problems.

    python tests/golden/make_oracle_grads.py c2 0     # -> tests/golden/oracle_grad_c2_128cube_seed0.npy

The gradient is dL/deps on the design box from the oracle's time reversal with
FP64 interface storage at every step (the exact derivative of the discrete
loss).  It calls oracle/ and workloads/ only; bench.py --sweep compares the GPU
gradients of every storage setting against these files.  One 128^3 x 1000-step
gradient takes a few minutes on one CPU core.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as w          # noqa: E402
from oracle import adjoint     # noqa: E402


def path_for(name: str, seed: int) -> str:
    return os.path.join(HERE, "oracle_grad_%s_seed%d.npy" % (name, seed))


def main():
    preset, seed = sys.argv[1], int(sys.argv[2])
    prob = w.make(preset, seed=seed)
    t0 = time.perf_counter()
    loss, g = adjoint.grad_time_reversal(prob, "fp64", 1)
    np.save(path_for(prob.name, seed), np.asarray(g, np.float64))
    print("%s seed %d: loss %.12e, |g| %.6e, %.0f s" % (prob.name, seed, loss, np.linalg.norm(g),
                                                       time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
