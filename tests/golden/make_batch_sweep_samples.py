"""Write batch_sweep_step5.txt: five TS2-GauSum steps (eqs. tssp1-tssp3) of one
instance of each grid size of the benchmarked 64-instance 2D sweep (instances
0, 17, 38, 63: 128^2, 256^2, 384^2, 512^2), computed by the FP64 oracle, at
sampled grid points.

The oracle needs minutes for these grids (mostly building the GauSum
multiplier), too long for a test, so the test compares the batched sweep and
single plans with these stored samples.  This script calls only oracle/ and
the seeded input generators of workloads/ (no library code).

Samples per instance: 512 points uniform over the grid and 512 points where
|psi0| >= 1e-2 max|psi0|, from a seeded generator.

Usage (about 3 minutes on one core):
    python tests/golden/make_batch_sweep_samples.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import scheme  # noqa: E402

OUT = os.path.join(HERE, "batch_sweep_step5.txt")
INSTANCES, STEPS, SAMPLE_SEED, NS = (0, 17, 38, 63), 5, 20261203, 512


def sample_indices(psi0, rng):
    a = np.abs(psi0).ravel()
    uni = rng.choice(a.size, NS, replace=False)
    cor = rng.choice(np.flatnonzero(a >= 1e-2 * a.max()), NS, replace=False)
    return np.unique(np.concatenate([uni, cor]))


def main():
    params = W.batch_sweep()
    rng = np.random.default_rng(SAMPLE_SEED)
    with open(OUT, "w") as f:
        f.write(f"# oracle TS2-GauSum (eqs. tssp1-tssp3), workloads.batch_sweep() instances {INSTANCES}, "
                f"psi0 = workloads.vortex_lattice_2d(N, L, seed=k), steps={STEPS}, t0=0; "
                f"written by make_batch_sweep_samples.py\n")
        f.write("# k i0 i1 re im\n")
        for k in INSTANCES:
            p = params[k]
            psi0 = W.vortex_lattice_2d(p.N, p.L, seed=k)
            ref, _ = scheme.Problem.from_params(p).run(psi0, STEPS, p.dt)
            idx = sample_indices(psi0, rng)
            ii = np.unravel_index(idx, p.N)
            for a, b, v in zip(ii[0], ii[1], ref.ravel()[idx]):
                f.write(f"{k} {a} {b} {float(v.real)!r} {float(v.imag)!r}\n")
            print(f"instance {k} N={p.N}: {idx.size} samples", flush=True)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
