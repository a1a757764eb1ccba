"""Write groundstate3d_256_step1.txt: one backward-Euler gradient-flow step
(GF-GauSum: the semi-implicit discretisation of the normalised gradient flow,
solved as the P_Delta-preconditioned system by BiCGStab to a relative residual
of 1e-12, then normalised) of the benchmarked 256^3 ground-state case from the
paper's initial guess, computed by the FP64 oracle, at sampled grid points.

The oracle needs minutes for this step (multiplier and Krylov solve on 16.7 M
unknowns), too long for a test, so the test compares the library's step with
these stored samples.  This script calls only oracle/ and workloads/ (no
library code).

Samples: 2048 points uniform over the grid and 2048 points where
|phi0| >= 1e-2 max|phi0|, from a seeded generator.

Usage (about 15 minutes on one core):
    python tests/golden/make_groundstate3d_256_samples.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import groundstate as ogs  # noqa: E402
from oracle import scheme  # noqa: E402

OUT = os.path.join(HERE, "groundstate3d_256_step1.txt")
PRESET, SAMPLE_SEED, NS = "gs3d_256", 20261203, 2048


def main():
    p = W.preset(PRESET)
    phi0 = ogs.initial_guess(p.N, p.L, p.Omega, p.gamma)
    g = ogs.GroundState(scheme.Problem.from_params(p), p.dt)
    ref, (its, res, diff) = g.step(phi0, rtol=1e-12)
    rng = np.random.default_rng(SAMPLE_SEED)
    a = np.abs(phi0).ravel()
    idx = np.unique(np.concatenate([rng.choice(a.size, NS, replace=False),
                                    rng.choice(np.flatnonzero(a >= 1e-2 * a.max()), NS, replace=False)]))
    ii = np.unravel_index(idx, p.N)
    with open(OUT, "w") as f:
        f.write(f"# oracle backward-Euler GFDN step (P_Delta-preconditioned BiCGStab, rtol 1e-12), workload {PRESET}, "
                f"N={p.N}, L={p.L}, s={p.s}, Omega={p.Omega}, beta={p.beta}, lam={p.lam}, kernel={p.kernel}, "
                f"dt={p.dt}\n")
        f.write(f"# phi0 = oracle.groundstate.initial_guess; oracle iterations {its}, residual {res:.3e}, "
                f"||phi1 - phi0||_inf {diff!r}; written by make_groundstate3d_256_samples.py\n")
        f.write("# i0 i1 i2 re im\n")
        for i0, i1, i2, v in zip(ii[0], ii[1], ii[2], ref.ravel()[idx]):
            f.write(f"{i0} {i1} {i2} {float(v.real)!r} {float(v.imag)!r}\n")
    print(f"wrote {OUT}: {idx.size} samples; {its} iterations, residual {res:.3e}, diff {diff:.6e}")


if __name__ == "__main__":
    main()
