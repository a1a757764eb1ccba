"""Write adjoint3d_96_grad.txt: the gradients of the benchmarked 96^3
differentiation case, computed by the FP64 oracle, at sampled grid points.

The case: 200 TS2-GauSum steps (eqs. tssp1-tssp3) of the adjoint3d_96
workload with V(x) = |x|^2/2 as a grid potential U, from psi0 =
anisotropic_gaussian(seed=0), and the loss L = |<psi_t, psi(T)>|^2 + 0.1 <Lz>
with psi_t = adjoint_target(seed=1).  Stored: dL/dpsi0 (g = dL/dRe + i dL/dIm)
and dL/dU, from the oracle's adjoint of the step (oracle/adjoint.py), and L.

The oracle needs minutes for this (200 steps forward and back), too long for a
test, so the test compares the library's adjoint with these stored samples.
This script calls only oracle/ and workloads/ (no library code).

Samples: 2048 points uniform over the grid and 2048 points where
|psi0| >= 1e-2 max|psi0|, from a seeded generator, the same points for both
gradients.

Usage (about 10 minutes on one core):
    python tests/golden/make_adjoint3d_96_samples.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
from oracle import scheme  # noqa: E402

OUT = os.path.join(HERE, "adjoint3d_96_grad.txt")
PRESET, STEPS, SAMPLE_SEED, NS = "adjoint3d_96", 200, 20261203, 2048


def main():
    p = W.preset(PRESET)
    psi0 = W.anisotropic_gaussian(p.N, p.L, (1.0, 1.0, 1.0), seed=0)
    U = W.harmonic_potential(p.N, p.L, (1.0, 1.0, 1.0))
    tgt = W.adjoint_target(p.N, p.L, seed=1)
    pr = scheme.Problem.from_params(p)
    pr.U = U
    psiT, _ = pr.run(psi0, STEPS, p.dt)
    loss, gT = adj.loss_and_grad(psiT, tgt, p.N, p.L)
    g0, gU = adj.run_adjoint(pr, psi0, STEPS, p.dt, gT)
    rng = np.random.default_rng(SAMPLE_SEED)
    a = np.abs(psi0).ravel()
    idx = np.unique(np.concatenate([rng.choice(a.size, NS, replace=False),
                                    rng.choice(np.flatnonzero(a >= 1e-2 * a.max()), NS, replace=False)]))
    ii = np.unravel_index(idx, p.N)
    with open(OUT, "w") as f:
        f.write(f"# oracle adjoint of {STEPS} TS2-GauSum steps, workload {PRESET}, N={p.N}, L={p.L}, s={p.s}, "
                f"Omega={p.Omega}, beta={p.beta}, lam={p.lam}, kernel={p.kernel}, dt={p.dt}; U = |x|^2/2\n")
        f.write(f"# psi0 = anisotropic_gaussian(seed=0), target = adjoint_target(seed=1), "
                f"L = |<target, psi(T)>|^2 + 0.1 <Lz> = {loss!r}; written by make_adjoint3d_96_samples.py\n")
        f.write("# i0 i1 i2 Re(dL/dpsi0) Im(dL/dpsi0) dL/dU\n")
        for i0, i1, i2, g, u in zip(ii[0], ii[1], ii[2], g0.ravel()[idx], gU.ravel()[idx]):
            f.write(f"{i0} {i1} {i2} {float(g.real)!r} {float(g.imag)!r} {float(u)!r}\n")
    print(f"wrote {OUT}: {idx.size} samples, loss {loss!r}")


if __name__ == "__main__":
    main()
