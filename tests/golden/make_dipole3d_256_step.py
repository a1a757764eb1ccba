"""Write dipole3d_256_step{1,2}.txt: one or two TS2-GauSum steps (eqs.
tssp1-tssp3) of the 256^3 dipolar workload, computed by the FP64 oracle, at
sampled grid points.  Two steps pass through the merged full-step kinetic
junction that every inner step of a longer call uses.  With order 4,
dipole3d_256_order4_step1.txt: one fourth-order step (the symmetric
triple-jump composition of TS2 steps of lengths w1 dt, w0 dt, w1 dt).  With
"local", dipole3d_256_local_step{n}.txt: the same workload with lam = 0 (no
nonlocal term).

The oracle needs minutes for one step at this size (the padded convolution
runs on a 512^3 box), too long for a test, so the test compares the library's
step with these stored samples.  This script calls only oracle/ and the seeded
input generators of workloads/ (no library code).

Samples: 2048 points uniform over the grid and 2048 points where
|psi0| >= 1e-2 max|psi0| (inside the condensate), from a seeded generator.
With "tiles", dipole3d_256_tiles_step1.txt: one step at 8192 points laid out
so that every tile of 8 adjacent columns of the axis-0 passes (i1, i2 // 8)
and of the axis-1 passes (i0, i2 // 8) holds exactly one of them: point k has
i1 = k // 32, i2 = 8 (k % 32) + i1 % 8, i0 = (i1 + 37 (k % 32)) % 256.

Usage (about 8 minutes per step on one core):
    python tests/golden/make_dipole3d_256_step.py [steps] [order] [local|tiles]   (steps 1 or 2, order 2 or 4;
    default 1 2)
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import scheme  # noqa: E402

PRESET, SEED, SAMPLE_SEED, NS = "dipole3d_256", 0, 20261203, 2048


def sample_indices(psi0):
    rng = np.random.default_rng(SAMPLE_SEED)
    n = psi0.size
    uni = rng.choice(n, NS, replace=False)
    a = np.abs(psi0).ravel()
    core = np.flatnonzero(a >= 1e-2 * a.max())
    cor = rng.choice(core, NS, replace=False)
    return np.unique(np.concatenate([uni, cor]))


def tile_indices(N):
    """Flat indices of the tile-covering points (one per 8-column tile of the axis-0 and of the axis-1 passes)."""
    k = np.arange(N[1] * (N[2] // 8))
    i1 = k // (N[2] // 8)
    t2 = k % (N[2] // 8)
    i2 = 8 * t2 + i1 % 8
    i0 = (i1 + 37 * t2) % N[0]
    return np.ravel_multi_index((i0, i1, i2), N)


def main(steps=1, order=2, local=False, tiles=False):
    tag = "_local" if local else ("_tiles" if tiles else ("" if order == 2 else f"_order{order}"))
    OUT = os.path.join(HERE, f"dipole3d_256{tag}_step{steps}.txt")
    p = W.preset(PRESET)
    if local:
        p = p.replace(lam=0.0)
    psi0 = W.initial_state(p, seed=SEED)
    prob = scheme.Problem.from_params(p)
    ref, _ = prob.run(psi0, steps, p.dt) if order == 2 else prob.run4(psi0, steps, p.dt)
    idx = tile_indices(p.N) if tiles else sample_indices(psi0)
    ii = np.unravel_index(idx, p.N)
    vals = ref.ravel()[idx]
    with open(OUT, "w") as f:
        f.write(f"# oracle TS2-GauSum (eqs. tssp1-tssp3), workload {PRESET}, N={p.N}, L={p.L}, s={p.s}, "
                f"Omega={p.Omega}, beta={p.beta}, lam={p.lam}, kernel={p.kernel}, dt={p.dt}\n")
        f.write(f"# psi0 = workloads.initial_state(seed={SEED}); steps={steps}; order={order}; t0=0; "
                f"written by make_dipole3d_256_step.py\n")
        f.write("# i0 i1 i2 re im\n")
        for a, b, c, v in zip(ii[0], ii[1], ii[2], vals):
            f.write(f"{a} {b} {c} {float(v.real)!r} {float(v.imag)!r}\n")
    print(f"wrote {OUT}: {idx.size} samples")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1, int(sys.argv[2]) if len(sys.argv) > 2 else 2,
         len(sys.argv) > 3 and sys.argv[3] == "local", len(sys.argv) > 3 and sys.argv[3] == "tiles")
