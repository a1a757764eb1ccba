"""Write the stored oracle samples of the configured runs at their full length:

* dipole3d_128_long.txt -- the 128^3 dipolar case (grid [-12,12]^3, s = 0.8,
  Omega = 0.7, gamma = (1,1,2), beta = 200, lam = 50 z-dipole GauSum on 256^3
  padding, dt = 5e-4) after 100 and 1000 TS2-GauSum steps (eqs.
  tssp1-tssp3) from workloads.initial_state(seed=0);
* batch_sweep_long.txt -- one instance of each grid size of the 64-instance
  2D sweep (instances 0, 17, 38, 63: 128^2, 256^2, 384^2, 512^2) after 500
  steps from workloads.vortex_lattice_2d(N, L, seed=k);
* plain2d_long.txt -- the 2D plain case (64^2 on [-8,8]^2, s = 0.75,
  Omega = 0.5, beta = 100, lam = 1 Coulomb GauSum on 128^2 padding,
  dt = 1e-3) after 100 and 1000 steps from workloads.initial_state(seed=0),
  at every grid point.

Each run records, per stored step, the FP64 oracle's mass, total energy and
<Lz> (eqs. mass, energy, AME; the energy in rotating coordinates at that
time) on "# scalars" lines, and the state at sampled grid points: half
uniform over the grid, half where |psi0| >= 1e-2 max|psi0|, from a seeded
generator.  The oracle needs minutes for these runs, too long for a test; the
GPU tests and the benchmark compare the library's trajectories with these
samples.  This script calls only oracle/ and the seeded input generators of
workloads/ (no library code).

Usage (about 15 minutes on 8 cores):
    python tests/golden/make_long_runs.py [case3d|batch|plain2d]   (default: all)
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import diagnostics, scheme  # noqa: E402

SAMPLE_SEED = 20261203
CASE3D = ("dipole3d_128", (100, 1000), 2048)     # preset, stored steps, samples per half
PLAIN2D = ("plain2d", (100, 1000))              # preset, stored steps (every grid point)
BATCH = ((0, 17, 38, 63), 500, 512)              # instances, steps, samples per half


def sample_indices(psi0, ns, rng):
    a = np.abs(psi0).ravel()
    uni = rng.choice(a.size, ns, replace=False)
    cor = rng.choice(np.flatnonzero(a >= 1e-2 * a.max()), ns, replace=False)
    return np.unique(np.concatenate([uni, cor]))


def scalars(prob, p, psi, t):
    m = diagnostics.mass(psi, p.N, p.L)
    e = diagnostics.energy_parts(prob, psi, t)[5]
    lz = diagnostics.angular_momentum(psi, p.N, p.L)
    return m, e, lz


def write_samples(f, key, idx, shape, psi):
    ii = np.unravel_index(idx, shape)
    for pos, v in zip(zip(*ii), psi.ravel()[idx]):
        f.write(f"{key} " + " ".join(str(int(q)) for q in pos) + f" {float(v.real)!r} {float(v.imag)!r}\n")


def case3d(full=False):
    name, steps, ns = PLAIN2D + (None,) if full else CASE3D
    p = W.preset(name)
    out = os.path.join(HERE, f"{name}_long.txt")
    psi = W.initial_state(p, seed=0)
    prob = scheme.Problem.from_params(p)
    idx = np.arange(psi.size) if full else sample_indices(psi, ns, np.random.default_rng(SAMPLE_SEED))
    with open(out, "w") as f:
        f.write(f"# oracle TS2-GauSum (eqs. tssp1-tssp3), workload {name}, N={p.N}, L={p.L}, s={p.s}, "
                f"Omega={p.Omega}, beta={p.beta}, lam={p.lam}, kernel={p.kernel}, dt={p.dt}\n")
        f.write("# psi0 = workloads.initial_state(seed=0); t0=0; written by make_long_runs.py\n")
        m, e, lz = scalars(prob, p, psi, 0.0)
        f.write(f"# scalars step=0 mass={m!r} energy={e!r} lz={lz!r}\n")
        f.write("# step " + " ".join(f"i{j}" for j in range(p.d)) + " re im\n")
        t, done = 0.0, 0
        for target in steps:
            psi, t = prob.run(psi, target - done, p.dt, t)
            done = target
            m, e, lz = scalars(prob, p, psi, t)
            f.write(f"# scalars step={done} mass={m!r} energy={e!r} lz={lz!r}\n")
            write_samples(f, done, idx, p.N, psi)
            f.flush()
            print(f"{name}: step {done}, mass {m!r}", flush=True)
    print(f"wrote {out}")


def batch():
    inst, steps, ns = BATCH
    params = W.batch_sweep()
    out = os.path.join(HERE, "batch_sweep_long.txt")
    rng = np.random.default_rng(SAMPLE_SEED)
    with open(out, "w") as f:
        f.write(f"# oracle TS2-GauSum (eqs. tssp1-tssp3), workloads.batch_sweep() instances {inst}, "
                f"psi0 = workloads.vortex_lattice_2d(N, L, seed=k), steps={steps}, t0=0; "
                "written by make_long_runs.py\n")
        f.write("# k i0 i1 re im\n")
        for k in inst:
            p = params[k]
            psi0 = W.vortex_lattice_2d(p.N, p.L, seed=k)
            prob = scheme.Problem.from_params(p)
            m0, e0, l0 = scalars(prob, p, psi0, 0.0)
            ref, t = prob.run(psi0, steps, p.dt)
            m, e, lz = scalars(prob, p, ref, t)
            f.write(f"# scalars k={k} step=0 mass={m0!r} energy={e0!r} lz={l0!r}\n")
            f.write(f"# scalars k={k} step={steps} mass={m!r} energy={e!r} lz={lz!r}\n")
            write_samples(f, k, sample_indices(psi0, ns, rng), p.N, ref)
            f.flush()
            print(f"instance {k} N={p.N}: mass {m!r}", flush=True)
    print(f"wrote {out}")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("batch", "all"):
        batch()
    if what in ("case3d", "all"):
        case3d()
    if what in ("plain2d", "all"):
        case3d(full=True)
