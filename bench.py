#!/usr/bin/env python3
"""Benchmark of the TS2-GauSum split step on one MI355X.

Default workload: the 3D 256^3 split step (grid [-12,12]^3, s = 0.8,
Omega = 0.7, gamma = (1,1,2), beta = 200, lambda = 50, dipole along z via
GauSum on 512^3 padding, dt = 5e-4), complex128, synthetic seeded Gaussian
initial state resident in HBM before the timed region.  One step = one pass
of the whole hot path (linear half steps merged across steps, GauSum
potential, nonlinear phase).  The timed region is one fse_step call of K
steps after W warm-up steps.

Prints one JSON line: the headline value is complex128 grid-point-steps/s;
the complex64 path is reported under "variants"; per-pass average durations
(HIP events on the launch stream) give the roofline of the dominant kernel;
the FP64 CPU oracle, timed on a bounded sample, is "cpu_baseline".
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point-steps/s and % HBM roofline, 3D 256³ split step, FP32-batched vs FP64"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_split_step_256cube.json")


def kernel_source_hash():
    """Hash of the HIP sources: measured traffic is only reported for the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1512_03210_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hpp", ".inc", ".hip")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(pass_name, precision):
    """HBM bytes per launch from the rocprofv3 counter runs, if taken on the current kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    entry = rec.get("passes", {}).get(precision, {}).get(pass_name)
    return None if entry is None else entry["read_bytes"] + entry["write_bytes"]
HBM_PEAK_GBS = 8000.0


def pass_bytes(p, csize):
    """Algorithmic HBM bytes per launch of each pass kind (compulsory reads + writes)."""
    rsize = csize // 2
    n = p.npts
    if p.kernel == "none" or p.lam == 0.0:
        # no nonlocal term: the phase pass reads and writes the state only
        kin = 1
        for Nj in p.N:
            kin *= Nj // 2 + 1
        out = {"c2r_phase": 2 * n * csize, "kin": 2 * n * csize + kin * csize, "edge": 2 * n * csize}
        if p.d == 3:
            out.update(f1=2 * n * csize, i1=2 * n * csize)
        return out
    if p.d == 3:
        N0, N1, N2 = p.N
        X1 = (N0 + 1) * N1 * N2
        X2 = (N0 + 1) * 2 * N1 * N2
        K = (N0 + 1) * (N1 + 1) * (N2 + 1)
        kin = (N0 // 2 + 1) * (N1 // 2 + 1) * (N2 // 2 + 1)
        return {
            "r2c": (n + X1) * csize,
            "pad_fwd": (X1 + X2) * csize,
            "conv": 2 * X2 * csize + K * rsize,
            "crop_inv": (X2 + X1) * csize,
            "c2r_phase": (X1 + 2 * n) * csize,
            "f1": 2 * n * csize,
            "kin": 2 * n * csize + kin * csize,
            "i1": 2 * n * csize,
            "edge": 2 * n * csize,
        }
    N0, N1 = p.N
    X1 = (N0 + 1) * N1
    K = (N0 + 1) * (N1 + 1)
    kin = (N0 // 2 + 1) * (N1 // 2 + 1)
    return {
        "r2c": (n + X1) * csize,
        "conv": 2 * X1 * csize + K * rsize,
        "c2r_phase": (X1 + 2 * n) * csize,
        "kin": 2 * n * csize + kin * csize,
        "edge": 2 * n * csize,
    }


def oracle_errors(state, idx, ref, scal, ref_scal):
    """Errors against the stored FP64 oracle values of a run (tests/golden/*_long.txt, written by a committed
    script that calls only the oracle): the state's relative L2 error over the stored points, |dmass|, the
    relative energy error and |d<Lz>|."""
    import numpy as np
    v = state[idx]
    return {"state_rel_l2": float(np.linalg.norm(v - ref) / np.linalg.norm(ref)),
            "mass_abs": abs(scal[0] - ref_scal[0]),
            "energy_rel": abs(scal[1] - ref_scal[1]) / abs(ref_scal[1]),
            "lz_abs": abs(scal[2] - ref_scal[2])}


def run_precision(p, prec, steps, warmup, prof_steps, tune=True):
    import numpy as np
    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    psi0 = W.initial_state(p, seed=0)
    dtype = np.complex128 if prec == fse.C128 else np.complex64
    csize = 16 if prec == fse.C128 else 8
    plan = fse.Plan.from_params(p, prec)
    default_schedule = plan.schedule()["schedule"]
    sched = plan.tune() if tune else plan.schedule()
    x = torch.from_numpy(psi0.astype(dtype)).to("cuda:0")
    del psi0
    if warmup > 0:
        plan.step(x, warmup, p.dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    plan.step(x, steps, p.dt)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    mass = plan.mass(x).item()
    # per-pass durations: HIP events around every launch, on the launch stream
    plan.set_profiling(True)
    plan.step(x, prof_steps, p.dt)
    torch.cuda.synchronize()
    prof = plan.profile()
    plan.set_profiling(False)
    by = pass_bytes(p, csize)
    passes = {}
    for name, (ms, cnt) in prof.items():
        avg = ms / cnt
        passes[name] = {
            "launches": cnt,
            "avg_ms": round(avg, 5),
            "bytes_per_launch": by[name],
            "gbs": round(by[name] / (avg * 1e-3) / 1e9, 1),
            "share": None,
        }
    tot = sum(v["avg_ms"] * v["launches"] for k, v in passes.items() if k != "edge")
    for k, v in passes.items():
        if k != "edge":
            v["share"] = round(v["avg_ms"] * v["launches"] / tot, 4)
    step_bytes = sum(v for k, v in by.items() if k != "edge")
    t_step = ev_ms * 1e-3 / steps
    del x, plan
    torch.cuda.empty_cache()
    return {
        "value": p.npts * steps / (ev_ms * 1e-3),
        "ms_per_step": ev_ms / steps,
        "wall_s": wall,
        "mass_after": mass,
        "model_bytes_per_point": step_bytes / p.npts,
        "step_hbm_gbs": step_bytes / t_step / 1e9,
        "step_hbm_frac": step_bytes / t_step / 1e9 / HBM_PEAK_GBS,
        "passes": passes,
        "schedule": {"default": default_schedule, "used": sched["schedule"], "tuned_ms": sched["tuned_ms"],
                     "tuned": tune},
    }


def run_batch(steps):
    """The batched sweep (64 2D instances, complex64, one graph): its first call of `steps` steps from psi0
    (graph capture included) gives the per-instance error against the stored oracle values at that step; a
    replay of the same graph is timed.  The same instances run one by one through the FP64 single-instance
    step give the speed-up."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    params = W.batch_sweep(steps=steps)
    states = [W.vortex_lattice_2d(p.N, p.L, seed=k) for k, p in enumerate(params)]
    npts = sum(p.npts for p in params)
    b = fse.Batch(params, fse.C64)
    x = b.pack(states)
    b.step(x, steps)  # from psi0: captures the graph for this step count and runs it
    torch.cuda.synchronize()
    err = None
    if steps == 500:
        scal, samples = W.stored_long_run("batch_sweep")
        red = b.reduce(x).cpu().numpy()
        st = b.unpack(x)
        err = {}
        for k in sorted(samples):
            pl = fse.Plan.from_params(params[k], fse.C64)
            lz = pl.angular_momentum(torch.from_numpy(np.ascontiguousarray(st[k])).cuda()).item()
            idx, ref = samples[k]
            err[f"instance_{k}_{params[k].N[0]}^2"] = oracle_errors(
                st[k].astype(np.complex128), idx, ref, (red[k, 0], red[k, 6], lz), scal[(k, steps)])
            del pl
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(x, steps)  # replay
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    red = b.reduce(x).cpu().numpy()
    del b, x
    # the same instances through the FP64 single-instance path, one at a time
    plans = [fse.Plan.from_params(p, fse.C128) for p in params]
    ys = [torch.from_numpy(s).cuda() for s in states]
    for pl, y, p in zip(plans, ys, params):
        pl.step(y, 5, p.dt)
    torch.cuda.synchronize()
    e0.record()
    for pl, y, p in zip(plans, ys, params):
        pl.step(y, steps, p.dt)
    e1.record()
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1)
    del plans, ys
    torch.cuda.empty_cache()
    sizes = sorted({p.N[0] for p in params})
    return {
        "workload": (f"{len(params)} 2D instances, 16 each of " + ", ".join(f"{n}^2" for n in sizes)
                     + ", s~U[0.3,1], Omega~U[0,0.9], beta=500, Coulomb GauSum, vortex-lattice psi0"),
        "steps": steps,
        "value": npts * steps / (ms * 1e-3),
        "unit": "grid-point-steps/s",
        "dtype": "f32 (complex64; FP64 reductions)",
        "ms_per_step": ms / steps,
        "fp64_single_one_by_one_value": npts * steps / (ms64 * 1e-3),
        "speedup_vs_fp64_single": ms64 / ms,
        "error_vs_oracle_at_step_500": err,
        "max_mass_drift_after_two_calls": float(np.max(np.abs(red[:, 0] - 1.0))),
    }


def run_case(p, prec, steps, warmup=5, keep=None, stored=None):
    """Throughput of one fse_step call of `steps` steps of a named case, and the
    drift of its invariants (mass, energy, <Lz>) over those steps.  With keep (a
    dict), the final state and scalars are stored there for comparison."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    psi0 = W.initial_state(p, seed=0)
    dtype = np.complex128 if prec == fse.C128 else np.complex64
    plan = fse.Plan.from_params(p, prec)
    x = torch.from_numpy(psi0.astype(dtype)).to("cuda:0")
    if warmup > 0:  # on a copy: the measured run starts from psi0 at t = 0
        w = x.clone()
        plan.step(w, warmup, p.dt)
        del w
        plan.time = 0.0
    m0, e0, l0 = plan.mass(x).item(), plan.energy(x)[5].item(), plan.angular_momentum(x).item()
    torch.cuda.synchronize()
    e_0, e_1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_0.record()
    plan.step(x, steps, p.dt)
    e_1.record()
    torch.cuda.synchronize()
    ms = e_0.elapsed_time(e_1)
    m1, e1, l1 = plan.mass(x).item(), plan.energy(x)[5].item(), plan.angular_momentum(x).item()
    err = None
    scal, samples = W.stored_long_run(stored) if stored else ({}, {})
    if steps in samples:
        idx, ref = samples[steps]
        err = oracle_errors(x.cpu().numpy().astype(np.complex128), idx, ref, (m1, e1, l1), scal[steps])
    if keep is not None:
        keep.update(state=x.to(torch.complex128), mass=m1, energy=e1, lz=l1)
    del plan, x
    torch.cuda.empty_cache()
    return {
        "steps": steps,
        "value": p.npts * steps / (ms * 1e-3),
        "unit": "grid-point-steps/s",
        "ms_per_step": ms / steps,
        "drift": {"mass_abs": abs(m1 - m0), "energy_rel": abs(e1 - e0) / abs(e0), "lz_abs": abs(l1 - l0)},
        "error_vs_oracle": err,
    }


def run_ops(p, prec, reps=10):
    """Per-call time of the FP64 reductions and of H psi on the headline grid."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    psi0 = W.initial_state(p, seed=0)
    dtype = np.complex128 if prec == fse.C128 else np.complex64
    csize = 16 if prec == fse.C128 else 8
    plan = fse.Plan.from_params(p, prec)
    x = torch.from_numpy(psi0.astype(dtype)).to("cuda:0")
    del psi0
    rho = (x.real * x.real + x.imag * x.imag).contiguous()
    out = torch.empty_like(x)
    calls = {
        "mass": lambda: plan.mass(x),
        "energy": lambda: plan.energy(x),
        "angular_momentum": lambda: plan.angular_momentum(x),
        "moments": lambda: plan.moments(x),
        "apply_H": lambda: plan.apply_H(x, out),
        "apply_H_frozen_rho": lambda: plan.apply_H(x, out, rho_frozen=rho),
    }
    res = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, f in calls.items():
        f()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": round(ms, 4), "grid_points_per_s": p.npts / (ms * 1e-3)}
    # the mass is one read of psi
    res["mass"]["gbs"] = round(p.npts * csize / (res["mass"]["ms"] * 1e-3) / 1e9, 1)
    del plan, x, out, rho
    torch.cuda.empty_cache()
    return res


def run_order4(p, prec, steps=20, warmup=2):
    """Fourth-order steps (triple-jump composition of the TS2 step) on the
    headline grid: time per step and its ratio to the TS2 step."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    psi0 = W.initial_state(p, seed=0)
    dtype = np.complex128 if prec == fse.C128 else np.complex64
    plan = fse.Plan.from_params(p, prec)
    x = torch.from_numpy(psi0.astype(dtype)).to("cuda:0")
    del psi0
    plan.step(x, warmup, p.dt, order=4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.step(x, steps, p.dt, order=4)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    mass = plan.mass(x).item()
    del plan, x
    torch.cuda.empty_cache()
    return {"steps": steps, "ms_per_step": round(ms, 4), "grid_point_steps_per_s": p.npts / (ms * 1e-3),
            "mass_after": mass}


def adjoint_loss_grad(plan, p, psi0, V, tgt, checkpoint):
    """Loss |<psi_t, psi(T)>|^2 + 0.1 <Lz> through the checkpointed adjoint; returns
    (loss, dL/dpsi0, dL/dV, forward seconds, backward seconds)."""
    import torch

    from paper_1512_03210_amd import autograd as fag

    x0 = torch.from_numpy(psi0).to("cuda:0", plan.cdtype).requires_grad_(True)
    U = torch.from_numpy(V).to("cuda:0", plan.rdtype).requires_grad_(True)
    t = torch.from_numpy(tgt).to("cuda:0", plan.cdtype)
    vol = math.prod(p.h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.time = 0.0
    xT = fag.evolve(plan, x0, U, p.steps, p.dt, checkpoint)
    o = vol * torch.sum(torch.conj(t) * xT)
    loss = torch.abs(o) ** 2 + 0.1 * fag.angular_momentum(plan, xT)
    lv = float(loss.detach())
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return lv, x0.grad.detach(), U.grad.detach(), t1 - t0, t2 - t1


def adjoint_fd(p, psi0, V, tgt, gpsi, gV, ndir, eps=1e-5, seed=7):
    """Central differences of the FP64 forward loss in ndir seeded directions
    (dpsi complex, dV real, each of unit discrete norm) against the adjoint's
    directional derivative Re <gpsi, dpsi> + <gV, dV> (sums, no volume factor)."""
    import numpy as np
    import torch

    from paper_1512_03210_amd import fse

    plan = fse.Plan.from_params(p, fse.C128)
    vol = math.prod(p.h)
    t = torch.from_numpy(tgt).to("cuda:0")
    x0 = torch.from_numpy(psi0).to("cuda:0")
    U0 = torch.from_numpy(V).to("cuda:0")
    gp = gpsi.to(torch.complex128)
    gv = gV.to(torch.float64)

    def loss(x, Uv):
        plan.time = 0.0
        plan.set_potential(Uv)
        x = x.clone()
        plan.step(x, p.steps, p.dt)
        o = vol * torch.sum(torch.conj(t) * x)
        return float(torch.abs(o) ** 2 + 0.1 * plan.angular_momentum(x)[0])

    rng = np.random.default_rng(seed)
    errs = []
    for _ in range(ndir):
        dpsi = rng.standard_normal(p.N) + 1j * rng.standard_normal(p.N)
        dpsi /= math.sqrt(vol * float(np.sum(np.abs(dpsi) ** 2)))
        dV = rng.standard_normal(p.N)
        dV /= math.sqrt(vol * float(np.sum(dV ** 2)))
        dp = torch.from_numpy(dpsi).to("cuda:0")
        dv = torch.from_numpy(dV).to("cuda:0")
        fd = (loss(x0 + eps * dp, (U0 + eps * dv).contiguous())
              - loss(x0 - eps * dp, (U0 - eps * dv).contiguous())) / (2 * eps)
        an = float(torch.real(torch.sum(torch.conj(gp) * dp)) + torch.sum(gv * dv))
        errs.append(abs(an - fd) / max(abs(fd), 1e-300))
    del plan
    return errs


def run_adjoint(p, checkpoint=20, ndir=32):
    """The differentiation case: nsteps steps forward with a checkpoint every
    `checkpoint` steps, the loss, and the adjoint back to psi0 and V, in
    complex64 and complex128; central finite differences of the FP64 forward
    in ndir directions check both gradients."""
    import statistics

    import torch

    from paper_1512_03210_amd import fse

    import workloads as W
    psi0, V, tgt = W.adjoint_case_inputs(p)
    out = {"checkpoint": checkpoint, "steps": p.steps}
    grads = {}
    for name, prec in (("c64", fse.C64), ("c128", fse.C128)):
        plan = fse.Plan.from_params(p, prec)
        adjoint_loss_grad(plan, p, psi0, V, tgt, checkpoint)  # warm-up: workspace, tables
        lv, gpsi, gV, tf, tb = adjoint_loss_grad(plan, p, psi0, V, tgt, checkpoint)
        grads[name] = (gpsi, gV)
        out[name] = {"loss": lv, "forward_ms": round(1e3 * tf, 3), "backward_ms": round(1e3 * tb, 3),
                     "forward_ms_per_step": round(1e3 * tf / p.steps, 4),
                     "backward_ms_per_step": round(1e3 * tb / p.steps, 4),
                     "backward_over_forward": round(tb / tf, 2)}
        del plan
        torch.cuda.empty_cache()
    g64, g128 = grads["c64"], grads["c128"]

    def rel(a, b):
        return float(torch.linalg.vector_norm((a.to(b.dtype) - b).flatten()) / torch.linalg.vector_norm(b.flatten()))
    out["c64_vs_c128_rel_l2"] = {"dL_dpsi0": rel(g64[0], g128[0]), "dL_dV": rel(g64[1], g128[1])}
    for name in ("c128", "c64"):
        errs = adjoint_fd(p, psi0, V, tgt, grads[name][0], grads[name][1], ndir)
        out[name]["fd_directions"] = ndir
        out[name]["fd_rel_err_max"] = max(errs)
        out[name]["fd_rel_err_median"] = statistics.median(errs)
    return out


def run_gs(p, prec, max_steps, tol, eps_energy=1e-8, maxit=200):
    """Ground-state steps (backward-Euler GFDN, preconditioned BiCGStab) from the rotating initial guess until
    the energy changes by at most eps_energy (fse_gs_run) or max_steps steps have run; time per step and per
    Krylov iteration, and the energy trace."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    psi0 = W.ground_state_guess(p.N, p.L, p.Omega, p.gamma, seed=0)
    dtype = np.complex128 if prec == fse.C128 else np.complex64
    plan = fse.Plan.from_params(p, prec)
    x = torch.from_numpy(psi0.astype(dtype)).to("cuda:0")
    del psi0
    plan.gs_step(x.clone(), p.dt, tol=tol, maxit=2)  # first call allocates the solver vectors
    plan.energy(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = plan.gs_run(x, p.dt, eps_energy=eps_energy, max_steps=max_steps, tol=tol, maxit=maxit)
    sec = time.perf_counter() - t0
    del plan, x
    torch.cuda.empty_cache()
    return {
        "max_steps": max_steps,
        "stop_rule": f"|E^(n+1) - E^n| <= {eps_energy:g}",
        "steps": st["steps"],
        "converged": st["converged"],
        "krylov_tol": tol,
        "ms_per_step": 1e3 * sec / st["steps"],
        "krylov_iterations": st["krylov_iterations"],
        "ms_per_krylov_iteration": 1e3 * sec / max(st["krylov_iterations"], 1),
        "energy_trace": st["energies"],
        "last_energy_change": st["energy_change"],
        "diff_inf_last": st["diff_inf"],
        "note": ("these parameters (s < 1, Omega > 0, attractive 3D dipole) lie where the paper's theory gives no "
                 "continuum ground state: per-step cost and the energy trace are reported, not convergence"),
    }


def copy_bandwidth(nbytes=4 << 30, reps=5):
    """Achieved bandwidth of the library's copy kernel, plain and with non-temporal loads and stores, on
    buffers of nbytes each (read + write bytes / time; 4 GiB each: far beyond the 256 MB last-level cache)."""
    import torch

    from paper_1512_03210_amd import fse

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for nt in (False, True):
        fse.device_copy(b, a, nbytes, nontemporal=nt)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fse.device_copy(b, a, nbytes, nontemporal=nt)
        e1.record()
        torch.cuda.synchronize()
        out["nontemporal" if nt else "plain"] = round(2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(p, nsteps=2):
    """The FP64 oracle on a bounded sample: nsteps steps of the same workload, its FFTs on the host cores this
    process may use (scipy's pocketfft, oracle._fft.WORKERS threads), pointwise numpy work on one."""
    import numpy as np

    import workloads as W
    from oracle import _fft, scheme

    psi = W.initial_state(p, seed=0)
    pr = scheme.Problem.from_params(p)
    # The multiplier's values do not change the cost of a step; building the
    # oracle's own multiplier is plan-time work that takes minutes at 512^3.
    pr._K = np.ones(tuple(2 * n for n in p.N))
    t = 0.0
    psi, t = pr.step(psi, t, p.dt)  # warm-up (FFT plans, page faults)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        psi, t = pr.step(psi, t, p.dt)
    sec = time.perf_counter() - t0
    return {
        "value": p.npts * nsteps / sec,
        "unit": "grid-point-steps/s",
        "cores": _fft.WORKERS,
        "cpu_model": cpu_model(),
        "os_cpu_count": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"{nsteps} step(s) of the {p.N[0]}^3 workload after one warm-up step by "
                   f"oracle.scheme.Problem.step (float64; FFTs by scipy.fft with {_fft.WORKERS} workers, "
                   f"pointwise numpy on one thread), {sec:.1f} s; GauSum multiplier replaced by a "
                   f"same-shape array (plan-time work excluded)"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="dipole3d_256", choices=["dipole3d_256", "dipole3d_128", "plain2d"])
    ap.add_argument("--prof-steps", type=int, default=20)
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="time the default pass schedule instead of the autotuned one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=500, help="steps of the batched sweep (0: skip)")
    ap.add_argument("--gs-steps", type=int, default=4,
                    help="at most this many ground-state steps at 256^3 complex64 (energy-change rule 1e-8; 0: skip)")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="skip the differentiation case (96^3, 200 steps, adjoint with checkpoints)")
    ap.add_argument("--no-cases", dest="cases", action="store_false",
                    help="skip the 128^3 (1000 steps) and 64^2 (100 steps) cases")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the split step of one grid is not sharded here "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_1512_03210_amd import fse

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    p = W.preset(args.workload)
    print(f"[bench] {p.name} N={p.N} c128: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    r64 = run_precision(p, fse.C128, args.steps, args.warmup, args.prof_steps, args.tune)
    print(f"[bench] c128 {r64['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    variants = {}
    if not args.no_c64:
        r32 = run_precision(p, fse.C64, args.steps, args.warmup, args.prof_steps, args.tune)
        print(f"[bench] c64 {r32['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        variants["c64"] = {
            "value": r32["value"], "ms_per_step": r32["ms_per_step"], "dtype": "f32 (complex64; FP64 reductions)",
            "step_hbm_frac": r32["step_hbm_frac"], "model_bytes_per_point": r32["model_bytes_per_point"],
            "speedup_vs_c128": r32["value"] / r64["value"], "passes": r32["passes"], "schedule": r32["schedule"],
        }
    ql = p.replace(lam=0.0, name=p.name + "-local")
    print(f"[bench] {ql.name}: lambda = 0", file=sys.stderr, flush=True)
    rl = run_precision(ql, fse.C128, args.steps, args.warmup, args.prof_steps, args.tune)
    variants["local_c128"] = {
        "workload": "the same 256^3 step without the nonlocal term (lambda = 0)",
        "value": rl["value"], "ms_per_step": rl["ms_per_step"], "dtype": "f64",
        "step_hbm_frac": rl["step_hbm_frac"], "model_bytes_per_point": rl["model_bytes_per_point"],
        "passes": rl["passes"],
    }
    print(f"[bench] local c128 {rl['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    print("[bench] reductions and H psi", file=sys.stderr, flush=True)
    ops = {"c128": run_ops(p, fse.C128)}
    if not args.no_c64:
        ops["c64"] = run_ops(p, fse.C64)
    print("[bench] fourth-order steps", file=sys.stderr, flush=True)
    order4 = {"c128": run_order4(p, fse.C128)}
    order4["c128"]["cost_vs_ts2"] = round(order4["c128"]["ms_per_step"] / r64["ms_per_step"], 3)
    if not args.no_c64:
        order4["c64"] = run_order4(p, fse.C64)
        order4["c64"]["cost_vs_ts2"] = round(order4["c64"]["ms_per_step"] / r32["ms_per_step"], 3)
    cases = {}
    if args.cases:
        for name, steps in (("dipole3d_128", 1000), ("plain2d", 1000)):
            q = W.preset(name)
            print(f"[bench] case {q.name}: {steps} steps", file=sys.stderr, flush=True)
            cases[q.name] = {"c128": run_case(q, fse.C128, steps, stored=name)}
            if not args.no_c64:
                cases[q.name]["c64"] = run_case(q, fse.C64, steps, stored=name)
            torch.cuda.empty_cache()
    gs = None
    if args.gs_steps > 0:
        q = W.preset("gs3d_256")
        print(f"[bench] ground state {q.name}: {args.gs_steps} steps", file=sys.stderr, flush=True)
        gs = {"workload": (f"{q.name}: {'x'.join(map(str, q.N))} on [-{q.L[0]:g},{q.L[0]:g}]^3, s={q.s}, "
                           f"Omega={q.Omega}, beta={q.beta}, lambda={q.lam} z-dipole GauSum, dt={q.dt}, "
                           "initial guess ((1-Omega) phi_ho + Omega phi_ho^v) x z-Gaussian"),
              "c64": run_gs(q, fse.C64, args.gs_steps, 1e-6)}
        print(f"[bench] ground state {gs['c64']['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    adjoint = None
    if args.adjoint:
        q = W.preset("adjoint3d_96")
        print(f"[bench] differentiation case {q.name}: {q.steps} steps, adjoint", file=sys.stderr, flush=True)
        adjoint = {"workload": (f"{q.name}: {'x'.join(map(str, q.N))} on [-{q.L[0]:g},{q.L[0]:g}]^3, s={q.s}, "
                                f"Omega={q.Omega}, beta={q.beta}, lambda={q.lam} Coulomb GauSum on "
                                f"{'x'.join(str(2 * n) for n in q.N)}, V(x) = |x|^2/2 as a grid potential, "
                                f"dt={q.dt}, loss |<psi_t, psi(T)>|^2 + 0.1 <Lz>"),
                   **run_adjoint(q)}
    if args.batch_steps > 0:
        print(f"[bench] batched sweep, {args.batch_steps} steps", file=sys.stderr, flush=True)
        variants["batch_c64"] = run_batch(args.batch_steps)
        print(f"[bench] batch {variants['batch_c64']['ms_per_step']:.3f} ms/step, speedup "
              f"{variants['batch_c64']['speedup_vs_fp64_single']:.2f}x", file=sys.stderr, flush=True)
    dom = max((k for k in r64["passes"] if k != "edge"),
              key=lambda k: r64["passes"][k]["avg_ms"] * r64["passes"][k]["launches"])
    dp = r64["passes"][dom]
    roof = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": dp["gbs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(dp["gbs"] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom, "c128"),
        "bytes_per_launch": dp["bytes_per_launch"],
        "avg_ms": dp["avg_ms"],
    }
    copy = copy_bandwidth()
    print(f"[bench] copy kernel {copy} GB/s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(p)
    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{p.name}: {'x'.join(map(str, p.N))} grid on [-{p.L[0]:g},{p.L[0]:g}]^{p.d}, "
                         f"s={p.s}, Omega={p.Omega}, gamma={p.gamma}, beta={p.beta}, lambda={p.lam}, "
                         f"kernel={p.kernel} GauSum on {'x'.join(str(2 * n) for n in p.N)} padding, dt={p.dt}"),
            "grid": list(p.N),
            "precision": "complex128",
        },
        "step_hbm_frac": r64["step_hbm_frac"],
        "copy_kernel_gbs": copy,
        "model_bytes_per_point": r64["model_bytes_per_point"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
        "reductions_and_H": ops,
        "fourth_order": order4,
        "cases": cases,
        "ground_state": gs,
        "differentiation": adjoint,
        "passes": r64["passes"],
        "schedule": r64["schedule"],
        "mass_after": r64["mass_after"],
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
