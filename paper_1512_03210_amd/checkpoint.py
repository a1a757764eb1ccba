"""Checkpoint / resume and a diagnostics log for split-step runs (host-side helpers; the paper has neither).

A checkpoint is the state psi in a safetensors file (as its real view, so that complex128 and complex64 round-trip
exactly) plus a JSON file with the time t, the precision and the problem parameters (any dataclass or mapping of
plain values, e.g. the parameter sets used by the tests and the benchmark).  Given the plan, it also keeps what the
plan holds beyond the parameters: the grid potential of set_potential (in the safetensors file, in the plan's
precision), the optical lattice of set_lattice, the pass schedule and the kernel options (delta, ht) the plan was
built with.  Resuming rebuilds the plan from all of it, sets its time and continues: splitting a run into calls is
exact algebra apart from the one merged half kinetic step that each call boundary undoes (round-off only).

run_logged advances a plan in chunks of `every` steps and appends one JSON line per chunk with t, the mass, the
energy parts and <Lz> (computed on the device, read back once per chunk).
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Any, Mapping

import torch
from safetensors.torch import load_file, save_file

from . import fse

_PREC = {fse.C128: "c128", fse.C64: "c64"}
_PREC_BACK = {v: k for k, v in _PREC.items()}


def _plain(params) -> dict:
    d = dataclasses.asdict(params) if dataclasses.is_dataclass(params) else dict(params)
    return {k: list(v) if isinstance(v, tuple) else v for k, v in d.items()}


def save(prefix: str, params: Any, psi: torch.Tensor, t: float, precision: int, plan: "fse.Plan | None" = None) -> None:
    """Write prefix.safetensors (psi, and the plan's grid potential U if any) and prefix.json (t, precision,
    params, and the plan's lattice, schedule and kernel options).  Without `plan` only params, psi and t are
    kept: the plan must then be one that from_params(params) rebuilds."""
    if precision not in _PREC:
        raise ValueError(f"unknown precision {precision}")
    want = torch.complex128 if precision == fse.C128 else torch.complex64
    if psi.dtype != want:
        raise ValueError(f"psi is {psi.dtype}, the precision says {want}")
    tensors = {"psi": torch.view_as_real(psi.detach().contiguous()).cpu()}
    meta = {"t": float(t), "precision": _PREC[precision], "shape": list(psi.shape), "params": _plain(params)}
    if plan is not None:
        if plan.precision != precision:
            raise ValueError("the plan's precision differs from the checkpoint's")
        if plan._U is not None:
            tensors["U"] = plan._U.detach().contiguous().cpu()
        meta["plan"] = {"lattice": plan._lattice, "schedule": plan.schedule()["schedule"],
                        "kernel_options": dict(plan._kernel_kw)}
    save_file(tensors, prefix + ".safetensors")
    tmp = prefix + ".json.tmp"
    with open(tmp, "w") as f:
        json.dump(meta, f, indent=1)
    os.replace(tmp, prefix + ".json")


def load(prefix: str, device: str = "cuda:0"):
    """(params dict, psi on device, t, precision) of a checkpoint written by save."""
    params, psi, t, prec, _ = load_full(prefix, device)
    return params, psi, t, prec


def load_full(prefix: str, device: str = "cuda:0"):
    """As load, plus the plan state: {"lattice", "schedule", "kernel_options", "U" (tensor on device or None)}
    (None if the checkpoint was saved without its plan)."""
    with open(prefix + ".json") as f:
        meta = json.load(f)
    tensors = load_file(prefix + ".safetensors")
    psi = torch.view_as_complex(tensors["psi"]).contiguous()
    if list(psi.shape) != meta["shape"]:
        raise ValueError(f"checkpoint state has shape {list(psi.shape)}, its metadata says {meta['shape']}")
    st = meta.get("plan")
    if st is not None:
        st = dict(st)
        st["U"] = tensors["U"].to(device) if "U" in tensors else None
    return meta["params"], psi.to(device), float(meta["t"]), _PREC_BACK[meta["precision"]], st


def resume(prefix: str, params_type, device: str = "cuda:0"):
    """(plan, psi, params) ready to continue: params = params_type(**stored fields, lists as tuples), the type
    the checkpoint was written from (it may derive further values, such as the kernel prefactor, from its
    fields), the plan built from it with the stored kernel options, grid potential, lattice and schedule, and
    its time set to the stored t."""
    pd, psi, t, prec, st = load_full(prefix, device)
    fields = {f.name for f in dataclasses.fields(params_type)} if dataclasses.is_dataclass(params_type) else None
    kw = {k: tuple(v) if isinstance(v, list) else v for k, v in pd.items() if fields is None or k in fields}
    params = params_type(**kw)
    plan = fse.Plan.from_params(params, prec, **((st or {}).get("kernel_options") or {}))
    if st is not None:
        if st.get("lattice") is not None:
            plan.set_lattice(*st["lattice"])
        if st.get("U") is not None:
            plan.set_potential(st["U"].contiguous())
        plan.set_schedule(st["schedule"])
    plan.time = t
    return plan, psi, params


def run_logged(plan: "fse.Plan", psi: torch.Tensor, nsteps: int, dt: float, every: int, log_path: str,
               order: int = 2) -> None:
    """nsteps steps in chunks of `every`, one JSON line per chunk appended to log_path:
    {"t", "steps", "mass", "energy": {kin, pot, int, non, rot, total}, "lz"}."""
    if every <= 0:
        raise ValueError("every must be positive")
    names = ["kin", "pot", "int", "non", "rot", "total"]
    done = 0
    with open(log_path, "a") as f:
        while done < nsteps:
            k = min(every, nsteps - done)
            plan.step(psi, k, dt, order=order)
            done += k
            vals = torch.cat([plan.mass(psi), plan.energy(psi), plan.angular_momentum(psi)]).cpu().tolist()
            rec: Mapping[str, Any] = {"t": plan.time, "steps": done, "mass": vals[0],
                                      "energy": dict(zip(names, vals[1:7])), "lz": vals[7]}
            f.write(json.dumps(rec) + "\n")
            f.flush()
