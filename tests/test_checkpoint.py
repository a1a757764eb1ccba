"""Checkpoint files round-trip exactly (host side; no GPU needed)."""
import dataclasses
import os

import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_1512_03210_amd import checkpoint, fse  # noqa: E402


@pytest.mark.parametrize("prec,dtype", [(fse.C128, torch.complex128), (fse.C64, torch.complex64)])
def test_save_load_round_trip_is_exact(tmp_path, prec, dtype):
    p = W.preset("plain2d")
    psi = torch.from_numpy(W.harmonic_vortex_2d(p.N, p.L, seed=4)).to(dtype)
    prefix = os.path.join(tmp_path, "ck")
    checkpoint.save(prefix, p, psi, 0.125, prec)
    pd, back, t, pr = checkpoint.load(prefix, device="cpu")
    assert back.dtype == dtype and torch.equal(back, psi)
    assert t == 0.125 and pr == prec
    want = {k: list(v) if isinstance(v, tuple) else v for k, v in dataclasses.asdict(p).items()}
    assert pd == want


def test_save_rejects_a_state_of_the_wrong_precision(tmp_path):
    p = W.preset("plain2d")
    psi = torch.zeros(p.N, dtype=torch.complex64)
    with pytest.raises(ValueError):
        checkpoint.save(os.path.join(tmp_path, "ck"), p, psi, 0.0, fse.C128)


def test_load_checks_the_stored_shape(tmp_path):
    p = W.preset("plain2d")
    prefix = os.path.join(tmp_path, "ck")
    checkpoint.save(prefix, p, torch.zeros(p.N, dtype=torch.complex128), 0.0, fse.C128)
    import json
    with open(prefix + ".json") as f:
        meta = json.load(f)
    meta["shape"] = [1, 2]
    with open(prefix + ".json", "w") as f:
        json.dump(meta, f)
    with pytest.raises(ValueError):
        checkpoint.load(prefix, device="cpu")


def test_plan_state_is_stored_and_read_back(tmp_path):
    # the plan's grid potential, lattice, schedule and kernel options go into the files (a bare binding object
    # stands in for the plan: no GPU here)
    p = W.preset("plain2d")
    plan = fse.Plan.__new__(fse.Plan)
    plan.precision = fse.C128
    plan._U = torch.arange(p.npts, dtype=torch.float64).reshape(p.N)
    plan._lattice = ([10.0, 10.0], [3.14, 3.14])
    plan._kernel_kw = {"delta": 1e-3, "ht": 0.12}
    plan.schedule = lambda: {"schedule": [1, 0, 0], "tuned_ms": [-1] * 8}
    prefix = os.path.join(tmp_path, "ck")
    psi = torch.zeros(p.N, dtype=torch.complex128)
    checkpoint.save(prefix, p, psi, 0.5, fse.C128, plan=plan)
    _, _, t, pr, st = checkpoint.load_full(prefix, device="cpu")
    assert (t, pr) == (0.5, fse.C128)
    assert torch.equal(st["U"], plan._U)
    assert st["lattice"] == [[10.0, 10.0], [3.14, 3.14]] and st["schedule"] == [1, 0, 0]
    assert st["kernel_options"] == {"delta": 1e-3, "ht": 0.12}
    checkpoint.save(prefix, p, psi, 0.5, fse.C128)  # without the plan: no plan state
    assert checkpoint.load_full(prefix, device="cpu")[4] is None
