"""Stored oracle fixtures under tests/golden/ stay consistent with the workloads they were written for.

dipole3d_256_step1.txt and dipole3d_256_step2.txt hold one and two of the FP64 oracle's TS2-GauSum steps
(eqs. tssp1-tssp3) of the 256^3 dipolar workload at sampled points, dipole3d_256_order4_step1.txt one
fourth-order step, dipole3d_256_local_step{1,2}.txt the same workload with lam = 0,
dipole3d_256_tiles_step1.txt one step at points that cover every column tile;
tests/golden/make_dipole3d_256_step.py writes them and the GPU parity suite compares the
library's steps there.  If the workload's parameters or
initial state change, the fixtures must be written again: these checks fail first.
"""
import os
import re

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# (file, steps, order, local)
FIXTURES = [("dipole3d_256_step1.txt", 1, 2, False), ("dipole3d_256_step2.txt", 2, 2, False),
            ("dipole3d_256_order4_step1.txt", 1, 4, False), ("dipole3d_256_local_step1.txt", 1, 2, True),
            ("dipole3d_256_local_step2.txt", 2, 2, True)]


def _workload(local):
    p = W.preset("dipole3d_256")
    return p.replace(lam=0.0) if local else p


def _path(name):
    return os.path.join(GOLDEN, name)


def _header(path):
    with open(path) as f:
        lines = [next(f) for _ in range(3)]
    return " ".join(lines)


@pytest.mark.parametrize("name,steps,order,local", FIXTURES)
def test_fixture_records_the_current_workload(name, steps, order, local):
    p = _workload(local)
    h = _header(_path(name))
    for key, val in [("N", p.N), ("L", p.L), ("s", p.s), ("Omega", p.Omega), ("beta", p.beta), ("lam", p.lam),
                     ("kernel", p.kernel), ("dt", p.dt)]:
        assert f"{key}={val}" in h, (key, val, h)
    order_field = rf" order={order};" if order != 2 else r"( order=2;)?"
    assert re.search(rf"initial_state\(seed=0\); steps={steps};{order_field} t0=0", h)


@pytest.mark.parametrize("name,steps,order,local", FIXTURES)
def test_fixture_samples_are_distinct_finite_and_cover_the_condensate(name, steps, order, local):
    p = _workload(local)
    r = np.loadtxt(_path(name), comments="#")
    assert r.shape == (4096, 5) or (r.shape[1] == 5 and 4000 <= r.shape[0] <= 4096)
    ijk = r[:, :3].astype(int)
    assert np.all(ijk >= 0) and np.all(ijk < np.array(p.N))
    assert len({tuple(x) for x in ijk}) == r.shape[0]
    v = r[:, 3] + 1j * r[:, 4]
    assert np.all(np.isfinite(v))
    # the condensate half of the samples carries most of the mass; a step or two
    # of size dt change |psi| there by far less than its size
    psi0 = W.initial_state(p, seed=0)
    a0 = np.abs(psi0[ijk[:, 0], ijk[:, 1], ijk[:, 2]])
    core = a0 >= 1e-2 * np.abs(psi0).max()
    assert core.sum() >= 2048
    rel = np.linalg.norm(np.abs(v[core]) - a0[core]) / np.linalg.norm(a0[core])
    assert rel < 0.05


def test_tile_fixture_puts_one_point_in_every_column_tile():
    path = _path("dipole3d_256_tiles_step1.txt")
    p = _workload(False)
    h = _header(path)
    for key, val in [("N", p.N), ("L", p.L), ("beta", p.beta), ("lam", p.lam), ("dt", p.dt)]:
        assert f"{key}={val}" in h, (key, val, h)
    assert re.search(r"initial_state\(seed=0\); steps=1;( order=2;)? t0=0", h)
    r = np.loadtxt(path, comments="#")
    i0, i1, i2 = (r[:, k].astype(int) for k in range(3))
    n = p.N[1] * p.N[2] // 8
    assert r.shape == (n, 5) and np.all(np.isfinite(r[:, 3:]))
    assert len(set(zip(i1, i2 // 8))) == n  # axis-0 passes: columns (i1, i2), tiles of 8 along i2
    assert len(set(zip(i0, i2 // 8))) == n  # axis-1 passes: columns (i0, i2)
    assert len(set(zip(i0, i1))) == n       # distinct lines of the contiguous axis


def test_batch_fixture_covers_one_instance_of_each_size():
    path = _path("batch_sweep_step5.txt")
    h = _header(path)
    assert "steps=5, t0=0" in h and "instances (0, 17, 38, 63)" in h
    r = np.loadtxt(path, comments="#")
    params = W.batch_sweep()
    ks = sorted(set(r[:, 0].astype(int)))
    assert ks == [0, 17, 38, 63]
    assert sorted({params[k].N for k in ks}) == [(128, 128), (256, 256), (384, 384), (512, 512)]
    for k in ks:
        rk = r[r[:, 0] == k]
        ij = rk[:, 1:3].astype(int)
        assert np.all(ij >= 0) and np.all(ij < np.array(params[k].N))
        assert len({tuple(x) for x in ij}) == rk.shape[0] >= 900
        assert np.all(np.isfinite(rk[:, 3:5]))


def test_groundstate_fixture_records_the_current_workload():
    p = W.preset("gs3d_256")
    path = _path("groundstate3d_256_step1.txt")
    h = _header(path)
    for key, val in [("N", p.N), ("L", p.L), ("s", p.s), ("Omega", p.Omega), ("beta", p.beta), ("lam", p.lam),
                     ("kernel", p.kernel), ("dt", p.dt)]:
        assert f"{key}={val}" in h, (key, val, h)
    r = np.loadtxt(path, comments="#")
    ijk = r[:, :3].astype(int)
    assert np.all(ijk >= 0) and np.all(ijk < np.array(p.N))
    assert len({tuple(x) for x in ijk}) == r.shape[0] >= 4000
    assert np.all(np.isfinite(r[:, 3:5]))


def test_adjoint_fixture_records_the_current_workload():
    p = W.preset("adjoint3d_96")
    path = _path("adjoint3d_96_grad.txt")
    h = _header(path)
    for key, val in [("N", p.N), ("L", p.L), ("s", p.s), ("Omega", p.Omega), ("beta", p.beta), ("lam", p.lam),
                     ("kernel", p.kernel), ("dt", p.dt)]:
        assert f"{key}={val}" in h, (key, val, h)
    assert "adjoint of 200 TS2-GauSum steps" in h
    r = np.loadtxt(path, comments="#")
    assert r.shape[1] == 6 and r.shape[0] >= 4000
    ijk = r[:, :3].astype(int)
    assert np.all(ijk >= 0) and np.all(ijk < np.array(p.N))
    assert len({tuple(x) for x in ijk}) == r.shape[0]
    assert np.all(np.isfinite(r[:, 3:6]))
