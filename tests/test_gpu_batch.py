"""GPU parity of the batched 2D sweep (graph-captured, one branch per grid size)."""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as dg
from oracle import scheme

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402


def _note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


def _instances():
    base = dict(L=(8.0, 8.0), beta=100.0, lam=1.0, kernel="coulomb", mu=1.0)
    return [
        W.Params(d=2, N=(64, 64), s=0.75, Omega=0.5, gamma=(1.0, 1.0), dt=1e-3, name="a", **base),
        W.Params(d=2, N=(64, 64), s=0.4, Omega=0.9, gamma=(1.0, 1.3), dt=2e-3, name="b", **base),
        W.Params(d=2, N=(96, 96), s=1.1, Omega=0.2, gamma=(1.2, 1.0), dt=1e-3, name="c", **base),
        W.Params(d=2, N=(64, 48), s=0.9, Omega=0.0, gamma=(1.0, 1.0), dt=5e-4, name="d", **base),
        W.Params(d=2, N=(128, 128), s=0.6, Omega=0.7, gamma=(1.0, 1.0), dt=1e-3, name="e",
                 **dict(base, beta=500.0)),
        W.Params(d=2, N=(64, 64), s=0.8, Omega=0.3, gamma=(1.0, 1.1), dt=1e-3, name="f",
                 **dict(base, lam=0.0, kernel="none")),
    ]


def _states(params, seed0=10):
    return [W.harmonic_vortex_2d(p.N, p.L, seed=seed0 + k) for k, p in enumerate(params)]


def _oracle(params, states, nsteps):
    out = []
    for p, s in zip(params, states):
        pr = scheme.Problem.from_params(p)
        out.append(pr.run(s, nsteps, p.dt)[0])
    return out


@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-11), (fse.C64, 1e-5)])
def test_batch_matches_oracle_per_instance(prec, tol):
    params = _instances()
    states = _states(params)
    ref = _oracle(params, states, 4)
    b = fse.Batch(params, prec)
    x = b.pack(states)
    b.step(x, 4)
    torch.cuda.synchronize()
    for k, (got, r) in enumerate(zip(b.unpack(x), ref)):
        err = float(np.linalg.norm(got - r) / np.linalg.norm(r))
        _note(f"[batch] prec={prec} instance {params[k].name} N={params[k].N}: {err:.3e}")
        assert err < tol
    assert np.allclose(b.times(), [4 * p.dt for p in params], rtol=0, atol=1e-15)


def test_batch_fp64_with_512_point_convolution_lines():
    # a 256-point contiguous axis pads to 512-point convolution lines: in FP64 these exchange one component at a
    # time through half-size LDS lines, inside the batch's own kernels too
    base = dict(L=(8.0, 8.0), beta=100.0, lam=1.0, kernel="coulomb", mu=1.0)
    params = [W.Params(d=2, N=(48, 256), s=0.8, Omega=0.5, gamma=(1.0, 1.2), dt=1e-3, name="w", **base),
              W.Params(d=2, N=(64, 64), s=0.7, Omega=0.3, gamma=(1.0, 1.0), dt=1e-3, name="s", **base)]
    states = _states(params, seed0=40)
    ref = _oracle(params, states, 3)
    b = fse.Batch(params, fse.C128)
    x = b.pack(states)
    b.step(x, 3)
    torch.cuda.synchronize()
    for k, (got, r) in enumerate(zip(b.unpack(x), ref)):
        err = float(np.linalg.norm(got - r) / np.linalg.norm(r))
        _note(f"[batch] FP64 instance {params[k].name} N={params[k].N}: {err:.3e}")
        assert err < 1e-11


def test_batch_graph_replays_with_eager_work_between():
    params = _instances()
    states = _states(params, seed0=20)
    b = fse.Batch(params, fse.C128)
    x = b.pack(states)
    other = fse.Plan.from_params(W.preset("plain2d"), fse.C128)
    y = torch.from_numpy(W.harmonic_vortex_2d((64, 64), (8.0, 8.0), seed=1)).cuda()
    for rep in range(1, 4):
        b.step(x, 2)          # first call captures, the others replay the same graph
        other.step(y, 3, 1e-3)  # unrelated eager work between replays
        torch.cuda.synchronize()
        ref = _oracle(params, states, 2 * rep)
        for k, (got, r) in enumerate(zip(b.unpack(x), ref)):
            err = float(np.linalg.norm(got - r) / np.linalg.norm(r))
            assert err < 1e-11, (rep, k, err)


def test_batch_equals_single_instance_plans():
    params = _instances()
    states = _states(params, seed0=30)
    b = fse.Batch(params, fse.C64)
    x = b.pack(states)
    b.step(x, 3)
    got = b.unpack(x)
    for k, p in enumerate(params):
        plan = fse.Plan.from_params(p, fse.C64)
        y = torch.from_numpy(states[k].astype(np.complex64)).cuda()
        plan.step(y, 3, p.dt)
        err = float(np.linalg.norm(got[k] - y.cpu().numpy()) / np.linalg.norm(got[k]))
        assert err < 1e-6, (k, err)


def test_batch_reduce():
    params = _instances()
    states = _states(params, seed0=40)
    b = fse.Batch(params, fse.C128)
    x = b.pack(states)
    b.step(x, 3)
    red = b.reduce(x).cpu().numpy()
    for k, (p, s) in enumerate(zip(params, b.unpack(x))):
        pr = scheme.Problem.from_params(p)
        eo = np.array(dg.energy_parts(pr, s, t=3 * p.dt))
        assert abs(red[k, 0] - dg.mass(s, p.N, p.L)) < 1e-12
        assert np.all(np.abs(red[k, 1:] - eo) <= 1e-11 * np.maximum(1.0, np.abs(eo)))


def test_batch_invalid():
    bad = _instances()[:1] + [W.Params(d=2, N=(62, 64), L=(8.0, 8.0), s=0.5, Omega=0.1, gamma=(1.0, 1.0),
                                       beta=1.0, lam=1.0, dt=1e-3)]
    with pytest.raises(fse.FseError):
        fse.Batch(bad, fse.C64)


def _sweep_samples():
    """{instance: (flat indices, oracle values)} of tests/golden/batch_sweep_step5.txt (five oracle steps;
    tests/golden/make_batch_sweep_samples.py writes it)."""
    rows = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_sweep_step5.txt"),
                      comments="#")
    params = W.batch_sweep()
    out = {}
    for k in np.unique(rows[:, 0]).astype(int):
        r = rows[rows[:, 0] == k]
        idx = np.ravel_multi_index((r[:, 1].astype(int), r[:, 2].astype(int)), params[k].N)
        out[k] = (idx, r[:, 3] + 1j * r[:, 4])
    return out


def test_full_sweep_sampled_against_fp64_single_plans_and_the_oracle():
    # The benchmarked sweep: 64 instances, 16 each of 128^2, 256^2, 384^2, 512^2; one instance of every
    # size against the FP64 single plan (whole state) and both against stored oracle samples.
    params = W.batch_sweep()
    states = [W.vortex_lattice_2d(p.N, p.L, seed=k) for k, p in enumerate(params)]
    samples = _sweep_samples()
    b = fse.Batch(params, fse.C64)
    x = b.pack(states)
    b.step(x, 5)
    red = b.reduce(x).cpu().numpy()
    got = b.unpack(x)
    for k in (0, 17, 38, 63):  # one instance of every size
        p = params[k]
        plan = fse.Plan.from_params(p, fse.C128)
        y = torch.from_numpy(states[k]).cuda()
        plan.step(y, 5, p.dt)
        ref = y.cpu().numpy()
        err = float(np.linalg.norm(got[k] - ref) / np.linalg.norm(ref))
        idx, orc = samples[k]
        e128 = float(np.linalg.norm(ref.ravel()[idx] - orc) / np.linalg.norm(orc))
        e64 = float(np.linalg.norm(got[k].ravel()[idx] - orc) / np.linalg.norm(orc))
        _note(f"[sweep] instance {k} N={p.N} s={p.s:.3f} Omega={p.Omega:.3f}: c64 vs c128 {err:.3e}; "
              f"oracle samples: c128 {e128:.3e}, batch c64 {e64:.3e}")
        assert err < 1e-5 and e128 < 1e-12 and e64 < 1e-5
    assert np.max(np.abs(red[:, 0] - 1.0)) < 1e-5


def test_batch_dipole_instances_keep_their_own_axis():
    # instances on one grid share a multiplier only when the kernel matches,
    # dipole axis included
    base = dict(d=2, N=(64, 64), L=(8.0, 8.0), s=0.8, gamma=(1.0, 1.0), beta=50.0, lam=-6.0, kernel="ddi2",
                dt=1e-3)
    params = [
        W.Params(Omega=0.4, axis=(0.0, 0.0, 1.0), name="z", **base),
        W.Params(Omega=0.0, axis=(1.0, 0.0, 0.0), name="x", **base),
        W.Params(Omega=0.0, axis=(0.0, 0.6, 0.8), name="yz", **base),
        W.Params(Omega=0.0, axis=(1.0, 0.0, 0.0), name="x2", **dict(base, lam=4.0)),
    ]
    states = _states(params, seed0=50)
    ref = _oracle(params, states, 3)
    b = fse.Batch(params, fse.C128)
    x = b.pack(states)
    b.step(x, 3)
    torch.cuda.synchronize()
    for k, (got, r) in enumerate(zip(b.unpack(x), ref)):
        err = float(np.linalg.norm(got - r) / np.linalg.norm(r))
        _note(f"[batch] dipole instance {params[k].name}: {err:.3e}")
        assert err < 1e-11


def test_complex64_batch_mass_renormalisation():
    # complex64, 300 steps in one call: with the FP64 renormalisation (the default) every instance returns the
    # mass it was given; without it the FP32 twiddle residuals bias the mass; the state against the FP64 batch
    # does not get worse
    params = _instances()
    states = _states(params, seed0=50)
    nsteps = 300
    out = {}
    for on in (True, False):
        b = fse.Batch(params, fse.C64)
        enabled, rn = b.mass_renorm()
        assert enabled and np.all(rn == 1.0)  # on by default, factor 1 before the first call
        b.set_mass_renorm(on)
        x = b.pack(states)
        m0 = b.reduce(x)[:, 0].cpu().numpy()
        b.step(x, nsteps)
        m1 = b.reduce(x)[:, 0].cpu().numpy()
        out[on] = ((m1 - m0) / m0, b.mass_renorm(), b.unpack(x))
    ref = fse.Batch(params, fse.C128)
    assert not ref.mass_renorm()[0]  # off for complex128
    y = ref.pack(states)
    ref.step(y, nsteps)
    ry = ref.unpack(y)
    e_on = [float(np.linalg.norm(a - r) / np.linalg.norm(r)) for a, r in zip(out[True][2], ry)]
    e_off = [float(np.linalg.norm(a - r) / np.linalg.norm(r)) for a, r in zip(out[False][2], ry)]
    _note(f"[batch renorm] relative dmass on {np.abs(out[True][0]).max():.2e}, off {np.abs(out[False][0]).max():.2e}; "
          f"factors {out[True][1][1][:, 0]}; state vs FP64 on {max(e_on):.3e}, off {max(e_off):.3e}")
    # the exit transform, after the mass is measured, adds its own FP32 rounding (~1e-8)
    assert np.abs(out[True][0]).max() < 1e-7
    f = out[True][1][1][:, 0]
    assert np.all(np.abs(f - 1.0) < 1e-3) and np.any(f != 1.0)
    # the start mass the call recorded is the reduced input mass
    assert np.allclose(out[True][1][1][:, 2], m0, rtol=1e-12, atol=0)
    assert not out[False][1][0]
    assert sum(e_on) <= sum(e_off) * 1.05


def test_batch_mass_renorm_switch_records_the_graph_again():
    # the same buffer and step count after switching the renormalisation off: the cached graph (which holds the
    # renormalising passes) must be recorded again, so the second call leaves the factors alone and the mass drifts
    params = _instances()
    states = _states(params, seed0=60)
    b = fse.Batch(params, fse.C64)
    x = b.pack(states)
    b.step(x, 200)
    f1 = b.mass_renorm()[1].copy()
    m1 = b.reduce(x)[:, 0].cpu().numpy()
    b.set_mass_renorm(False)
    b.step(x, 200)
    enabled, f2 = b.mass_renorm()
    m2 = b.reduce(x)[:, 0].cpu().numpy()
    _note(f"[batch renorm] after switching off: relative dmass {np.abs((m2 - m1) / m1).max():.2e}")
    assert not enabled and np.array_equal(f1, f2)
    assert np.abs((m2 - m1) / m1).max() > 1e-7
    b.set_mass_renorm(True)
    b.step(x, 200)
    m3 = b.reduce(x)[:, 0].cpu().numpy()
    assert np.abs((m3 - m2) / m2).max() < 1e-7 and not np.array_equal(b.mass_renorm()[1], f2)
