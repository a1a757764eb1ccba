"""GPU parity of the split step's adjoint (fse_step_adjoint), the grid
potential (fse_set_potential), Lz psi (fse_apply_Lz) and the autograd wrapper
against the oracle (oracle/adjoint.py), plus finite differences on the GPU.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj
from oracle import diagnostics as dg
from oracle import scheme

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1512_03210_amd import fse  # noqa: E402
from paper_1512_03210_amd import autograd as fag  # noqa: E402


def _note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fse.lib()


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {
    # 2D rotating anisotropic trap, Coulomb kernel, smooth + rough U
    "rot2d": W.Params(d=2, N=(48, 64), L=(6.0, 7.0), s=0.7, Omega=0.5, gamma=(1.0, 1.3), beta=20.0, lam=3.0,
                      kernel="coulomb", coef=1 / (2 * math.pi), dt=0.02, name="rot2d"),
    # 3D rotating z-dipole, ragged radix-3 axis
    "ddi3d": W.Params(d=3, N=(24, 24, 16), L=(5.0, 5.0, 4.0), s=0.9, Omega=0.4, gamma=(1.0, 1.0, 1.5), beta=30.0,
                      lam=8.0, kernel="ddi3", dt=0.02, name="ddi3d"),
    # no nonlocal term, no rotation
    "local2d": W.Params(d=2, N=(32, 32), L=(6.0, 6.0), s=1.2, Omega=0.0, gamma=(1.0, 1.0), beta=50.0, lam=0.0,
                        kernel="none", dt=0.02, name="local2d"),
}


def _setup(name, seed=3):
    p = CASES[name]
    rng = np.random.default_rng(seed)
    X = np.meshgrid(*scheme.axes(p.N, p.L), indexing="ij")
    U = 0.3 * np.sin(X[0]) * np.cos(0.5 * X[1]) + 0.05 * rng.standard_normal(p.N)
    if p.d == 2:
        psi0 = W.harmonic_vortex_2d(p.N, p.L, seed=seed)
    else:
        psi0 = W.anisotropic_gaussian(p.N, p.L, p.gamma, seed=seed)
    tgt = W.adjoint_target(p.N, p.L, seed=seed + 1)
    pr = scheme.Problem.from_params(p)
    pr.U = U
    return p, pr, U, psi0, tgt


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-11), (fse.C64, 2e-5)])
def test_step_with_grid_potential_against_oracle(name, prec, tol):
    p, pr, U, psi0, _ = _setup(name)
    cd, rd = (np.complex128, np.float64) if prec == fse.C128 else (np.complex64, np.float32)
    ref, _ = pr.run(psi0, 5, p.dt)
    plan = fse.Plan.from_params(p, prec)
    Ud = _dev(U, rd)
    plan.set_potential(Ud)
    x = _dev(psi0, cd)
    plan.step(x, 5, p.dt)
    err = _rel(x.cpu().numpy().astype(np.complex128), ref)
    _note(f"[adjoint] step with U {name} prec={prec}: {err:.3e}")
    assert err < tol
    # the energy's potential part includes U
    e = plan.energy(x).cpu().numpy()
    eo = np.array(dg.energy_parts(pr, x.cpu().numpy().astype(np.complex128), t=5 * p.dt))
    assert np.all(np.abs(e - eo) <= (1e-11 if prec == fse.C128 else 1e-5) * np.maximum(1.0, np.abs(eo)))
    plan.set_potential(None)
    y = _dev(psi0, cd)
    plan.time = 0.0
    plan.step(y, 5, p.dt)
    assert _rel(y.cpu().numpy().astype(np.complex128), ref) > 10 * tol  # U really entered


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-11), (fse.C64, 5e-5)])
def test_adjoint_against_oracle(name, prec, tol):
    p, pr, U, psi0, tgt = _setup(name)
    n = 6
    cd, rd = (np.complex128, np.float64) if prec == fse.C128 else (np.complex64, np.float32)
    psiT, _ = pr.run(psi0, n, p.dt)
    _, gT = adj.loss_and_grad(psiT, tgt, p.N, p.L)
    g_ref, gU_ref = adj.run_adjoint(pr, psi0, n, p.dt, gT)
    plan = fse.Plan.from_params(p, prec)
    plan.set_potential(_dev(U, rd))
    g = _dev(gT, cd)
    gU = torch.zeros(p.N, dtype=torch.float64 if prec == fse.C128 else torch.float32, device="cuda:0")
    plan.step_adjoint(_dev(psi0, cd), n, p.dt, g, gU)
    e1 = _rel(g.cpu().numpy().astype(np.complex128), g_ref)
    e2 = _rel(gU.cpu().numpy().astype(np.float64), gU_ref)
    _note(f"[adjoint] {name} prec={prec}: dL/dpsi0 {e1:.3e}, dL/dU {e2:.3e}")
    assert e1 < tol and e2 < tol
    assert plan.time == 0.0


def test_adjoint_segments_compose():
    # two calls over 3 + 4 steps (the second from the state after 3 steps)
    # equal one call over 7 steps
    p, pr, U, psi0, tgt = _setup("rot2d")
    plan = fse.Plan.from_params(p, fse.C128)
    plan.set_potential(_dev(U, np.float64))
    x0 = _dev(psi0, np.complex128)
    x3 = x0.clone()
    plan.step(x3, 3, p.dt)
    gT = _dev(tgt, np.complex128)
    g1 = gT.clone()
    gU1 = torch.zeros(p.N, dtype=torch.float64, device="cuda:0")
    plan.time = 0.0
    plan.step_adjoint(x0, 7, p.dt, g1, gU1)
    g2 = gT.clone()
    gU2 = torch.zeros_like(gU1)
    plan.time = 3 * p.dt
    plan.step_adjoint(x3, 4, p.dt, g2, gU2)
    plan.time = 0.0
    plan.step_adjoint(x0, 3, p.dt, g2, gU2)
    assert _rel(g2.cpu().numpy(), g1.cpu().numpy()) < 1e-12
    assert _rel(gU2.cpu().numpy(), gU1.cpu().numpy()) < 1e-12


@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-10), (fse.C64, 1e-4)])
def test_autograd_with_checkpoints_against_oracle(prec, tol):
    # loss |<psi_t, psi(T)>|^2 + 0.1 <Lz> through evolve() with checkpoints
    # every 3 steps over 10 steps, against the oracle's adjoint
    p, pr, U, psi0, tgt = _setup("rot2d", seed=5)
    n = 10
    cd, rd = (np.complex128, np.float64) if prec == fse.C128 else (np.complex64, np.float32)
    psiT, _ = pr.run(psi0, n, p.dt)
    L_ref, gT = adj.loss_and_grad(psiT, tgt, p.N, p.L)
    g_ref, gU_ref = adj.run_adjoint(pr, psi0, n, p.dt, gT)
    plan = fse.Plan.from_params(p, prec)
    x0 = _dev(psi0, cd).requires_grad_(True)
    Ut = _dev(U, rd).requires_grad_(True)
    t = _dev(tgt, cd)
    vol = math.prod(p.h)
    xT = fag.evolve(plan, x0, Ut, n, p.dt, checkpoint=3)
    o = vol * torch.sum(torch.conj(t) * xT)
    loss = torch.abs(o) ** 2 + 0.1 * fag.angular_momentum(plan, xT)
    loss.backward()
    e0 = abs(float(loss) - L_ref) / abs(L_ref)
    e1 = _rel(x0.grad.cpu().numpy().astype(np.complex128), g_ref)
    e2 = _rel(Ut.grad.cpu().numpy().astype(np.float64), gU_ref)
    _note(f"[adjoint] autograd prec={prec}: loss {e0:.2e}, dL/dpsi0 {e1:.3e}, dL/dU {e2:.3e}")
    assert e0 < tol and e1 < tol and e2 < tol
    assert abs(plan.time - n * p.dt) < 1e-15


def test_gradient_by_finite_differences_on_gpu():
    # directional derivatives of the GPU loss (FP64) against central differences
    p, pr, U, psi0, tgt = _setup("ddi3d", seed=7)
    n = 8
    plan = fse.Plan.from_params(p, fse.C128)
    rng = np.random.default_rng(9)
    vol = math.prod(p.h)
    t = _dev(tgt, np.complex128)

    def loss(x0, Uv):
        plan.time = 0.0
        plan.set_potential(Uv)
        x = x0.clone()
        plan.step(x, n, p.dt)
        o = vol * torch.sum(torch.conj(t) * x)
        return float(torch.abs(o) ** 2 + 0.1 * plan.angular_momentum(x)[0])

    x0 = _dev(psi0, np.complex128).requires_grad_(True)
    Ut = _dev(U, np.float64).requires_grad_(True)
    plan.time = 0.0
    xT = fag.evolve(plan, x0, Ut, n, p.dt, checkpoint=4)
    o = vol * torch.sum(torch.conj(t) * xT)
    (torch.abs(o) ** 2 + 0.1 * fag.angular_momentum(plan, xT)).backward()
    eps = 1e-6
    for k in range(4):
        dpsi = _dev(rng.standard_normal(p.N) + 1j * rng.standard_normal(p.N), np.complex128)
        dU = _dev(rng.standard_normal(p.N), np.float64)
        fd = (loss(x0.detach() + eps * dpsi, (Ut + eps * dU).detach())
              - loss(x0.detach() - eps * dpsi, (Ut - eps * dU).detach())) / (2 * eps)
        an = float(torch.real(torch.sum(torch.conj(x0.grad) * dpsi)) + torch.sum(Ut.grad * dU))
        _note(f"[adjoint] FD direction {k}: fd {fd:.12e} adjoint {an:.12e}")
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-12), (fse.C64, 1e-5)])
def test_apply_Lz_against_oracle(prec, tol):
    p, pr, U, psi0, _ = _setup("ddi3d")
    cd = np.complex128 if prec == fse.C128 else np.complex64
    plan = fse.Plan.from_params(p, prec)
    x = _dev(psi0 * np.exp(0.4j * scheme.axes(p.N, p.L)[0][:, None, None]), cd)
    out = plan.apply_Lz(x).cpu().numpy().astype(np.complex128)
    ref = dg.apply_Lz(x.cpu().numpy().astype(np.complex128), p.N, p.L)
    assert _rel(out, ref) < tol


def test_grid_potential_in_H_and_ground_state_without_rotation():
    p, pr, U, psi0, _ = _setup("local2d")
    plan = fse.Plan.from_params(p, fse.C128)
    plan.set_potential(_dev(U, np.float64))
    x = _dev(psi0, np.complex128)
    H = plan.apply_H(x).cpu().numpy()
    assert _rel(H, dg.apply_H(pr, psi0)) < 1e-12
    from oracle import groundstate as ogs
    g = ogs.GroundState(pr, 0.05)
    ref, _ = g.step(psi0, rtol=1e-12)
    plan.gs_step(x, 0.05, tol=1e-12)
    assert _rel(x.cpu().numpy(), ref) < 1e-10


def test_grid_potential_rejected_with_rotation_where_frames_differ():
    p, pr, U, psi0, _ = _setup("rot2d")
    plan = fse.Plan.from_params(p, fse.C128)
    plan.set_potential(_dev(U, np.float64))
    x = _dev(psi0, np.complex128)
    with pytest.raises(fse.FseError):
        plan.apply_H(x)
    with pytest.raises(fse.FseError):
        plan.gs_step(x, 0.05)
    plan.step(x, 1, p.dt)  # the step itself takes it


def _case_loss_grad(plan, p, psi0, V, tgt, checkpoint):
    """Loss |<psi_t, psi(T)>|^2 + 0.1 <Lz> of the differentiation case through the checkpointed autograd path;
    returns (loss, dL/dpsi0, dL/dV)."""
    import math
    x0 = torch.from_numpy(psi0).to("cuda:0", plan.cdtype).requires_grad_(True)
    U = torch.from_numpy(V).to("cuda:0", plan.rdtype).requires_grad_(True)
    t = torch.from_numpy(tgt).to("cuda:0", plan.cdtype)
    plan.time = 0.0
    xT = fag.evolve(plan, x0, U, p.steps, p.dt, checkpoint)
    o = math.prod(p.h) * torch.sum(torch.conj(t) * xT)
    loss = torch.abs(o) ** 2 + 0.1 * fag.angular_momentum(plan, xT)
    loss.backward()
    return float(loss.detach()), x0.grad.detach(), U.grad.detach()


def _case_fd(p, psi0, V, tgt, gpsi, gV, ndir, eps=1e-5, seed=7):
    """Central differences of the FP64 forward loss in ndir seeded unit directions against Re<g, d>."""
    import math
    plan = fse.Plan.from_params(p, fse.C128)
    vol = math.prod(p.h)
    t = torch.from_numpy(tgt).to("cuda:0")
    x0, U0 = torch.from_numpy(psi0).to("cuda:0"), torch.from_numpy(V).to("cuda:0")

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
        dp, dv = torch.from_numpy(dpsi).to("cuda:0"), torch.from_numpy(dV).to("cuda:0")
        fd = (loss(x0 + eps * dp, (U0 + eps * dv).contiguous()) - loss(x0 - eps * dp, (U0 - eps * dv).contiguous())) / (2 * eps)
        an = float(torch.real(torch.sum(torch.conj(gpsi.to(torch.complex128)) * dp)) + torch.sum(gV.double() * dv))
        errs.append(abs(an - fd) / max(abs(fd), 1e-300))
    return errs


def test_full_size_differentiation_case():
    # the 96^3 case over 200 steps with a checkpoint every 20: FP64 adjoint
    # against central differences of the FP64 forward (4 directions), and the
    # complex64 gradients against the FP64 ones
    p = W.preset("adjoint3d_96")
    psi0, V, tgt = W.adjoint_case_inputs(p)
    _note(f"[adjoint] full size {p.N}, {p.steps} steps")
    res = {}
    for prec in (fse.C128, fse.C64):
        plan = fse.Plan.from_params(p, prec)
        res[prec] = _case_loss_grad(plan, p, psi0, V, tgt, 20)
        del plan
    L128, gp128, gv128 = res[fse.C128]
    L64, gp64, gv64 = res[fse.C64]
    errs = _case_fd(p, psi0, V, tgt, gp128, gv128, 4)
    e_psi = float(torch.linalg.vector_norm((gp64.to(torch.complex128) - gp128).flatten())
                  / torch.linalg.vector_norm(gp128.flatten()))
    e_v = float(torch.linalg.vector_norm((gv64.double() - gv128).flatten()) / torch.linalg.vector_norm(gv128.flatten()))
    _note(f"[adjoint] full size: FD rel errs {errs}; c64 vs c128: dpsi0 {e_psi:.3e}, dV {e_v:.3e}, "
          f"loss {L64:.8f} vs {L128:.8f}")
    assert max(errs) < 1e-6
    assert e_psi < 1e-3 and e_v < 1e-3
    # complex64 loss: a state error of at most 1e-6 relative per step (the one-step measurements are 3e-7 to
    # 7e-7), growing at most linearly over the 200 steps, doubled by the quadratic loss: 4e-4
    assert abs(L64 - L128) < 2 * p.steps * 1e-6 * abs(L128)


@pytest.mark.parametrize("prec,tol", [(fse.C128, 1e-9), (fse.C64, 5e-4)])
def test_full_size_differentiation_case_against_oracle_samples(prec, tol):
    """The benchmarked 96^3 differentiation case (200 steps, U = |x|^2/2, loss
    |<psi_t, psi(T)>|^2 + 0.1 <Lz>): dL/dpsi0 and dL/dU from fse_step_adjoint
    against the oracle's at 4096 stored points (tests/golden/make_adjoint3d_96_samples.py
    writes them); dL/dpsi(T) is the oracle's loss gradient at the library's own final state."""
    import os
    p = W.preset("adjoint3d_96")
    rows = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint3d_96_grad.txt"),
                      comments="#")
    idx = np.ravel_multi_index((rows[:, 0].astype(int), rows[:, 1].astype(int), rows[:, 2].astype(int)), p.N)
    g_ref, u_ref = rows[:, 3] + 1j * rows[:, 4], rows[:, 5]
    cd, rd = (np.complex128, np.float64) if prec == fse.C128 else (np.complex64, np.float32)
    psi0 = W.anisotropic_gaussian(p.N, p.L, (1.0, 1.0, 1.0), seed=0)
    V = W.harmonic_potential(p.N, p.L, (1.0, 1.0, 1.0))
    tgt = W.adjoint_target(p.N, p.L, seed=1)
    plan = fse.Plan.from_params(p, prec)
    Ud = _dev(V, rd)
    plan.set_potential(Ud)
    x = _dev(psi0, cd)
    plan.step(x, 200, p.dt)
    _, gT = adj.loss_and_grad(x.cpu().numpy().astype(np.complex128), tgt, p.N, p.L)
    plan.time = 0.0
    g = _dev(gT, cd)
    gU = torch.zeros(p.N, dtype=torch.float64 if prec == fse.C128 else torch.float32, device="cuda:0")
    plan.step_adjoint(_dev(psi0, cd), 200, p.dt, g, gU)
    it = torch.from_numpy(idx).to("cuda:0")
    e1 = _rel(g.reshape(-1)[it].cpu().numpy().astype(np.complex128), g_ref)
    e2 = _rel(gU.reshape(-1)[it].cpu().numpy().astype(np.float64), u_ref)
    _note(f"[adjoint] 96^3 x 200 steps prec={prec}: dL/dpsi0 {e1:.3e}, dL/dU {e2:.3e} at the stored points")
    assert e1 < tol and e2 < tol
