"""Thin ctypes binding of libfse.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors to device pointers and HIP streams, and status codes to exceptions.
There is no CPU fallback: if libfse.so is missing the import of the library
raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FSE_LIB", os.path.join(_PKG, "libfse.so"))

FSE_OK = 0
STATUS = {0: "FSE_OK", -1: "FSE_ERR_ARG", -2: "FSE_ERR_UNSUPPORTED", -3: "FSE_ERR_NOMEM",
          -4: "FSE_ERR_HIP", -5: "FSE_ERR_NUMERIC", -6: "FSE_ERR_STATE"}
STATUS_CODES = {name: code for code, name in STATUS.items()}
C128, C64 = 0, 1
NSCHED = 5  # FSE_NSCHED: entries of a pass schedule
K_NONE, K_COULOMB, K_DDI3, K_DDI2 = 0, 1, 2, 3
KERNEL_KINDS = {"none": K_NONE, "coulomb": K_COULOMB, "ddi3": K_DDI3, "ddi2": K_DDI2}

EXPORTS = [
    "fse_plan_check", "fse_plan_create", "fse_plan_destroy", "fse_workspace_size", "fse_scratch_size",
    "fse_set_workspace",
    "fse_set_time", "fse_get_time", "fse_step", "fse_step4", "fse_plan_tune", "fse_plan_get_schedule", "fse_plan_set_schedule",
    "fse_set_potential", "fse_set_lattice", "fse_step_adjoint", "fse_apply_Lz", "fse_apply_H", "fse_nonlocal_potential",
    "fse_mass", "fse_energy", "fse_angular_momentum", "fse_moments", "fse_gausum_symbol_host",
    "fse_get_symbol", "fse_last_error", "fse_version", "fse_set_profiling", "fse_get_profile",
    "fse_device_copy", "fse_batch_create", "fse_batch_destroy", "fse_batch_offsets", "fse_batch_step",
    "fse_batch_reduce", "fse_batch_times", "fse_gs_step", "fse_set_guard", "fse_guard_status",
    "fse_mass_noalloc", "fse_gs_run", "fse_angular_momentum_grad", "fse_set_mass_renorm", "fse_get_mass_renorm",
    "fse_device_copy_nt", "fse_batch_set_mass_renorm", "fse_batch_get_mass_renorm",
]
PASS_NAMES = ["edge", "r2c", "pad_fwd", "conv", "crop_inv", "c2r_phase", "f1", "kin", "i1"]


class FseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("mu", ctypes.c_double), ("prefactor", ctypes.c_double),
                ("n", ctypes.c_double * 3), ("delta", ctypes.c_double), ("ht", ctypes.c_double)]


class GsStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("residual", ctypes.c_double),
                ("diff_inf", ctypes.c_double)]


class GsRunStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("converged", ctypes.c_int), ("rule", ctypes.c_int),
                ("krylov_iterations", ctypes.c_int), ("diff_inf", ctypes.c_double), ("energy", ctypes.c_double),
                ("energy_change", ctypes.c_double), ("residual", ctypes.c_double)]


class Instance(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int * 2), ("L", ctypes.c_double * 2), ("s", ctypes.c_double),
                ("Omega", ctypes.c_double), ("gamma", ctypes.c_double * 2), ("beta", ctypes.c_double),
                ("lam", ctypes.c_double), ("dt", ctypes.c_double), ("m", ctypes.c_double), ("kernel", Kernel)]


_lib = None


def lib():
    """Load libfse.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1512_03210_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, st = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    kp = ctypes.POINTER(Kernel)
    sig = {
        "fse_plan_check": (st, [i, ip, dp, d, d, dp, d, d, kp, i]),
        "fse_plan_create": (st, [ctypes.POINTER(vp), i, ip, dp, d, d, dp, d, d, kp, i, d, vp]),
        "fse_plan_destroy": (st, [vp]),
        "fse_workspace_size": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "fse_scratch_size": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "fse_set_workspace": (st, [vp, vp, ctypes.c_size_t]),
        "fse_set_time": (st, [vp, d]),
        "fse_get_time": (st, [vp, dp]),
        "fse_step": (st, [vp, vp, i, d, vp]),
        "fse_step4": (st, [vp, vp, i, d, vp]),
        "fse_set_guard": (st, [vp, d]),
        "fse_set_mass_renorm": (st, [vp, i]),
        "fse_get_mass_renorm": (st, [vp, ip, dp]),
        "fse_guard_status": (st, [vp, ip, dp]),
        "fse_set_potential": (st, [vp, vp]),
        "fse_set_lattice": (st, [vp, dp, dp]),
        "fse_plan_tune": (st, [vp, ctypes.c_char_p, vp]),
        "fse_plan_get_schedule": (st, [vp, ip, dp]),
        "fse_plan_set_schedule": (st, [vp, ip]),
        "fse_step_adjoint": (st, [vp, vp, i, d, vp, vp, vp]),
        "fse_apply_Lz": (st, [vp, vp, vp, vp]),
        "fse_angular_momentum_grad": (st, [vp, vp, vp, vp, vp]),
        "fse_apply_H": (st, [vp, vp, vp, vp, vp]),
        "fse_nonlocal_potential": (st, [vp, vp, vp, vp]),
        "fse_mass": (st, [vp, vp, vp, vp]),
        "fse_mass_noalloc": (st, [vp, vp, vp, vp]),
        "fse_energy": (st, [vp, vp, vp, vp]),
        "fse_angular_momentum": (st, [vp, vp, vp, vp]),
        "fse_moments": (st, [vp, vp, vp, vp]),
        "fse_gausum_symbol_host": (st, [i, ip, dp, kp, dp]),
        "fse_get_symbol": (st, [vp, dp]),
        "fse_last_error": (ctypes.c_char_p, []),
        "fse_version": (ctypes.c_char_p, []),
        "fse_set_profiling": (st, [vp, i]),
        "fse_get_profile": (st, [vp, dp, ip, i]),
        "fse_device_copy": (st, [vp, vp, ctypes.c_size_t, vp]),
        "fse_device_copy_nt": (st, [vp, vp, ctypes.c_size_t, vp]),
        "fse_batch_create": (st, [ctypes.POINTER(vp), i, ctypes.POINTER(Instance), i, vp]),
        "fse_batch_destroy": (st, [vp]),
        "fse_batch_offsets": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "fse_batch_step": (st, [vp, vp, i, vp]),
        "fse_batch_reduce": (st, [vp, vp, vp, vp]),
        "fse_batch_times": (st, [vp, dp]),
        "fse_batch_set_mass_renorm": (st, [vp, i]),
        "fse_batch_get_mass_renorm": (st, [vp, ip, dp]),
        "fse_gs_step": (st, [vp, vp, d, d, i, ctypes.POINTER(GsStats), vp]),
        "fse_gs_run": (st, [vp, vp, d, d, i, i, d, d, dp, ctypes.POINTER(GsRunStats), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != FSE_OK:
        raise FseError(status, lib().fse_last_error().decode())


def make_kernel(kind: str = "coulomb", mu: float = 1.0, prefactor: float = 1.0,
                axis=(0.0, 0.0, 1.0), delta: float = 0.0, ht: float = 0.0) -> Kernel:
    k = Kernel()
    k.kind = KERNEL_KINDS[kind]
    k.mu = mu
    k.prefactor = prefactor
    k.n = (ctypes.c_double * 3)(*axis)
    k.delta = delta
    k.ht = ht
    return k


def _iarr(v):
    return (ctypes.c_int * len(v))(*[int(x) for x in v])


def _darr(v):
    return (ctypes.c_double * len(v))(*[float(x) for x in v])


def _check_axes(d, **arrays):
    """The library reads d values from each per-axis array: refuse shorter ones here (a d other than 2 or 3 the
    library rejects before it reads any array)."""
    if int(d) not in (2, 3):
        return
    for name, a in arrays.items():
        if a is None or len(a) < int(d):
            raise ValueError(f"{name} needs {int(d)} values (one per axis)")


def plan_check(d, N, L, s, Omega, gamma, beta, lam, kernel: Optional[Kernel], precision=C128) -> int:
    """Host-only validation; returns the status code (no exception; arrays shorter than d raise ValueError)."""
    _check_axes(d, N=N, L=L, gamma=gamma)
    return lib().fse_plan_check(d, _iarr(N), _darr(L), s, Omega, _darr(gamma), beta, lam,
                                ctypes.byref(kernel) if kernel is not None else None, precision)


def gausum_symbol_host(d, N, L, kernel: Kernel) -> np.ndarray:
    """The multiplier on the non-negative frequency octant, shape (N_j + 1,) per axis (host)."""
    _check_axes(d, N=N, L=L)
    shape = tuple(int(n) + 1 for n in N)
    out = np.zeros(int(np.prod(shape)), dtype=np.float64)
    _check(lib().fse_gausum_symbol_host(d, _iarr(N), _darr(L), ctypes.byref(kernel),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(shape)


def device_copy(dst, src, nbytes: int, stream=None, nontemporal: bool = False):
    """Streaming copy kernel (HBM calibration); dst/src are device tensors; nontemporal: loads and stores that
    bypass the caches (fse_device_copy_nt)."""
    fn = lib().fse_device_copy_nt if nontemporal else lib().fse_device_copy
    _check(fn(_ptr(dst), _ptr(src), int(nbytes), _stream(stream)))


def version() -> str:
    return lib().fse_version().decode()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """One grid + parameter set; wraps fse_plan (device memory owned by the library).

    psi tensors are torch complex128 (precision C128) or complex64 (C64) on the
    current HIP device, C-contiguous with shape N.
    """

    def __init__(self, d: int, N: Sequence[int], L: Sequence[float], s: float, Omega: float,
                 gamma: Sequence[float], beta: float, lam: float, kernel: Optional[Kernel] = None,
                 precision: int = C128, m: float = 0.0, stream=None):
        import torch
        _check_axes(d, N=N, L=L, gamma=gamma)
        self.d, self.N, self.L = int(d), tuple(int(n) for n in N), tuple(float(x) for x in L)
        self.precision = precision
        self.cdtype = torch.complex128 if precision == C128 else torch.complex64
        self.rdtype = torch.float64 if precision == C128 else torch.float32
        self._h = ctypes.c_void_p()
        self._U = None
        self._ws = None
        self._lattice = None  # (v, k) as set by set_lattice, for checkpoints
        self._kernel_kw = {}  # kernel options beyond the parameter set (delta, ht), for checkpoints
        _check(lib().fse_plan_create(ctypes.byref(self._h), self.d, _iarr(self.N), _darr(self.L), s, Omega,
                                     _darr(gamma), beta, lam,
                                     ctypes.byref(kernel) if kernel is not None else None,
                                     precision, m, _stream(stream)))

    @classmethod
    def from_params(cls, p, precision=C128, stream=None, **kw):
        """Plan of a parameter set; kw: further kernel options (delta, ht of make_kernel)."""
        kern = None if p.kernel == "none" else make_kernel(p.kernel, mu=p.mu, prefactor=p.c, axis=p.axis, **kw)
        plan = cls(p.d, p.N, p.L, p.s, p.Omega, p.gamma, p.beta, p.lam, kern, precision, p.m, stream)
        plan._kernel_kw = {k: float(v) for k, v in kw.items()}
        return plan

    def close(self):
        if self._h:
            _check(lib().fse_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_psi(self, psi):
        if psi.dtype != self.cdtype or tuple(psi.shape) != self.N or not psi.is_contiguous() or not psi.is_cuda:
            raise ValueError(f"psi must be a contiguous {self.cdtype} device tensor of shape {self.N}")

    def _check_real(self, a, what):
        if a.dtype != self.rdtype or tuple(a.shape) != self.N or not a.is_contiguous() or not a.is_cuda:
            raise ValueError(f"{what} must be a contiguous {self.rdtype} device tensor of shape {self.N}")

    def tune(self, cache_path: Optional[str] = None, stream=None) -> dict:
        """Time the plan's schedule alternatives and keep the fastest (fse_plan_tune)."""
        _check(lib().fse_plan_tune(self._h, None if cache_path is None else cache_path.encode(), _stream(stream)))
        return self.schedule()

    def schedule(self) -> dict:
        """{"schedule": [kinetic radix, convolution radix, kinetic order, column plan, fused phase plan],
        "tuned_ms": ms per step of schedule {k, c, o, v, f} at index k + 2c + 4o + 8v + 16f (-1: not timed)}"""
        sc = (ctypes.c_int * NSCHED)()
        ms = (ctypes.c_double * (1 << NSCHED))()
        _check(lib().fse_plan_get_schedule(self._h, sc, ms))
        return {"schedule": [int(x) for x in sc], "tuned_ms": [float(x) for x in ms]}

    def set_schedule(self, sched):
        """Force a schedule (a list of NSCHED entries 0 or 1; a shorter list is completed with zeros)."""
        sched = list(sched) + [0] * (NSCHED - len(sched))
        if len(sched) != NSCHED:
            raise ValueError(f"a schedule has {NSCHED} entries")
        _check(lib().fse_plan_set_schedule(self._h, _iarr(sched)))

    def set_lattice(self, v=None, k=None):
        """Optical lattice sum_j v[j] sin^2(k[j] x_j) added to the trap (fse_set_lattice); None removes it."""
        if v is None:
            _check(lib().fse_set_lattice(self._h, None, None))
            self._lattice = None
        else:
            _check_axes(self.d, v=v, k=k)
            _check(lib().fse_set_lattice(self._h, _darr(v), _darr(k)))
            self._lattice = ([float(a) for a in v], [float(a) for a in k])

    def set_potential(self, U=None):
        """Grid potential U(x~) added to the step's phase and the energy (fse_set_potential);
        the plan holds a reference to the tensor.  None clears it."""
        if U is not None:
            self._check_real(U, "U")
        _check(lib().fse_set_potential(self._h, None if U is None else _ptr(U)))
        self._U = U

    def step_adjoint(self, psi0, nsteps: int, dt: float, grad, grad_U=None, stream=None):
        """Reverse of nsteps steps from psi0 at the plan's time (fse_step_adjoint): grad is
        dL/dpsi at the end on entry and dL/dpsi0 on exit; grad_U, if given, gains dL/dU."""
        self._check_psi(psi0)
        self._check_psi(grad)
        if grad_U is not None:
            self._check_real(grad_U, "grad_U")
        _check(lib().fse_step_adjoint(self._h, _ptr(psi0), int(nsteps), float(dt), _ptr(grad),
                                      None if grad_U is None else _ptr(grad_U), _stream(stream)))
        return grad

    def apply_Lz(self, psi, out=None, stream=None):
        """Lz psi = -i (x d_y - y d_x) psi (fse_apply_Lz)."""
        import torch
        self._check_psi(psi)
        out = torch.empty_like(psi) if out is None else out
        self._check_psi(out)
        _check(lib().fse_apply_Lz(self._h, _ptr(psi), _ptr(out), _stream(stream)))
        return out

    def angular_momentum_grad(self, psi, g=None, out=None, stream=None):
        """2 h^d g Lz psi, the gradient of g <Lz> (fse_angular_momentum_grad); g: a float64 device scalar
        tensor (None: 1)."""
        import torch
        self._check_psi(psi)
        out = torch.empty_like(psi) if out is None else out
        self._check_psi(out)
        gp = None
        if g is not None:
            if g.dtype != torch.float64 or not g.is_cuda or g.numel() != 1:
                raise ValueError("g must be a float64 device tensor with one element")
            g = g.contiguous()
            gp = _ptr(g)
        _check(lib().fse_angular_momentum_grad(self._h, _ptr(psi), gp, _ptr(out), _stream(stream)))
        return out

    @property
    def time(self) -> float:
        t = ctypes.c_double()
        _check(lib().fse_get_time(self._h, ctypes.byref(t)))
        return t.value

    @time.setter
    def time(self, t: float):
        _check(lib().fse_set_time(self._h, float(t)))

    def set_mass_renorm(self, enable: bool):
        """FP64 mass renormalisation of each step call (fse_set_mass_renorm; default on for complex64)."""
        _check(lib().fse_set_mass_renorm(self._h, 1 if enable else 0))

    def mass_renorm(self):
        """(enabled, last factor, mass before the exit pass, mass at the call's start) (fse_get_mass_renorm)."""
        e = ctypes.c_int()
        r = (ctypes.c_double * 3)()
        _check(lib().fse_get_mass_renorm(self._h, ctypes.byref(e), r))
        return bool(e.value), float(r[0]), float(r[1]), float(r[2])

    def set_guard(self, tol: float = 0.0):
        """Numeric guard (fse_set_guard): with tol > 0 every step call ends with a device-side mass check
        against the mass at the first guarded call; a later step call raises FseError (FSE_ERR_NUMERIC)
        once a check has failed.  Resets the reference mass and the flag; tol <= 0 turns it off."""
        _check(lib().fse_set_guard(self._h, float(tol)))

    def guard_status(self):
        """(tripped, reference mass, mass at the last completed check), waiting for the last check."""
        t = ctypes.c_int()
        m = (ctypes.c_double * 2)()
        _check(lib().fse_guard_status(self._h, ctypes.byref(t), m))
        return bool(t.value), float(m[0]), float(m[1])

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().fse_workspace_size(self._h, ctypes.byref(b)))
        return b.value

    def scratch_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().fse_scratch_size(self._h, ctypes.byref(b)))
        return b.value

    def set_workspace(self, buf=None):
        """Take the step's scratch from a device tensor of at least scratch_bytes() bytes
        (fse_set_workspace); the plan holds a reference to it.  None returns to plan-owned scratch."""
        if buf is None:
            _check(lib().fse_set_workspace(self._h, None, 0))
        else:
            if not buf.is_cuda or not buf.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            _check(lib().fse_set_workspace(self._h, _ptr(buf), buf.numel() * buf.element_size()))
        self._ws = buf

    def step(self, psi, nsteps: int, dt: float, stream=None, order: int = 2):
        """nsteps steps in place: TS2-GauSum (order 2, fse_step) or its fourth-order
        triple-jump composition (order 4, fse_step4)."""
        self._check_psi(psi)
        if order not in (2, 4):
            raise ValueError("order must be 2 or 4")
        fn = lib().fse_step if order == 2 else lib().fse_step4
        _check(fn(self._h, _ptr(psi), int(nsteps), float(dt), _stream(stream)))
        return psi

    def apply_H(self, psi, out=None, rho_frozen=None, stream=None):
        import torch
        self._check_psi(psi)
        out = torch.empty_like(psi) if out is None else out
        self._check_psi(out)
        rp = None
        if rho_frozen is not None:
            self._check_real(rho_frozen, "rho_frozen")
            rp = _ptr(rho_frozen)
        _check(lib().fse_apply_H(self._h, _ptr(psi), _ptr(out), rp, _stream(stream)))
        return out

    def nonlocal_potential(self, psi, out=None, stream=None):
        import torch
        self._check_psi(psi)
        out = torch.empty(self.N, dtype=self.rdtype, device=psi.device) if out is None else out
        self._check_real(out, "out")
        _check(lib().fse_nonlocal_potential(self._h, _ptr(psi), _ptr(out), _stream(stream)))
        return out

    def _scalar(self, fn, psi, n, stream):
        import torch
        self._check_psi(psi)
        out = torch.empty(n, dtype=torch.float64, device=psi.device)
        _check(fn(self._h, _ptr(psi), _ptr(out), _stream(stream)))
        return out

    def mass(self, psi, stream=None):
        return self._scalar(lib().fse_mass, psi, 1, stream)

    def mass_noalloc(self, psi, out, stream=None):
        """fse_mass_noalloc into the caller's float64 device tensor `out` (at least one element): the
        library allocates nothing for this call."""
        import torch
        self._check_psi(psi)
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 1 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor with at least one element")
        _check(lib().fse_mass_noalloc(self._h, _ptr(psi), _ptr(out), _stream(stream)))
        return out

    def energy(self, psi, stream=None):
        """Device tensor [E_kin, E_pot, E_int, E_non, E_rot, E_total]."""
        return self._scalar(lib().fse_energy, psi, 6, stream)

    def angular_momentum(self, psi, stream=None):
        return self._scalar(lib().fse_angular_momentum, psi, 1, stream)

    def moments(self, psi, stream=None):
        """Device tensor [N, x_c, y_c, z_c, delta_x, delta_y, delta_z], lab frame at the plan's time
        (fse_moments)."""
        return self._scalar(lib().fse_moments, psi, 7, stream)

    def gs_step(self, psi, dt: float, tol: float = 1e-12, maxit: int = 1000, stream=None) -> dict:
        """One backward-Euler gradient-flow step toward the ground state, in place on psi
        (fse_gs_step); returns the solver statistics."""
        self._check_psi(psi)
        st = GsStats()
        _check(lib().fse_gs_step(self._h, _ptr(psi), float(dt), float(tol), int(maxit), ctypes.byref(st),
                                 _stream(stream)))
        return {"iterations": st.iterations, "converged": bool(st.converged), "residual": st.residual,
                "diff_inf": st.diff_inf}

    def gs_run(self, psi, dt: float, eps_diff: float = 0.0, eps_energy: float = 0.0, max_steps: int = 1000,
               tol: float = 1e-12, maxit: int = 1000, trace: bool = True, stream=None) -> dict:
        """Ground-state steps until ||psi^n - psi^{n+1}||_inf <= eps_diff dt or |E^{n+1} - E^n| <= eps_energy
        (fse_gs_run; a tolerance <= 0 disables its rule), in place on psi; returns the statistics and, with
        trace, the energies E(psi^0), ..., E(psi^steps)."""
        self._check_psi(psi)
        st = GsRunStats()
        buf = (ctypes.c_double * (int(max_steps) + 1))() if trace else None
        _check(lib().fse_gs_run(self._h, _ptr(psi), float(dt), float(tol), int(maxit), int(max_steps),
                                float(eps_diff), float(eps_energy), buf, ctypes.byref(st), _stream(stream)))
        out = {k: getattr(st, k) for k, _ in GsRunStats._fields_}
        out["converged"] = bool(out["converged"])
        if trace:
            out["energies"] = [float(buf[k]) for k in range(st.steps + 1)]
        return out

    def set_profiling(self, enable: bool):
        _check(lib().fse_set_profiling(self._h, 1 if enable else 0))

    def profile(self):
        """{pass name: (total ms, launches)} accumulated since profiling was enabled."""
        n = len(PASS_NAMES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(lib().fse_get_profile(self._h, ms, cnt, n))
        return {PASS_NAMES[k]: (ms[k], cnt[k]) for k in range(n) if cnt[k] > 0}

    def symbol(self) -> np.ndarray:
        shape = tuple(n + 1 for n in self.N)
        out = np.zeros(int(np.prod(shape)), dtype=np.float64)
        _check(lib().fse_get_symbol(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(shape)


class Batch:
    """Batched sweep over 2D instances (wraps fse_batch); states in one packed tensor."""

    def __init__(self, params, precision: int = C64, stream=None):
        import torch
        self.params = list(params)
        self.count = len(self.params)
        self.precision = precision
        self.cdtype = torch.complex128 if precision == C128 else torch.complex64
        arr = (Instance * self.count)()
        for k, p in enumerate(self.params):
            if p.d != 2:
                raise ValueError("batched instances are 2D")
            q = arr[k]
            q.N = (ctypes.c_int * 2)(*p.N)
            q.L = (ctypes.c_double * 2)(*p.L)
            q.s, q.Omega, q.beta, q.lam, q.dt, q.m = p.s, p.Omega, p.beta, p.lam, p.dt, p.m
            q.gamma = (ctypes.c_double * 2)(*p.gamma)
            q.kernel = (make_kernel(p.kernel, mu=p.mu, prefactor=p.c, axis=p.axis) if p.kernel != "none"
                        else make_kernel("none"))
        self._h = ctypes.c_void_p()
        _check(lib().fse_batch_create(ctypes.byref(self._h), self.count, arr, precision, _stream(stream)))
        off = (ctypes.c_size_t * (self.count + 1))()
        _check(lib().fse_batch_offsets(self._h, off))
        self.offsets = [int(x) for x in off]

    def close(self):
        if self._h:
            _check(lib().fse_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, states):
        """Packed device tensor from a list of numpy arrays (one per instance)."""
        import torch
        flat = np.concatenate([np.asarray(s).ravel() for s in states])
        if flat.size != self.offsets[-1]:
            raise ValueError("state sizes do not match the batch")
        np_dtype = np.complex128 if self.precision == C128 else np.complex64
        return torch.from_numpy(flat.astype(np_dtype)).to("cuda")

    def unpack(self, packed):
        h = packed.detach().cpu().numpy()
        return [h[self.offsets[k]:self.offsets[k + 1]].reshape(self.params[k].N) for k in range(self.count)]

    def _check_packed(self, packed):
        if (packed.dtype != self.cdtype or packed.numel() != self.offsets[-1] or not packed.is_contiguous()
                or not packed.is_cuda):
            raise ValueError("packed state must be a contiguous device tensor of the batch's dtype and size")

    def step(self, packed, nsteps: int, stream=None):
        self._check_packed(packed)
        _check(lib().fse_batch_step(self._h, _ptr(packed), int(nsteps), _stream(stream)))
        return packed

    def reduce(self, packed, stream=None):
        """Device tensor (count, 7): mass, E_kin, E_pot, E_int, E_non, E_rot, E_total."""
        import torch
        self._check_packed(packed)
        out = torch.empty(self.count * 7, dtype=torch.float64, device=packed.device)
        _check(lib().fse_batch_reduce(self._h, _ptr(packed), _ptr(out), _stream(stream)))
        return out.view(self.count, 7)

    def times(self):
        t = (ctypes.c_double * self.count)()
        _check(lib().fse_batch_times(self._h, t))
        return list(t)

    def set_mass_renorm(self, enable: bool):
        """FP64 mass renormalisation of every instance per step call (fse_batch_set_mass_renorm; default on for
        complex64)."""
        _check(lib().fse_batch_set_mass_renorm(self._h, 1 if enable else 0))

    def mass_renorm(self):
        """(enabled, array (count, 3): per instance the last factor, the mass before the exit pass and the mass at
        the call's start) (fse_batch_get_mass_renorm)."""
        import numpy as np
        e = ctypes.c_int()
        r = (ctypes.c_double * (3 * self.count))()
        _check(lib().fse_batch_get_mass_renorm(self._h, ctypes.byref(e), r))
        return bool(e.value), np.array(r[:], dtype=np.float64).reshape(self.count, 3)
