"""CPU tests of libfse.so: it loads, exports every declared entry point, its
host-side validation returns the documented codes, and its host FP64 GauSum
multiplier agrees with the oracle's (independent implementations)."""
import math
import os
import re

import numpy as np
import pytest

from paper_1512_03210_amd import fse
from oracle import gausum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "fse.h")).read()
    return sorted(set(re.findall(r"^\s*(?:fse_status|const char\*)\s+(fse_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = fse.lib()
    declared = _declared_symbols()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(fse.EXPORTS) == declared
    assert "gfx950" in fse.version()


@pytest.mark.parametrize("args,code", [
    (dict(d=4), -1),
    (dict(N=(64, 62)), -1),           # 62 = 2 * 31
    (dict(N=(64, 8)), -1),            # below the minimum size
    (dict(N=(64, 1024)), -1),         # above the maximum size
    (dict(L=(8.0, -1.0)), -1),
    (dict(s=0.0), -1),
    (dict(s=float("nan")), -1),
    (dict(beta=float("inf")), -1),
    (dict(kernel=fse.make_kernel("coulomb", mu=1.5)), -1),   # mu > d - 1 in 2D
    (dict(kernel=fse.make_kernel("ddi3")), -1),               # dipole needs d = 3
    (dict(precision=7), -1),
    (dict(), 0),
    (dict(N=(96, 48)), 0),
])
def test_plan_check_codes(args, code):
    a = dict(d=2, N=(64, 64), L=(8.0, 8.0), s=0.75, Omega=0.5, gamma=(1.0, 1.0), beta=100.0, lam=1.0,
             kernel=fse.make_kernel("coulomb", prefactor=1 / (2 * math.pi)), precision=fse.C128)
    a.update(args)
    st = fse.plan_check(a["d"], a["N"], a["L"], a["s"], a["Omega"], a["gamma"] + (1.0,) * 2, a["beta"], a["lam"],
                        a["kernel"], a["precision"])
    assert st == code, fse.lib().fse_last_error()


def test_plan_check_3d_and_unsupported_axis():
    k = fse.make_kernel("ddi3", axis=(0.0, 0.0, 1.0))
    assert fse.plan_check(3, (32, 32, 32), (6.0,) * 3, 0.8, 0.7, (1, 1, 2), 200, 50, k) == 0
    k2 = fse.make_kernel("ddi3", axis=(1.0, 0.0, 0.0))  # turns in the rotating frame: quadratic form
    assert fse.plan_check(3, (32, 32, 32), (6.0,) * 3, 0.8, 0.7, (1, 1, 2), 200, 50, k2) == 0
    assert fse.plan_check(3, (512, 32, 32), (6.0,) * 3, 0.8, 0.7, (1, 1, 2), 200, 50, k) == -1


def test_plan_check_dipole_axes():
    # any unit axis; tilted or turning axes need the one-pass convolution
    ok3 = [((1.0, 0.0, 0.0), 0.0), ((0.0, 1.0, 0.0), 0.0), ((0.0, 0.0, -1.0), 0.7)]
    for axis, Om in ok3:
        k = fse.make_kernel("ddi3", axis=axis)
        assert fse.plan_check(3, (32, 32, 32), (6.0,) * 3, 0.8, Om, (1, 1, 2), 200, 50, k) == 0, axis
    k = fse.make_kernel("ddi3", axis=(0.6, 0.8, 0.0))  # tilted: quadratic form
    assert fse.plan_check(3, (32, 32, 32), (6.0,) * 3, 0.8, 0.0, (1, 1, 2), 200, 50, k) == 0
    with pytest.raises(fse.FseError):  # no even table for a tilted axis
        fse.gausum_symbol_host(3, (32, 32, 32), (6.0,) * 3, k)
    ok2 = [((0.0, 0.0, 1.0), 0.5), ((0.6, 0.0, 0.8), 0.0), ((0.0, 1.0, 0.0), 0.0), ((1.0, 0.0, 0.0), 0.0)]
    for axis, Om in ok2:
        k = fse.make_kernel("ddi2", axis=axis)
        assert fse.plan_check(2, (64, 48), (8.0, 6.0), 0.8, Om, (1, 1), 20, 5, k) == 0, axis
    cases2 = [((0.36, 0.48, 0.8), 0.0, 0), ((0.6, 0.0, 0.8), 0.5, 0), ((0.6, 0.0, 0.0), 0.0, -1),
              ((float("nan"), 0.0, 1.0), 0.0, -1)]
    for axis, Om, want in cases2:
        k = fse.make_kernel("ddi2", axis=axis)
        assert fse.plan_check(2, (64, 48), (8.0, 6.0), 0.8, Om, (1, 1), 20, 5, k) == want, axis
    # the quadratic form runs in the one-pass padded convolution: contiguous axis <= 256
    k = fse.make_kernel("ddi2", axis=(0.6, 0.0, 0.8))
    assert fse.plan_check(2, (64, 384), (8.0, 8.0), 0.8, 0.5, (1, 1), 20, 5, k) == -2
    assert fse.plan_check(2, (64, 384), (8.0, 8.0), 0.8, 0.0, (1, 1), 20, 5, k) == 0  # fixed, even: stored whole
    k = fse.make_kernel("ddi2")
    assert fse.plan_check(3, (32, 32, 32), (6.0,) * 3, 0.8, 0.0, (1, 1, 2), 200, 50, k) == -1
    k = fse.make_kernel("ddi3")
    assert fse.plan_check(2, (64, 48), (8.0, 6.0), 0.8, 0.0, (1, 1), 20, 5, k) == -1


@pytest.mark.parametrize("d,N,L,kind,c", [
    (2, (64, 64), (8.0, 8.0), "coulomb", 1 / (2 * math.pi)),
    (2, (48, 96), (6.0, 9.0), "coulomb", 1.0),
    (3, (32, 24, 16), (6.0, 5.0, 4.0), "coulomb", 1 / (4 * math.pi)),
    (2, (32, 32), (4.0, 4.0), "coulomb-mu0.5", 1.0),
])
def test_host_coulomb_symbol_matches_oracle(d, N, L, kind, c):
    mu = 0.5 if kind.endswith("0.5") else 1.0
    K = fse.gausum_symbol_host(d, N, L, fse.make_kernel("coulomb", mu=mu, prefactor=c))
    Ko = gausum.coulomb_symbol(N, L, mu=mu, c=c)[tuple(slice(0, n + 1) for n in N)]
    assert np.max(np.abs(K - Ko)) < 1e-14 * np.max(np.abs(Ko))


def test_host_ddi3_symbol_matches_oracle():
    N, L = (32, 32, 24), (6.0, 6.0, 5.0)
    K = fse.gausum_symbol_host(3, N, L, fse.make_kernel("ddi3"))
    Ko = gausum.ddi3_symbol(N, L)[tuple(slice(0, n + 1) for n in N)]
    # the dipole multiplier is -1 + 3 kz^2 Khat_C: round-off of Khat_C is
    # amplified by 3 kz^2, so compare on that scale
    KC = gausum.coulomb_symbol(N, L, mu=1.0, c=1 / (4 * math.pi))
    kz = math.pi * np.arange(N[2] + 1) / (2 * L[2])
    scale = 1.0 + 3.0 * kz[None, None, :] ** 2 * np.max(np.abs(KC))
    assert np.max(np.abs(K - Ko) / scale) < 1e-14
    assert abs(K[0, 0, 0] + 1.0) < 1e-15  # kappa = 0: -1


@pytest.mark.parametrize("ax", [0, 1])
def test_host_ddi3_symbol_other_axes(ax):
    N, L = (24, 32, 16), (5.0, 6.0, 4.0)
    axis = tuple(1.0 if j == ax else 0.0 for j in range(3))
    K = fse.gausum_symbol_host(3, N, L, fse.make_kernel("ddi3", axis=axis))
    Ko = gausum.ddi3_symbol(N, L, axis=axis)[tuple(slice(0, n + 1) for n in N)]
    KC = gausum.coulomb_symbol(N, L, mu=1.0, c=1 / (4 * math.pi))
    k = math.pi * np.arange(N[ax] + 1) / (2 * L[ax])
    shape = [1, 1, 1]
    shape[ax] = -1
    scale = 1.0 + 3.0 * k.reshape(shape) ** 2 * np.max(np.abs(KC))
    assert np.max(np.abs(K - Ko) / scale) < 1e-14


@pytest.mark.parametrize("axis", [(0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.6, 0.0, 0.8),
                                  (0.0, -0.8, 0.6)])
def test_host_ddi2_symbol_matches_oracle(axis):
    N, L = (48, 64), (6.0, 8.0)
    K = fse.gausum_symbol_host(2, N, L, fse.make_kernel("ddi2", axis=axis))
    Ko = gausum.ddi2_symbol(N, L, axis=axis)[tuple(slice(0, n + 1) for n in N)]
    KC = gausum.coulomb_symbol(N, L, mu=1.0, c=1 / (2 * math.pi))
    k0 = math.pi * np.arange(N[0] + 1) / (2 * L[0])
    k1 = math.pi * np.arange(N[1] + 1) / (2 * L[1])
    scale = 1.0 + 1.5 * (k0[:, None] ** 2 + k1[None, :] ** 2) * np.max(np.abs(KC))
    assert np.max(np.abs(K - Ko) / scale) < 1e-14
    assert K[0, 0] == 0.0  # kappa = 0: no mean-field term in 2D


def test_gpu_entry_points_fail_cleanly_without_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = fse.ctypes.c_void_p()
    st = fse.lib().fse_plan_create(fse.ctypes.byref(h), 2, fse._iarr((64, 64)), fse._darr((8.0, 8.0)), 0.75, 0.5,
                                   fse._darr((1.0, 1.0)), 1.0, 1.0, None, 0, 0.0, None)
    assert st == -4 and not h.value


def _declarations():
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "fse.h")).read(), flags=re.S)
    for m in re.finditer(r"^\s*fse_status\s+(fse_\w+)\s*\(([^)]*)\)\s*;", text, re.M):
        yield m.group(1), [a.strip() for a in m.group(2).split(",")]


def test_null_handles_are_rejected_on_the_host():
    # every entry point that takes a plan or batch handle (or returns one): NULL and zero arguments give
    # FSE_ERR_ARG with a message, without a device; destroying NULL is a no-op
    lib, seen = fse.ctypes.CDLL(fse.lib()._name), 0  # a private wrapper: the binding's argtypes stay as they are
    for name, args in _declarations():
        if not args[0].startswith(("fse_plan", "fse_batch")):
            continue
        vals, types = [], []
        for a in args:
            if "*" in a or a.startswith(("fse_plan", "fse_batch")):
                vals.append(None), types.append(fse.ctypes.c_void_p)
            elif a.startswith("double"):
                vals.append(0.0), types.append(fse.ctypes.c_double)
            elif a.startswith("size_t"):
                vals.append(0), types.append(fse.ctypes.c_size_t)
            else:
                assert a.startswith("int "), (name, a)
                vals.append(0), types.append(fse.ctypes.c_int)
        f = getattr(lib, name)
        f.argtypes, f.restype = types, fse.ctypes.c_int
        st = f(*vals)
        if name.endswith("_destroy"):
            assert st == 0, name
        else:
            assert st == -1, (name, st)
            assert fse.lib().fse_last_error(), name
        seen += 1
    assert seen >= 40


def test_per_axis_arrays_shorter_than_d_are_refused_before_the_library():
    # the library reads d values from N, L and gamma (and from the lattice's v and k): the binding refuses shorter
    # sequences, which would make it read past the end of a host array
    k = fse.make_kernel("coulomb", prefactor=1 / (2 * math.pi))
    for args in (((32, 32), (6.0,) * 3, (1.0,) * 3), ((32,) * 3, (6.0,) * 2, (1.0,) * 3), ((32,) * 3, (6.0,) * 3, (1.0,) * 2)):
        with pytest.raises(ValueError):
            fse.plan_check(3, args[0], args[1], 0.8, 0.5, args[2], 10.0, 1.0, k)
        with pytest.raises(ValueError):
            fse.Plan(3, args[0], args[1], 0.8, 0.5, args[2], 10.0, 1.0, k)
    with pytest.raises(ValueError):
        fse.gausum_symbol_host(3, (32, 32), (6.0,) * 3, k)
    p = fse.Plan.__new__(fse.Plan)
    p.d, p._h = 3, None
    with pytest.raises(ValueError):
        p.set_lattice(v=(1.0, 1.0), k=(1.0, 1.0, 1.0))
    with pytest.raises(ValueError):
        p.set_lattice(v=(1.0, 1.0, 1.0), k=(1.0,))
    assert fse.plan_check(4, (32,) * 4, (6.0,) * 4, 0.8, 0.5, (1.0,) * 4, 10.0, 1.0, k) == -1  # the library's own check
