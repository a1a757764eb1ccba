"""Multi-dimensional DFTs of the oracle: scipy's pocketfft on the host cores this process may use.

Unnormalised forward transform exp(-2 pi i n k / M) and its inverse with the
1/M factor, the conventions of numpy.fft.fftn / ifftn.  A library primitive,
used as one step of the method; nothing here is specific to it.
"""
from __future__ import annotations

import os

import scipy.fft


def _host_cores():
    """Cores this process may use: OMP_NUM_THREADS if set, else its CPU affinity, else os.cpu_count()."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


WORKERS = _host_cores()


def fftn(a):
    return scipy.fft.fftn(a, workers=WORKERS)


def ifftn(a):
    return scipy.fft.ifftn(a, workers=WORKERS)
