"""Multi-dimensional DFTs of the oracle: scipy's pocketfft on every host core.

Unnormalised forward transform exp(-2 pi i n k / M) and its inverse with the
1/M factor, the conventions of numpy.fft.fftn / ifftn.  A library primitive,
used as one step of the method; nothing here is specific to it.
"""
from __future__ import annotations

import os

import scipy.fft

WORKERS = os.cpu_count() or 1


def fftn(a):
    return scipy.fft.fftn(a, workers=WORKERS)


def ifftn(a):
    return scipy.fft.ifftn(a, workers=WORKERS)
