"""FP64 reference of the kinetic-energy spectrum of the Kelvin-Helmholtz
analysis (Sec. 4.3.1).

TEST INFRASTRUCTURE ONLY (the oracle): the tests compare the GPU library's
spectrum with this one; the library never calls it.

The spectrum is the plain definition: the discrete Fourier coefficients of
each component of sqrt(rho) v on the periodic box of side L (numpy's FFT is
the transform step, divided by the cell count so that the coefficients are
mean-normalised), their squared magnitudes summed over components, and
binned on shells of |k| = 2 pi s / L of width dk = 2 pi / L, s the integer
nearest to |n| for the integer wavevector n of the coefficient (numpy's FFT
frequency order: n = i for i < N/2, i - N otherwise).  The normalisation
makes sum_s e(s) dk the box integral of rho |v|^2 / 2 (Parseval).
"""
from __future__ import annotations

import math

import numpy as np


def shell_index(nvec_sq: np.ndarray) -> np.ndarray:
    """Shell of an integer wavevector from its squared length: the nearest
    integer to its length (no ties: a length is never a half-integer)."""
    return np.floor(np.sqrt(nvec_sq.astype(np.float64)) + 0.5).astype(np.int64)


def kinetic_spectrum(W: np.ndarray, box: float):
    """W: primitives (nv, [nz,] ny, nx) with the same cell count along every
    active axis, on a periodic cube of side ``box``.  Returns (k, e): the
    shell wavenumbers 2 pi s / box, s = 0, 1, ..., and e_kin on each."""
    nd = W.shape[0] - 2
    shape = W.shape[1:]
    n = shape[-1]
    assert all(s == n for s in shape), "the spectrum needs the same cell count along every axis"
    sq = np.sqrt(W[0])
    power = np.zeros(shape)
    for q in range(nd):
        F = np.fft.fftn(sq * W[1 + q]) / W[0].size
        power += np.abs(F) ** 2
    freqs = np.fft.fftfreq(n, d=1.0 / n)  # integer frequencies in FFT order
    grids = np.meshgrid(*([freqs] * nd), indexing="ij")
    nsq = sum(g.astype(np.int64) ** 2 for g in grids)
    shell = shell_index(nsq)
    dk = 2.0 * math.pi / box
    e = np.bincount(shell.ravel(), weights=0.5 * box ** nd * power.ravel()) / dk
    return dk * np.arange(e.size), e


def spectral_cutoff(k, e, level: float) -> float:
    """The largest shell wavenumber at which e_kin stays above ``level``
    (the paper compares solvers by where their spectra fall below 1e-9)."""
    above = np.nonzero(e > level)[0]
    return float(k[above.max()]) if above.size else 0.0
