"""Kinetic-energy diagnostics of the Kelvin-Helmholtz analysis (Sec. 4.3.1).

E_kin,y(t), the integral of rho v_y^2 / 2, comes from the library's FP64
reduction (Patch.kinetic_energy).  The spectral distribution e_kin(k) is
post-processing of a state copied to the host: the Fourier coefficients of
the components of sqrt(rho) v on a periodic box, binned on shells of
|k| = 2 pi n / L of width 2 pi / L, normalised so that the sum of e_kin(k) dk
over the shells is the integral of rho |v|^2 / 2 over the box (Parseval).
"""
from __future__ import annotations

import math

import numpy as np


def kinetic_spectrum(W: np.ndarray, box: float):
    """W: primitives (nv, [nz,] ny, nx) on a periodic cube of side ``box``
    with the same number of cells along every active axis.  Returns (k, e):
    shell wavenumbers 2 pi n / box, n = 0, 1, ... and e_kin at each."""
    nd = W.shape[0] - 2
    shape = W.shape[1:]
    n = shape[-1]
    assert all(s == n for s in shape), "the spectrum needs the same cell count along every axis"
    volume = box ** nd
    sq = np.sqrt(W[0])
    power = np.zeros(shape)
    for q in range(nd):
        F = np.fft.fftn(sq * W[1 + q]) / W[0].size  # mean-normalised coefficients
        power += np.abs(F) ** 2
    # integer wavevector magnitudes on the FFT grid
    freqs = np.fft.fftfreq(n, d=1.0 / n)
    grids = np.meshgrid(*([freqs] * nd), indexing="ij")
    kmag = np.sqrt(sum(g ** 2 for g in grids))
    shell = np.floor(kmag + 0.5).astype(np.int64)
    dk = 2.0 * math.pi / box
    e = np.bincount(shell.ravel(), weights=0.5 * volume * power.ravel()) / dk
    k = dk * np.arange(e.size)
    return k, e


def spectral_cutoff(k, e, level: float) -> float:
    """The largest shell wavenumber at which e_kin stays above ``level``
    (the paper compares solvers by where their spectra fall below 1e-9)."""
    above = np.nonzero(e > level)[0]
    return float(k[above.max()]) if above.size else 0.0
