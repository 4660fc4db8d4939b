"""Kinetic-energy diagnostics of the Kelvin-Helmholtz analysis (Sec. 4.3.1).

E_kin,y(t), the integral of rho v_y^2 / 2, comes from the library's FP64
reduction (Patch.kinetic_energy); the spectral distribution e_kin(k) from its
device spectrum (Patch.kinetic_spectrum: the Fourier coefficients of the
components of sqrt(rho) v on the periodic box, binned on shells of
|k| = 2 pi n / L of width 2 pi / L, normalised so that the sum of e_kin(k) dk
over the shells is the integral of rho |v|^2 / 2 over the box).  Both run on
the GPU; this module only names them and post-processes their output.
"""
from __future__ import annotations

import numpy as np


def kinetic_spectrum(patch):
    """(k, e) of a 2D N x N patch's current state (hy_kinetic_spectrum)."""
    return patch.kinetic_spectrum()


def spectral_cutoff(k, e, level: float) -> float:
    """The largest shell wavenumber at which e_kin stays above ``level``
    (the paper compares solvers by where their spectra fall below 1e-9)."""
    above = np.nonzero(np.asarray(e) > level)[0]
    return float(k[above.max()]) if above.size else 0.0
