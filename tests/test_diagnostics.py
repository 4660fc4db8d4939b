"""Kinetic-energy diagnostics (Sec. 4.3.1): the oracle's E_kin per component
against closed forms, and the spectrum's normalisation (Parseval) and shell
placement."""
import math

import numpy as np

import oracle
from paper_1207_3392_amd import diagnostics as dg
from paper_1207_3392_amd import workloads as wl


def _prob(W, n, box=1.0):
    nd = W.shape[0] - 2
    ns = (n,) * nd + (1,) * (3 - nd)
    hi = (box,) * nd + (1.0,) * (3 - nd)
    return wl.Problem(nd, ns, (0, 0, 0), hi, 1.4, ((0, 0),) * 3, W)


def test_kinetic_energy_closed_forms():
    n = 64
    W = np.zeros((4, n, n))
    W[0], W[1], W[2], W[3] = 2.0, 0.3, -0.4, 1.0
    d = oracle.Desc.from_problem(_prob(W, n))
    E = oracle.kinetic_energy(d, oracle.prim_to_cons(d, W.reshape(4, -1)))
    assert np.allclose(E, [0.5 * 2.0 * 0.09, 0.5 * 2.0 * 0.16, 0.0], rtol=1e-14)
    # v_y = A sin(2 pi 3 x): the mean of sin^2 over whole periods at cell centres is 1/2
    x = (np.arange(n) + 0.5) / n
    W[1] = 0.0
    W[2] = 0.25 * np.sin(2 * np.pi * 3 * x)[None, :]
    E = oracle.kinetic_energy(d, oracle.prim_to_cons(d, W.reshape(4, -1)))
    assert math.isclose(E[1], 0.5 * 2.0 * 0.25 ** 2 * 0.5, rel_tol=1e-13) and E[0] == 0.0


def test_spectrum_parseval_and_single_mode():
    n = 32
    rng = np.random.default_rng(3)
    for nd in (2, 3):
        shape = (n,) * nd
        W = np.empty((nd + 2,) + shape)
        W[0] = 1.0 + 0.5 * rng.random(shape)
        for q in range(nd):
            W[1 + q] = rng.normal(size=shape)
        W[-1] = 1.0
        box = 0.7
        d = oracle.Desc.from_problem(_prob(W, n, box))
        E = oracle.kinetic_energy(d, oracle.prim_to_cons(d, W.reshape(nd + 2, -1))).sum()
        k, e = dg.kinetic_spectrum(W, box)
        assert math.isclose(np.sum(e) * (k[1] - k[0]), E, rel_tol=1e-12)
    # one Fourier mode of wavevector (0, 5): all energy on shell 5
    W = np.zeros((4, n, n))
    y = (np.arange(n) + 0.5) / n
    W[0] = 1.0
    W[1] = 0.2 * np.cos(2 * np.pi * 5 * y)[:, None]
    W[3] = 1.0
    k, e = dg.kinetic_spectrum(W, 1.0)
    dk = k[1] - k[0]
    assert math.isclose(e[5] * dk, 0.5 * 0.2 ** 2 * 0.5, rel_tol=1e-12)
    assert np.sum(np.abs(np.delete(e, 5))) < 1e-12 * e[5]
    assert dg.spectral_cutoff(k, e, 1e-9) == k[5]
