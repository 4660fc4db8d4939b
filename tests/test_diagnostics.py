"""Kinetic-energy diagnostics (Sec. 4.3.1): the oracle's E_kin per component
against closed forms, and the oracle's spectrum against its normalisation
(Parseval), single Fourier modes on known shells (Nyquist included) and a
brute-force discrete Fourier sum on a small grid."""
import math

import numpy as np

import oracle
from oracle import spectrum as sp
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
        k, e = sp.kinetic_spectrum(W, box)
        assert math.isclose(np.sum(e) * (k[1] - k[0]), E, rel_tol=1e-12)
    # one Fourier mode of wavevector (0, 5): all energy on shell 5
    W = np.zeros((4, n, n))
    y = (np.arange(n) + 0.5) / n
    W[0] = 1.0
    W[1] = 0.2 * np.cos(2 * np.pi * 5 * y)[:, None]
    W[3] = 1.0
    k, e = sp.kinetic_spectrum(W, 1.0)
    dk = k[1] - k[0]
    assert math.isclose(e[5] * dk, 0.5 * 0.2 ** 2 * 0.5, rel_tol=1e-12)
    assert np.sum(np.abs(np.delete(e, 5))) < 1e-12 * e[5]
    assert sp.spectral_cutoff(k, e, 1e-9) == k[5]


def test_spectrum_modes_on_their_shells():
    """A cosine mode of integer wavevector (a, b) puts its energy on the shell
    nearest to sqrt(a^2 + b^2); the Nyquist mode (N/2 along one axis) on
    shell N/2."""
    n = 16
    y, x = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n, indexing="ij")
    for (a, b), shell in (((3, 4), 5), ((1, 1), 1), ((2, 2), 3), ((5, 5), 7), ((n // 2, 0), n // 2), ((0, 0), 0)):
        W = np.zeros((4, n, n))
        W[0] = 1.0
        amp = 0.3
        W[2] = amp * np.cos(2 * np.pi * (a * x + b * y) + 0.3)  # (the phase keeps the Nyquist mode nonzero)
        W[3] = 1.0
        k, e = sp.kinetic_spectrum(W, 1.0)
        dk = k[1] - k[0]
        total = 0.5 * np.mean(W[2] ** 2)
        assert math.isclose(e[shell] * dk, total, rel_tol=1e-12), (a, b)
        assert np.sum(np.abs(np.delete(e, shell))) * dk < 1e-13 * total, (a, b)
    # the shell of a squared length m is the nearest integer to sqrt(m)
    m = np.arange(0, 2000)
    want = np.array([min(range(0, 50), key=lambda s: abs(s - math.sqrt(v))) for v in m])
    assert np.array_equal(sp.shell_index(m), want)


def test_spectrum_matches_brute_force_fourier_sums():
    """Direct double sums over cells and wavevectors (no FFT), binned by
    explicit nearest-integer shells, on an 8 x 8 random state."""
    n, box = 8, 1.7
    rng = np.random.default_rng(11)
    W = np.empty((4, n, n))
    W[0] = 0.5 + rng.random((n, n))
    W[1] = rng.normal(size=(n, n))
    W[2] = rng.normal(size=(n, n))
    W[3] = 1.0
    nshell = int(math.floor(math.sqrt(2) * n / 2 + 0.5)) + 1
    e = [0.0] * nshell
    for jy in range(n):
        for jx in range(n):
            fy = jy if jy < n // 2 else jy - n
            fx = jx if jx < n // 2 else jx - n
            p = 0.0
            for q in (1, 2):
                acc = 0j
                for y in range(n):
                    for x in range(n):
                        acc += math.sqrt(W[0, y, x]) * W[q, y, x] * complex(
                            math.cos(2 * math.pi * (fx * x + fy * y) / n), -math.sin(2 * math.pi * (fx * x + fy * y) / n))
                p += abs(acc / n ** 2) ** 2
            s = min(range(nshell), key=lambda t: abs(t - math.sqrt(fx * fx + fy * fy)))
            e[s] += 0.5 * box ** 2 * p / (2 * math.pi / box)
    k, eo = sp.kinetic_spectrum(W, box)
    assert eo.size == nshell
    assert np.allclose(eo, e, rtol=1e-12, atol=1e-14 * max(e))
    assert np.allclose(k, 2 * math.pi / box * np.arange(nshell), rtol=1e-15)
