"""The device kinetic-energy spectrum (Sec. 4.3.1) against the oracle's.

Both sides start from the same stored state: the patch's conserved state read
back as FP64 gives the oracle's primitives.  The device transform is FP64 and
its shell sums are fixed point at 2^-61 of the total, so every shell must
agree with the oracle to 1e-12 of the total energy (a radix-2 FFT's rounding
is of order log2(N) unit roundoffs of the total; the fixed-point truncation
below 2^-61 of it per term)."""
import math

import numpy as np
import pytest

import oracle
from oracle import spectrum as osp
from paper_1207_3392_amd import workloads as wl

pytestmark = pytest.mark.gpu

hydro = pytest.importorskip("paper_1207_3392_amd.hydro")


def _torch_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


if not _torch_ok():
    pytest.skip("no GPU", allow_module_level=True)


def _oracle_spectrum(p, prob):
    """The oracle's spectrum of the patch's stored state (FP64 primitives
    from the stored conserved values)."""
    U = p.get_state(hydro.CONSERVED)
    ny, nx = prob.n[1], prob.n[0]
    W = np.empty((4, ny, nx))
    W[0] = U[0].reshape(ny, nx)
    W[1] = (U[1] / U[0]).reshape(ny, nx)
    W[2] = (U[2] / U[0]).reshape(ny, nx)
    W[3] = 1.0
    return osp.kinetic_spectrum(W, prob.hi[0] - prob.lo[0])


def _compare(p, prob):
    k, e = p.kinetic_spectrum()
    ko, eo = _oracle_spectrum(p, prob)
    assert e.size == eo.size
    total = float(np.sum(eo))
    assert np.max(np.abs(e - eo)) <= 1e-12 * total, np.max(np.abs(e - eo)) / total
    assert np.allclose(k, ko, rtol=1e-15)
    return k, e, eo


@pytest.mark.parametrize("prec", [32, 64])
def test_spectrum_matches_oracle_random_states(prec):
    """Random periodic states, N = 2 .. 256 (every transform size up to a
    few tiles of the transpose), each shell against the oracle; two calls
    give the same bits; Parseval against the device's E_kin."""
    for n, box in ((2, 1.0), (4, 0.5), (32, 1.0), (64, 2.0), (128, 1.0), (256, 1.0)):
        prob = wl.random_smooth_patch(2, (n, n), seed=100 + n, amp=0.3)
        prob.hi = (prob.lo[0] + box, prob.lo[1] + box, prob.hi[2])
        p = hydro.Patch(prob, precision=prec)
        k, e, eo = _compare(p, prob)
        k2, e2 = p.kinetic_spectrum()
        assert np.array_equal(e, e2)
        ek = p.kinetic_energy()
        assert math.isclose(np.sum(e) * (k[1] - k[0]), ek[0] + ek[1], rel_tol=1e-12), n
        p.close()


def test_spectrum_single_modes_on_their_shells():
    """One Fourier mode of wavevector (a, b) puts all its energy on the shell
    nearest to sqrt(a^2 + b^2), the Nyquist mode on shell N/2."""
    n = 64
    y, x = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n, indexing="ij")
    for (a, b), shell in (((3, 4), 5), ((2, 2), 3), ((0, 7), 7), ((n // 2, 0), n // 2), ((21, 21), 30)):
        W = np.zeros((4, n, n))
        W[0] = 1.0
        W[1] = 0.2 * np.cos(2 * np.pi * (a * x + b * y) + 0.3)
        W[3] = 1.0
        prob = wl.Problem(2, (n, n, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 1.4, ((0, 0),) * 3, W)
        p = hydro.Patch(prob, precision=64)
        k, e = p.kinetic_spectrum()
        dk = k[1] - k[0]
        total = 0.5 * np.mean(W[1] ** 2)
        assert math.isclose(e[shell] * dk, total, rel_tol=1e-12), (a, b)
        assert np.sum(np.delete(e, shell)) * dk < 1e-13 * total, (a, b)
        p.close()


def test_spectrum_kelvin_helmholtz_full_size():
    """The Kelvin-Helmholtz workload at 2048^2 (its initial state and after a
    few steps): every shell against the oracle, and the 1e-9 cutoff the
    paper compares solvers by."""
    prob = wl.kelvin_helmholtz(2048)
    p = hydro.Patch(prob, precision=32)
    for steps in (0, 20):
        if steps:
            p.advance(steps, 0.4, solver=hydro.HLLC)
        k, e, eo = _compare(p, prob)
        assert osp.spectral_cutoff(k, e, 1e-9) == osp.spectral_cutoff(k, eo, 1e-9)
    p.close()


def test_spectrum_largest_transform():
    """N = 8192, the largest transform the device spectrum takes (one row of
    2^13 points in LDS): every shell against the oracle's."""
    prob = wl.random_smooth_patch(2, (8192, 8192), seed=8192, amp=0.3)
    p = hydro.Patch(prob, precision=32)
    _compare(p, prob)
    p.close()


def test_spectrum_rejects_unsupported_patches():
    cases = [wl.random_smooth_patch(2, (48, 48), seed=1),   # not a power of two
             wl.random_smooth_patch(2, (64, 32), seed=2),   # not square
             wl.random_smooth_patch(3, (16, 16, 16), seed=3),
             wl.random_smooth_patch(1, (64,), seed=4)]
    prob = wl.random_smooth_patch(2, (32, 32), seed=5)
    prob.hi = (prob.lo[0] + 1.0, prob.lo[1] + 2.0, prob.hi[2])  # not a square box
    cases.append(prob)
    for prob in cases:
        p = hydro.Patch(prob, precision=32)
        with pytest.raises(hydro.HydroError) as ei:
            p.kinetic_spectrum()
        assert ei.value.status == hydro.HY_EUNSUPPORTED
        p.close()
