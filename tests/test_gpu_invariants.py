"""Degenerate cases in which the method's result is fixed exactly, on the GPU.

A uniform state is a fixed point of every flux and limiter: every face sees
the same left and right state, so every flux difference is exactly zero and
both Runge-Kutta stages return the state bit for bit.  A stationary contact
(fluid at rest, uniform pressure, any density) is a fixed point of HLLC,
which resolves contacts exactly (Sec. 4.2.1): Batten's middle speed is
exactly zero, so the mass and energy fluxes vanish and the momentum flux is
the uniform pressure.  Both hold whatever limiter forms the density slopes,
the learned one included (the pressure and velocity stencils are flat, and a
flat stencil has slope zero)."""
import numpy as np
import pytest

from paper_1207_3392_amd import workloads as wl

pytestmark = pytest.mark.gpu
hydro = pytest.importorskip("paper_1207_3392_amd.hydro")


def _gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


if not _gpu():
    pytest.skip("no GPU", allow_module_level=True)

SHAPES = {1: (70,), 2: (70, 19), 3: (67, 11, 13)}


def _problem(ndim, W, bc):
    n = SHAPES[ndim] + (1,) * (3 - ndim)
    dx = 1.0 / n[0]
    hi = tuple(n[q] * dx if q < ndim else 1.0 for q in range(3))
    bcs = tuple((bc, bc) if q < ndim else (wl.BC_PERIODIC, wl.BC_PERIODIC) for q in range(3))
    return wl.Problem(ndim, n, (0.0, 0.0, 0.0), hi, 1.4, bcs, W.reshape((ndim + 2,) + n[::-1]), theta=2.0)


def _cases(ndim):
    solvers = [hydro.HLL, hydro.HLLC] + ([hydro.HLLC_SWITCH] if ndim > 1 else [])
    out = [(s, prec, hydro.LIM_THETA) for s in solvers for prec in (32, 64)]
    return out + [(hydro.HLLC, 32, hydro.LIM_LEARNED)]


def _patch(prob, prec, lim):
    from paper_1207_3392_amd import limiter

    p = hydro.Patch(prob, precision=prec, limiter=lim)
    if lim == hydro.LIM_LEARNED:
        p.set_mlp(limiter.trained_params())
    return p


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW])
def test_uniform_state_is_a_fixed_point(ndim, bc):
    """A uniform moving state under periodic or outflow boundaries stays the
    same bit for bit through ten steps with the device's CFL step, for every
    solver, both precisions and the learned limiter."""
    ncell = int(np.prod(SHAPES[ndim]))
    W0 = np.array([1.3, 0.3, -0.2, 0.1][: 1 + ndim] + [0.9])
    W = np.repeat(W0[:, None], ncell, axis=1)
    prob = _problem(ndim, W, bc)
    for solver, prec, lim in _cases(ndim):
        p = _patch(prob, prec, lim)
        U0 = p.get_state(hydro.CONSERVED)
        assert np.all(U0 == U0[:, :1])
        p.advance(10, 0.4, solver=solver)
        U = p.get_state(hydro.CONSERVED)
        assert p.time() > 0
        p.close()
        assert np.array_equal(U, U0), (solver, prec, lim)


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT])
def test_stationary_contact_is_a_fixed_point_of_hllc(ndim, bc):
    """Fluid at rest at uniform pressure with a random density field (jumps
    between neighbouring cells of up to a factor 4) stays the same bit for
    bit through ten HLLC steps, with the switch, in both precisions and with
    the learned limiter, under every boundary kind (a reflecting wall mirrors
    a zero velocity)."""
    ncell = int(np.prod(SHAPES[ndim]))
    rng = np.random.default_rng(40 + 10 * ndim + bc)
    W = np.zeros((ndim + 2, ncell))
    W[0] = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=ncell))
    W[-1] = 0.7
    prob = _problem(ndim, W, bc)
    cases = [(s, prec, lim) for s, prec, lim in _cases(ndim) if s != hydro.HLL]
    for solver, prec, lim in cases:
        p = _patch(prob, prec, lim)
        U0 = p.get_state(hydro.CONSERVED)
        assert np.all(U0[1:-1] == 0.0)
        p.advance(10, 0.4, solver=solver)
        U = p.get_state(hydro.CONSERVED)
        p.close()
        assert np.array_equal(U, U0), (solver, prec, lim, np.max(np.abs(U - U0), axis=1))


def test_uniform_tubes_in_the_batch_are_fixed_points():
    """Uniform tubes of several sizes in one batched launch, HLL and HLLC
    (outflow and periodic ends): every tube is unchanged bit for bit at
    t_end."""
    probs = []
    for k, n in enumerate((2, 5, 130, 1000, 4096)):
        W = np.repeat(np.array([[0.8 + 0.1 * k], [0.5 - 0.2 * k], [1.0 + 0.3 * k]]), n, axis=1)
        pr = wl.riemann_tube(n, tuple(W[:, 0]), tuple(W[:, 0]), 0.5, 1.4, theta=2.0, cfl=0.4, t_end=0.01)
        if k % 2:
            pr.bc = ((wl.BC_PERIODIC, wl.BC_PERIODIC), (0, 0), (0, 0))
        probs.append(pr)
    for solver in (hydro.HLL, hydro.HLLC):
        B = hydro.Batch(probs)
        U0 = [B.get_state(i, hydro.CONSERVED) for i in range(len(probs))]
        B.run_to(0.01, 0.4, solver)
        for i in range(len(probs)):
            steps, t = B.status(i)
            assert steps > 0 and t == pytest.approx(0.01, rel=1e-12)
            assert np.array_equal(B.get_state(i, hydro.CONSERVED), U0[i]), (solver, i)
        B.close()
