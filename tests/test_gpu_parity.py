"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case starts both sides from the same state: the GPU's initial conserved
state read back as FP64 is what the oracle steps, so a one-step comparison
isolates the kernels' arithmetic.  FP64 kernels must match to 1e-12
(relative to each variable's scale); FP32 kernels to the precision the state
is held in (per element 2e-5 of the variable's scale, on average 2e-6 of it)."""
import math
import types

import numpy as np
import pytest

import oracle
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


def scale(U):
    """Per-variable scale: the variable's maximum; for momentum components at
    least the state's characteristic momentum sqrt(2 max D max G) (~ rho c),
    because their fluxes carry the pressure and their rounding follows it."""
    s = np.max(np.abs(U), axis=1, keepdims=True)
    m = math.sqrt(2.0 * s[0, 0] * s[-1, 0])
    s[1:-1] = np.maximum(s[1:-1], m)
    return np.maximum(s, 1e-300)


def assert_close(gpu, ref, prec, what=""):
    s = scale(ref)
    err = np.abs(gpu - ref) / s
    if prec == 64:
        assert err.max() < 1e-12, (what, err.max())
    else:
        assert err.max() < 2e-5, (what, err.max(axis=1))
        # mean absolute deviation relative to each variable's scale
        mad = np.mean(np.abs(gpu - ref), axis=1) / s[:, 0]
        assert np.all(mad < 2e-6), (what, mad)


def one_step_case(prob, solver, prec, theta=None, nsteps=1, cfl=0.4):
    d = oracle.Desc.from_problem(prob, solver=solver, theta=theta)
    p = hydro.Patch(prob, precision=prec, theta=theta)
    U0 = p.get_state(hydro.CONSERVED)
    U_ref = U0.copy()
    for _ in range(nsteps):
        dt = oracle.cfl_dt(d, U_ref, cfl)
        U_ref = oracle.step(d, U_ref, dt)
        p.step(dt, solver)
    U = p.get_state(hydro.CONSERVED)
    p.close()
    return U, U_ref


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", [oracle.HLL, oracle.HLLC])
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT])
def test_1d_random_patch(prec, solver, bc):
    prob = wl.random_smooth_patch(1, (150,), seed=100 + bc, bc=bc)
    for theta in (1.0, 1.4, 2.0):
        U, R = one_step_case(prob, solver, prec, theta=theta, nsteps=3)
        assert_close(U, R, prec, (theta,))


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", [oracle.HLL, oracle.HLLC])
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT])
def test_2d_random_patch_ragged(prec, solver, bc):
    # 2 x-tiles with a ragged tail, 3 y-tiles with a ragged tail
    prob = wl.random_smooth_patch(2, (70, 19), seed=200 + bc, bc=bc)
    U, R = one_step_case(prob, solver, prec, theta=1.4, nsteps=2)
    assert_close(U, R, prec)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", [oracle.HLL, oracle.HLLC])
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT])
def test_3d_random_patch_ragged(prec, solver, bc):
    prob = wl.random_smooth_patch(3, (67, 11, 13), seed=300 + bc, bc=bc)
    U, R = one_step_case(prob, solver, prec, theta=2.0, nsteps=2, cfl=0.3)
    assert_close(U, R, prec)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", [oracle.HLL, oracle.HLLC])
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT])
def test_smallest_patches(prec, solver, bc):
    """Patches of the fewest cells an active dimension takes (two: every
    ghost layer maps onto the interior) and a few more, in 1D, 2D and 3D."""
    for k, n in enumerate(((2,), (3,), (2, 2), (3, 2), (2, 5), (2, 2, 2), (3, 2, 4), (2, 3, 2))):
        prob = wl.random_smooth_patch(len(n), n, seed=500 + 10 * bc + k, bc=bc)
        U, R = one_step_case(prob, solver, prec, theta=1.4, nsteps=2, cfl=0.3)
        assert_close(U, R, prec, n)


@pytest.mark.parametrize("prec", [64, 32])
def test_3d_mixed_boundaries_and_gravity(prec):
    prob = wl.random_smooth_patch(3, (20, 9, 18), seed=7)
    prob.bc = ((0, 0), (1, 2), (2, 2))
    prob.accel = (0.05, 0.0, -0.1)
    U, R = one_step_case(prob, oracle.HLLC, prec, theta=1.4, nsteps=2, cfl=0.3)
    assert_close(U, R, prec)


def test_sod_fp64_config_matches_oracle_and_exact():
    """1D Sod, 400 cells, FP64, HLLC, minmod, C = 0.4, outflow, t = 0.2: the
    GPU takes the oracle's time steps and must agree to 1e-12; both must lie
    within the first-order discretisation error of the exact solution."""
    prob = wl.sod(400, theta=1.0, cfl=0.4, t_end=0.2)
    d = oracle.Desc.from_problem(prob, solver=oracle.HLLC)
    p = hydro.Patch(prob, precision=64)
    U_ref = p.get_state(hydro.CONSERVED)
    t = 0.0
    while t < 0.2:
        dt = min(oracle.cfl_dt(d, U_ref, 0.4), 0.2 - t)
        gdt = min(p.cfl_dt(0.4), 0.2 - t)
        assert gdt == pytest.approx(dt, rel=1e-13)
        U_ref = oracle.step(d, U_ref, dt)
        p.step(dt, hydro.HLLC)
        t += dt
    U = p.get_state(hydro.CONSERVED)
    assert_close(U, U_ref, 64)
    from oracle import exact_riemann as er
    W = p.get_state(hydro.PRIMITIVE)
    r, u, pr = er.sample_cells((1, 0, 1), (0.125, 0, 0.1), 1.4, 400, 0.5, 0.2)
    assert oracle.l1_error(W[0], r) < 1.5e-2
    assert p.time() == pytest.approx(0.2, rel=1e-14)


@pytest.mark.parametrize("prec", [64, 32])
def test_cfl_dt_matches_oracle(prec):
    for ndim, n in ((1, (130,)), (2, (70, 33)), (3, (40, 17, 9))):
        prob = wl.random_smooth_patch(ndim, n, seed=11 + ndim)
        d = oracle.Desc.from_problem(prob)
        p = hydro.Patch(prob, precision=prec)
        U = p.get_state(hydro.CONSERVED)
        tol = 1e-13 if prec == 64 else 2e-6
        assert p.cfl_dt(0.4) == pytest.approx(oracle.cfl_dt(d, U, 0.4), rel=tol)
        dt = oracle.cfl_dt(d, U, 0.3)
        p.step(dt, hydro.HLLC)  # the fused rate of stage 2
        U1 = p.get_state(hydro.CONSERVED)
        assert p.cfl_dt(0.4) == pytest.approx(oracle.cfl_dt(d, U1, 0.4), rel=tol)
        p.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_totals_match_exact_sums(prec):
    prob = wl.random_smooth_patch(3, (50, 21, 17), seed=5)
    d = oracle.Desc.from_problem(prob)
    p = hydro.Patch(prob, precision=prec)
    U = p.get_state(hydro.CONSERVED)
    got = p.totals()
    want = oracle.totals(d, U)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * np.max(np.abs(want)))
    assert np.array_equal(got, p.totals())  # bitwise reproducible


@pytest.mark.parametrize("solver", [oracle.HLL, oracle.HLLC])
def test_conservation_periodic_fp32(solver):
    prob = wl.smooth_periodic_3d(32)
    p = hydro.Patch(prob, precision=32)
    t0 = p.totals()
    U = p.get_state(hydro.CONSERVED)
    absum = np.array([np.sum(np.abs(U[k])) for k in range(5)]) / 32 ** 3
    nsteps = 50
    p.advance(nsteps, 0.3, solver=solver)
    t1 = p.totals()
    eps32 = 2.0 ** -24
    for k in range(5):
        assert abs(t1[k] - t0[k]) <= 4 * nsteps * eps32 * absum[k], (k, t1[k] - t0[k])


def test_device_dt_loop_matches_host_loop():
    prob = wl.random_smooth_patch(2, (80, 40), seed=9, bc=wl.BC_REFLECT)
    a = hydro.Patch(prob, precision=64)
    b = hydro.Patch(prob, precision=64)
    for _ in range(5):
        a.step(a.cfl_dt(0.4), hydro.HLLC)
    b.advance(5, 0.4, solver=hydro.HLLC)
    assert np.allclose(a.get_state(), b.get_state(), rtol=1e-14, atol=1e-14)
    assert a.time() == pytest.approx(b.time(), rel=1e-14)
    # clipping at t_end: the remaining steps leave the state unchanged
    t_end = b.time() + 0.5 * b.cfl_dt(0.4)
    b.advance(3, 0.4, t_end=t_end, solver=hydro.HLLC)
    assert b.time() == pytest.approx(t_end, rel=1e-14)


@pytest.mark.parametrize("solver", [hydro.HLLC, hydro.HLLC_SWITCH])
def test_graph_replayed_steps_equal_launched_steps(solver):
    """hy_advance_graph replays captured device-dt steps: bit for bit the
    eager hy_advance result, for odd step counts (the graph kept per starting
    parity), repeated replays with state reads between them, a new t_end
    (recapture), and with the timing switch on (events stay out of the
    graph: the replays add no timed launches, eager launches still count)."""
    prob = wl.random_smooth_patch(3, (70, 20, 13), seed=31, bc=wl.BC_PERIODIC)
    a = hydro.Patch(prob, precision=32)
    b = hydro.Patch(prob, precision=32)
    b.set_timing(True)
    b.advance_graph(3, 0.3, solver=solver, prepare_only=True)  # capture only: nothing runs
    assert np.array_equal(a.get_state(), b.get_state()) and b.time() == 0.0
    b.kernel_times()
    for rep in range(3):
        a.advance(3, 0.3, solver=solver)
        b.advance_graph(3, 0.3, solver=solver)
        assert np.array_equal(a.get_state(), b.get_state()), rep
        assert a.time() == b.time()
    ms, launches = b.kernel_times()
    assert list(launches) == [0, 0]
    a.advance(1, 0.3, solver=solver)
    b.advance(1, 0.3, solver=solver)
    ms, launches = b.kernel_times()
    assert list(launches) == [1, 1] and ms[0] > 0 and ms[1] > 0
    assert np.array_equal(a.get_state(), b.get_state())
    t_end = a.time() + 1.5 * a.cfl_dt(0.3)
    a.advance(4, 0.3, t_end=t_end, solver=solver)
    b.advance_graph(4, 0.3, t_end=t_end, solver=solver)
    assert np.array_equal(a.get_state(), b.get_state()) and b.time() == pytest.approx(t_end, rel=1e-14)
    b.set_timing(False)
    a.advance(2, 0.3, solver=solver)
    b.advance_graph(2, 0.3, solver=solver)
    assert np.array_equal(a.get_state(), b.get_state())
    a.close()
    b.close()


def test_one_dimensional_problem_along_x_and_z_fp32():
    """A 1D Sod tube run along z of a 3D patch matches the 1D run along x.
    The two axes go through separately compiled code paths (LDS plane versus
    register z window) whose fused multiply-adds may round differently, so the
    agreement is to FP32 rounding rather than bitwise (the oracle, built
    without contraction, is pinned bitwise)."""
    n = 96
    sod = wl.sod(n, theta=1.4)
    a = hydro.Patch(sod, precision=32)
    W = np.zeros((5, n, 4, 4))
    W[0] = sod.W[0][:, None, None]
    W[3] = sod.W[1][:, None, None]
    W[4] = sod.W[2][:, None, None]
    P3 = types.SimpleNamespace(ndim=3, n=(4, 4, n), lo=(0, 0, 0), hi=(4 / n, 4 / n, 1.0), gamma=1.4,
                               bc=((0, 0), (0, 0), (1, 1)), theta=1.4, accel=(0, 0, 0), W=W)
    b = hydro.Patch(P3, precision=32)
    for _ in range(20):
        dt = a.cfl_dt(0.3)
        assert b.cfl_dt(0.3) == pytest.approx(dt, rel=1e-5)
        a.step(dt, hydro.HLLC)
        b.step(dt, hydro.HLLC)
    Ua = a.get_state()
    Ub = b.get_state().reshape(5, n, 4, 4)
    assert np.all(Ub[1] == 0.0) and np.all(Ub[2] == 0.0)
    for k, src in ((0, 0), (3, 1), (4, 2)):
        ref = np.broadcast_to(Ua[src][:, None, None], (n, 4, 4))
        assert np.max(np.abs(Ub[k] - ref)) <= 1e-5 * np.max(np.abs(Ua[src])) + 1e-7
        # the 16 columns of the 3D patch are identical to each other
        assert np.all(Ub[k] == Ub[k][:, :1, :1])


def test_error_latch_and_host_checks():
    prob = wl.sod(64)
    p = hydro.Patch(prob, precision=32)
    with pytest.raises(hydro.HydroError) as e:
        p.step(-1.0)
    assert e.value.status == hydro.HY_EINVAL
    with pytest.raises(hydro.HydroError) as e:
        p.step(float("nan"))
    assert e.value.status == hydro.HY_EINVAL
    bad = prob.W.copy()
    bad[2, 10] = -1.0
    with pytest.raises(hydro.HydroError) as e:
        p.set_state(bad)
    assert e.value.status == hydro.HY_ESTATE
    bad[2, 10] = float("nan")
    with pytest.raises(hydro.HydroError) as e:
        p.set_state(bad)
    assert e.value.status == hydro.HY_ESTATE
    p.set_state(prob.W)  # a good state clears the latch
    p.step(p.cfl_dt(0.4))
    # a time step far above the CFL limit drives the state non-physical
    for _ in range(20):
        p.step(1.0)
    with pytest.raises(hydro.HydroError) as e:
        p.get_state()
    assert e.value.status == hydro.HY_ESTATE


def _subbox(U, n, lo, size, halo):
    """Periodic extraction of a (size+2 halo)^3 box starting at lo - halo."""
    nx, ny, nz = n
    U4 = U.reshape(5, nz, ny, nx)
    iz = (np.arange(lo[2] - halo, lo[2] + size + halo)) % nz
    iy = (np.arange(lo[1] - halo, lo[1] + size + halo)) % ny
    ix = (np.arange(lo[0] - halo, lo[0] + size + halo)) % nx
    return np.ascontiguousarray(U4[:, iz][:, :, iy][:, :, :, ix])


@pytest.mark.parametrize("solver", [oracle.HLL, oracle.HLLC])
def test_smooth_periodic_256_sampled_against_oracle(solver):
    """Full-size 256^3 periodic smooth flow in the benchmark's launch
    configuration: one step checked on sampled sub-boxes (the oracle steps a
    box with a 4-cell halo, the domain of dependence of one two-stage step)."""
    prob = wl.smooth_periodic_3d(256)
    p = hydro.Patch(prob, precision=32)
    U0 = p.get_state(hydro.CONSERVED)
    dt = p.cfl_dt(0.4)
    p.step(dt, solver)
    U1 = p.get_state(hydro.CONSERVED)
    n = (256, 256, 256)
    rng = np.random.default_rng(3)
    size, halo = 8, 4
    dx = 1.0 / 256
    for _ in range(6):
        lo = rng.integers(0, 256, size=3)
        box0 = _subbox(U0, n, lo, size, halo)
        m = size + 2 * halo
        d = oracle.Desc(3, (m, m, m), (0, 0, 0), (m * dx,) * 3, prob.gamma, ((1, 1),) * 3,
                        solver=solver, theta=2.0)
        ref = oracle.step(d, box0.reshape(5, -1), dt).reshape(5, m, m, m)[:, halo:-halo, halo:-halo, halo:-halo]
        got = _subbox(U1, n, lo, size, 0)
        assert_close(got.reshape(5, -1), ref.reshape(5, -1), 32, tuple(lo))


@pytest.mark.parametrize("nd", [2, 3])
def test_graph_replayed_learned_steps_equal_launched_steps(nd):
    """The learned limiter's steps (slope launches, then the stage kernels
    reading the slopes) replayed from a captured graph: bit for bit the eager
    steps, over repeated replays."""
    from paper_1207_3392_amd import limiter

    n = (70, 20) if nd == 2 else (70, 20, 13)
    prob = wl.random_smooth_patch(nd, n, seed=33, bc=wl.BC_PERIODIC)
    P = limiter.trained_params()
    a = hydro.Patch(prob, precision=32, limiter=hydro.LIM_LEARNED)
    b = hydro.Patch(prob, precision=32, limiter=hydro.LIM_LEARNED)
    a.set_mlp(P)
    b.set_mlp(P)
    b.advance_graph(3, 0.3, solver=hydro.HLLC, prepare_only=True)
    for rep in range(3):
        a.advance(3, 0.3, solver=hydro.HLLC)
        b.advance_graph(3, 0.3, solver=hydro.HLLC)
        assert np.array_equal(a.get_state(), b.get_state()), rep
        assert a.time() == b.time()
    a.close()
    b.close()


@pytest.mark.parametrize("nd", [2, 3])
def test_launch_shapes_give_identical_results_and_autotune(nd, tmp_path):
    """Every supported plane tile computes the same cells with the same
    arithmetic, so two steps agree bit for bit for a given z chunk; z chunks
    (down to a single plane, ragged last chunks) enter the z march at other
    planes, whose entry code may round the z face differently in the last
    place, so across chunks results agree to FP32 roundoff and each matches
    the FP64 oracle to the FP32 bar.  The autotuner keeps one of the shapes
    and leaves U^n, the time and the next step's result unchanged; its JSON
    cache applies the tuned shape."""
    n = (70, 37, 29) if nd == 3 else (150, 77, 1)
    prob = wl.random_smooth_patch(nd, n[:nd], seed=21, bc=wl.BC_REFLECT)
    d = oracle.Desc.from_problem(prob, solver=oracle.HLLC)
    ref = hydro.Patch(prob, precision=32)
    U0 = ref.get_state(hydro.CONSERVED)
    dt = ref.cfl_dt(0.4)
    ref.step(dt, hydro.HLLC)
    ref.step(dt, hydro.HLLC)
    want = ref.get_state(hydro.CONSERVED)
    ref.close()
    orc = oracle.step(d, oracle.step(d, U0, dt), dt)
    tiles = [(64, 8), (64, 4), (32, 8), (32, 16)]
    chunks = [1, 2, 3, 5, 8, 29] if nd == 3 else [1]
    for zc in chunks:
        first = None
        for bx, by in tiles:
            p = hydro.Patch(prob, precision=32)
            p.set_launch_cfg(bx, by, zc)
            assert p.launch_cfg() == (bx, by, zc)
            p.step(dt, hydro.HLLC)
            p.step(dt, hydro.HLLC)
            got = p.get_state(hydro.CONSERVED)
            p.close()
            if first is None:
                first = got
                assert_close(got, orc, 32, ("chunk", zc))
                s = np.max(np.abs(want), axis=1, keepdims=True)
                s[1:-1] = np.maximum(s[1:-1], np.sqrt(2 * s[0] * s[-1]))
                assert np.max(np.abs(got - want) / s) < 1e-6, zc
            else:
                assert np.array_equal(got, first), (bx, by, zc)
    p = hydro.Patch(prob, precision=32)
    with pytest.raises(hydro.HydroError):
        p.set_launch_cfg(16, 8, 1)
    with pytest.raises(hydro.HydroError):
        p.set_launch_cfg(64, 8, n[2] + 1 if nd == 3 else 2)
    dflt = p.launch_cfg()
    Ua, t0 = p.get_state(hydro.CONSERVED), p.time()
    cache = str(tmp_path / "tune.json")
    bx, by, zc, ms = p.autotune(hydro.HLLC, reps=2, cache=cache)
    assert (bx, by) in tiles and ms > 0 and p.launch_cfg() == (bx, by, zc)
    assert np.array_equal(p.get_state(hydro.CONSERVED), Ua) and p.time() == t0
    p.set_launch_cfg(*dflt)
    p.advance(2, 0.4, solver=hydro.HLLC)
    q = hydro.Patch(prob, precision=32)
    q.advance(2, 0.4, solver=hydro.HLLC)
    assert np.array_equal(p.get_state(hydro.CONSERVED), q.get_state(hydro.CONSERVED))
    assert p.time() == q.time()
    p.close()
    q.close()
    r = hydro.Patch(prob, precision=32)
    assert r.autotune(hydro.HLLC, reps=2, cache=cache) == (bx, by, zc, None)
    assert r.launch_cfg() == (bx, by, zc)
    r.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_kinetic_energy_matches_oracle(prec):
    """E_kin per component (the FP64 fixed-order reduction) against the
    oracle's exactly rounded sum over the same stored state; bitwise
    reproducible."""
    for nd, n in ((1, (300,)), (2, (70, 33)), (3, (40, 21, 13))):
        prob = wl.random_smooth_patch(nd, n, seed=40 + nd)
        d = oracle.Desc.from_problem(prob)
        p = hydro.Patch(prob, precision=prec)
        U = p.get_state(hydro.CONSERVED)
        got = p.kinetic_energy()
        want = oracle.kinetic_energy(d, U)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-16), (nd, got, want)
        assert np.all(got[nd:] == 0.0)
        assert np.array_equal(got, p.kinetic_energy())
        p.close()
