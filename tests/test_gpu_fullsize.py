"""Full-size configurations in the benchmark's launch configuration, checked
on sampled sub-boxes that the FP64 oracle steps one by one.

One two-stage step reaches 2 cells per stage with the generalised minmod (a
face needs the slopes of its two cells, a slope the neighbours of its cell)
and 3 with the learned limiter's 5-cell stencil, so an oracle box with a halo
of 4 (6) cells reproduces its interior exactly.  Where a box touches a
reflecting wall it starts at the wall and the oracle applies the wall there;
periodic dimensions wrap."""
import numpy as np
import pytest

import oracle
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


def box_indices(n, lo, size, halo, mode):
    """Index window along one dimension and the (start, stop) of the compared
    cells inside it; mode is 'wrap', 'low' (box starts at the wall), 'high'
    (box ends at the wall) or 'inner' (no wall within reach)."""
    if mode == "wrap":
        return np.arange(lo - halo, lo + size + halo) % n, (halo, halo + size)
    if mode == "low":
        return np.arange(0, size + halo), (0, size)
    if mode == "high":
        return np.arange(n - size - halo, n), (halo, halo + size)
    assert lo - halo >= 0 and lo + size + halo <= n
    return np.arange(lo - halo, lo + size + halo), (halo, halo + size)


def oracle_box_step(prob, U, lo, size, halo, modes, dt, **desc_kw):
    nd, nv = prob.ndim, prob.ndim + 2
    n = list(prob.n)
    shape = (nv,) + tuple(n[q] for q in reversed(range(3)))  # (nv, nz, ny, nx)
    U4 = U.reshape(shape)
    idx, cmp = [], []
    for q in range(3):
        if q < nd:
            i, c = box_indices(n[q], lo[q], size, halo, modes[q])
        else:
            i, c = np.arange(1), (0, 1)
        idx.append(i)
        cmp.append(c)
    box = U4[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]
    m = [len(idx[q]) for q in range(3)]
    dx = [(prob.hi[q] - prob.lo[q]) / n[q] for q in range(3)]
    bc = []
    for q in range(3):
        wall = prob.bc[q]
        lo_bc = wall[0] if modes[q] == "low" else wl.BC_OUTFLOW
        hi_bc = wall[1] if modes[q] == "high" else wl.BC_OUTFLOW
        bc.append((lo_bc, hi_bc) if q < nd else (wl.BC_PERIODIC, wl.BC_PERIODIC))
    d = oracle.Desc(nd, tuple(m), (0.0, 0.0, 0.0), tuple(m[q] * dx[q] for q in range(3)), prob.gamma, tuple(bc),
                    accel=prob.accel, **desc_kw)
    ref = oracle.step(d, np.ascontiguousarray(box).reshape(nv, -1), dt).reshape(box.shape)
    sl = (slice(None),) + tuple(slice(*cmp[q]) for q in reversed(range(3)))
    return ref[sl], idx, cmp


def gpu_box(prob, U1, idx, cmp):
    nv = prob.ndim + 2
    shape = (nv,) + tuple(prob.n[q] for q in reversed(range(3)))
    U4 = U1.reshape(shape)
    sel = [idx[q][cmp[q][0]:cmp[q][1]] for q in range(3)]
    return U4[:, sel[2]][:, :, sel[1]][:, :, :, sel[0]]


def scale(ref):
    s = np.max(np.abs(ref.reshape(ref.shape[0], -1)), axis=1)
    s[1:-1] = np.maximum(s[1:-1], np.sqrt(2.0 * s[0] * s[-1]))
    return s.reshape((-1,) + (1,) * (ref.ndim - 1))


def test_kelvin_helmholtz_2048_plain_and_learned_sampled():
    """2D Kelvin-Helmholtz at 2048^2 after 40 steps (shear layers rolled
    into structure), one more step checked on 8 boxes, plain MC limiter and
    the shipped learned limiter."""
    from paper_1207_3392_amd import limiter

    prob = wl.kelvin_helmholtz(2048)
    P = limiter.trained_params()
    rng = np.random.default_rng(11)
    for learned in (False, True):
        lim = hydro.LIM_LEARNED if learned else hydro.LIM_THETA
        p = hydro.Patch(prob, precision=32, limiter=lim, set_initial=False)
        if learned:
            p.set_mlp(P)
        p.set_state(prob.W)
        p.advance(40, 0.4, solver=hydro.HLLC)
        U0 = p.get_state(hydro.CONSERVED)
        dt = p.cfl_dt(0.4)
        p.step(dt, hydro.HLLC)
        U1 = p.get_state(hydro.CONSERVED)
        p.close()
        kw = dict(solver=oracle.HLLC, theta=2.0)
        if learned:
            kw.update(limiter=oracle.LIM_LEARNED, mlp=P.astype(np.float64), mlp_bf16=True)
        halo = 6 if learned else 4
        for _ in range(8):
            lo = rng.integers(0, 2048, size=3)
            lo[0] = lo[0] if rng.random() < 0.5 else 2048 - 8  # some boxes across the periodic seam
            ref, idx, cmp = oracle_box_step(prob, U0, lo, 32, halo, ("wrap", "wrap", None), dt, **kw)
            got = gpu_box(prob, U1, idx, cmp)
            err = np.abs(got - ref) / scale(ref)
            if learned:
                assert err.mean() < 1e-4 and err.max() < 1e-2, (tuple(lo), err.mean(), err.max())
            else:
                assert err.max() < 2e-5 and err.mean() < 2e-6, (tuple(lo), err.max(), err.mean())


def test_rayleigh_taylor_512_sampled():
    """3D Rayleigh-Taylor at 512^3 (gravity, periodic x and y, reflecting z
    walls), one HLLC step at C = 0.3 after 10 steps, checked on boxes inside
    the domain and on boxes against each wall."""
    prob = wl.rayleigh_taylor_3d(512)
    p = hydro.Patch(prob, precision=32)
    p.advance(10, 0.3, solver=hydro.HLLC)
    U0 = p.get_state(hydro.CONSERVED)
    dt = p.cfl_dt(0.3)
    p.step(dt, hydro.HLLC)
    U1 = p.get_state(hydro.CONSERVED)
    m0 = p.totals()[0]
    p.close()
    rng = np.random.default_rng(12)
    for zmode in ("inner", "inner", "low", "low", "high", "high"):
        lo = rng.integers(0, 512, size=3)
        lo[2] = rng.integers(8, 512 - 16)
        ref, idx, cmp = oracle_box_step(prob, U0, lo, 8, 4, ("wrap", "wrap", zmode), dt, solver=oracle.HLLC,
                                        theta=2.0)
        got = gpu_box(prob, U1, idx, cmp)
        err = np.abs(got - ref) / scale(ref)
        assert err.max() < 2e-5 and err.mean() < 2e-6, (zmode, tuple(lo), err.max(), err.mean())
    assert np.isfinite(m0) and m0 > 0


def test_rayleigh_taylor_512_200_steps_learned_vs_plain_and_oracle_subbox():
    """The 3D Rayleigh-Taylor configuration as specified: 512^3, 200 HLLC steps
    with the shipped learned limiter and with the plain MC limiter.  Both
    conserve mass to roundoff and stay physical; the learned run stays close to
    the plain one (the interface has only begun to grow); and the 200th learned
    and plain steps match the FP64 oracle on a 64^3 sub-box across the
    interface (halo 6 for the learned 5-cell stencil, 4 for MC)."""
    from paper_1207_3392_amd import limiter

    prob = wl.rayleigh_taylor_3d(512)
    P = limiter.trained_params()
    lo = np.array([224, 224, 224])  # z = 224..287 straddles the interface at z = 0
    dens = {}
    for learned in (True, False):
        lim = hydro.LIM_LEARNED if learned else hydro.LIM_THETA
        p = hydro.Patch(prob, precision=32, limiter=lim, set_initial=False)
        if learned:
            p.set_mlp(P)
        p.set_state(prob.W)
        m0 = p.totals()[0]
        p.advance(199, prob.cfl, solver=hydro.HLLC)
        U0 = p.get_state(hydro.CONSERVED)
        dt = p.cfl_dt(prob.cfl)
        p.step(dt, hydro.HLLC)
        U1 = p.get_state(hydro.CONSERVED)
        m1 = p.totals()[0]
        p.close()
        assert np.all(np.isfinite(U1))
        assert abs(m1 - m0) <= 4 * 200 * 2 ** -24 * abs(m0), (learned, m0, m1)
        dens[learned] = U1[0]
        kw = dict(solver=oracle.HLLC, theta=2.0)
        if learned:
            kw.update(limiter=oracle.LIM_LEARNED, mlp=P.astype(np.float64), mlp_bf16=True)
        ref, idx, cmp = oracle_box_step(prob, U0, lo, 64, 6 if learned else 4, ("wrap", "wrap", "inner"), dt, **kw)
        del U0
        got = gpu_box(prob, U1, idx, cmp)
        del U1
        err = np.abs(got - ref) / scale(ref)
        if learned:
            assert err.mean() < 1e-4 and err.max() < 1e-2, (err.mean(), err.max())
        else:
            assert err.max() < 2e-5 and err.mean() < 2e-6, (err.max(), err.mean())
    diff = np.sum(np.abs(dens[True] - dens[False])) / np.sum(np.abs(dens[False]))
    print(f"RT 512^3 200 steps: relative L1 density difference learned vs plain {diff:.3e}")
    assert diff < 1e-4, diff  # measured 2.2e-6: at t = 0.06 the interface has barely moved


@pytest.mark.parametrize("solver,cfl,nz", [(oracle.HLLC, 0.4, 512), (oracle.HLL, 0.3, 512),
                                           (oracle.HLLC_SWITCH, 0.4, 512), (oracle.HLLC, 0.4, 64)])
def test_smooth_periodic_512_graph_replayed_step_sampled(solver, cfl, nz):
    """The 512^3 periodic smooth flow (FP32, gamma 5/3) in the benchmark's
    launch configuration, and the 512 x 512 x 64 slab of cubic cells (one
    GPU's share of the 512^3 patch split eight ways): two launched steps, then
    one step replayed from a captured graph with the step size from the
    device's CFL reduction.  The step size matches the oracle's CFL step of
    the whole state, and sampled sub-boxes match the oracle's step of a box
    with a 4-cell halo."""
    prob = wl.smooth_periodic_3d(512, nz=nz)
    prob.hi = (prob.hi[0], prob.hi[1], prob.lo[2] + nz / 512)
    d = oracle.Desc.from_problem(prob, solver=solver, theta=2.0, shock_fp32=True)
    p = hydro.Patch(prob, precision=32)
    p.advance(2, cfl, solver=solver)
    p.advance_graph(1, cfl, solver=solver, prepare_only=True)
    U0 = p.get_state(hydro.CONSERVED)
    t0 = p.time()
    p.advance_graph(1, cfl, solver=solver)
    U1 = p.get_state(hydro.CONSERVED)
    dt = p.time() - t0
    p.close()
    assert dt == pytest.approx(oracle.cfl_dt(d, U0, cfl), rel=2e-6)
    rng = np.random.default_rng(5)
    for _ in range(6):
        lo = rng.integers(0, (512, 512, nz))
        ref, idx, cmp = oracle_box_step(prob, U0, lo, 8, 4, ("wrap",) * 3, dt, solver=solver, theta=2.0,
                                        shock_fp32=True)
        got = gpu_box(prob, U1, idx, cmp)
        err = np.abs(got - ref) / scale(ref)
        assert err.max() < 2e-5 and err.mean() < 2e-6, (tuple(lo), err.max(), err.mean())


def test_largest_patch_one_step_sampled():
    """The largest patch the library takes in FP32: 1023 x 1023 x 1024 cells,
    each variable's array 4.29e9 bytes, just under the 4 GiB that the
    kernels' 32-bit byte offsets address (the host refuses one cell layer
    more).  A smooth periodic shear flow with an FP32-representable
    conserved state; one HLLC step checked on sampled sub-boxes, among them
    boxes at the far end of the arrays (the largest offsets)."""
    n = (1023, 1023, 1024)
    nv = 5
    gamma = 5.0 / 3.0
    prob = wl.Problem(3, n, (0.0, 0.0, 0.0), (1.0, 1.0, 1024 / 1023), gamma, ((0, 0),) * 3, None, theta=2.0)
    c = [np.cos(2 * np.pi * (np.arange(m) + 0.5) / m) for m in n]
    s = [np.sin(2 * np.pi * (np.arange(m) + 0.5) / m) for m in n]
    U = np.empty((nv, n[2], n[1], n[0]))
    rho = U[0]
    rho[...] = 1.0
    rho += 0.1 * c[0][None, None, :]
    rho += 0.1 * c[1][None, :, None]
    rho += 0.1 * c[2][:, None, None]
    np.multiply(rho, 0.1 * s[1][None, :, None], out=U[1])  # S_x = rho v_x(y)
    np.multiply(rho, 0.1 * s[2][:, None, None], out=U[2])  # S_y = rho v_y(z)
    np.multiply(rho, 0.1 * s[0][None, None, :], out=U[3])  # S_z = rho v_z(x)
    for k in range(4):
        U[k] = U[k].astype(np.float32)
    # G = p / (gamma - 1) + |S|^2 / (2 rho), p = 1
    G = U[4]
    np.square(U[1], out=G)
    G += np.square(U[2])
    G += np.square(U[3])
    G /= 2.0 * rho
    G += 1.0 / (gamma - 1.0)
    U[4] = G.astype(np.float32)
    U = U.reshape(nv, -1)
    p = hydro.Patch(prob, precision=32, set_initial=False)
    p.set_state(U, hydro.CONSERVED)
    dt = p.cfl_dt(0.4)
    p.step(dt, hydro.HLLC)
    U1 = p.get_state(hydro.CONSERVED)
    p.close()
    rng = np.random.default_rng(9)
    los = [rng.integers(0, n) for _ in range(4)] + [np.array(n) - 8, np.array(n) - 5]
    for lo in los:
        ref, idx, cmp = oracle_box_step(prob, U, lo, 8, 4, ("wrap",) * 3, dt, solver=oracle.HLLC, theta=2.0)
        got = gpu_box(prob, U1, idx, cmp)
        err = np.abs(got - ref) / scale(ref)
        assert err.max() < 2e-5 and err.mean() < 2e-6, (tuple(lo), err.max(), err.mean())
