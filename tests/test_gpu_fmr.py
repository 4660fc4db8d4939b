"""Fixed multilevel refinement on the GPU (Sec. 3.6, Algs. Evolve,
EvolveLevel, StepLevel) against the oracle's, through the C ABI.

Both sides start from the GPU's initial level states read back as FP64 and
take the same deepest-level time step, so a comparison isolates the kernels'
arithmetic: FP64 within 1e-11 of each variable's scale, FP32 within the
precision the state is held in.  Leaf-cell totals stay constant to the
state's precision, as Sec. 4.2.3 states for the multilevel Sedov runs."""
import math

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


def scale(U):
    s = np.max(np.abs(U), axis=1, keepdims=True)
    m = math.sqrt(2.0 * s[0, 0] * s[-1, 0])
    s[1:-1] = np.maximum(s[1:-1], m)
    return np.maximum(s, 1e-300)


def oracle_fmr(lv, solver, theta=None):
    b = lv.base
    d = oracle.Desc(b.ndim, b.n, b.lo, b.hi, b.gamma, b.bc, solver, b.theta if theta is None else theta)
    return oracle.FmrDesc(d, lv.boxes)


def compare(F, f, Us, prec, what):
    worst = 0.0
    for l in range(F.nlev):
        got = F.get_state(l, hydro.CONSERVED)
        s = scale(Us[l])
        err = np.abs(got - Us[l]) / s
        worst = max(worst, float(err.max()))
        if prec == 64:
            assert err.max() < 1e-11, (what, l, err.max(axis=1))
        else:
            assert err.max() < 1e-4, (what, l, err.max(axis=1))
            assert np.all(np.mean(np.abs(got - Us[l]), axis=1) / s[:, 0] < 5e-6), (what, l)
    return worst


CASES = [
    ("sedov1d", lambda: wl.sedov_levels(1, 64, 4)),
    ("sedov2d", lambda: wl.sedov_levels(2, 32, 3)),
    ("sedov3d", lambda: wl.sedov_levels(3, 16, 2)),
    # seven levels, as in the paper's 2D multilevel runs (finest spacing 1/2048)
    ("sedov2d_7levels", lambda: wl.sedov_levels(2, 32, 7)),
    # uneven boxes and a non-square base: ragged tiles on every level
    ("smooth2d_ragged", lambda: wl.smooth_levels(2, 0, boxes=[((5, 3, 0), (13, 9, 1)), ((4, 2, 0), (9, 7, 1))],
                                                 n=(40, 24))),
    ("smooth3d_ragged", lambda: wl.smooth_levels(3, 0, boxes=[((3, 2, 4), (7, 9, 5))], n=(13, 14, 15))),
    # the smallest boxes the margin rule allows: one or two parent cells
    ("tiny1d", lambda: wl.smooth_levels(1, 0, boxes=[((2, 0, 0), (1, 1, 1))], n=(5,))),
    ("tiny2d", lambda: wl.smooth_levels(2, 0, boxes=[((2, 2, 0), (2, 3, 1))], n=(6, 7))),
    ("tiny3d", lambda: wl.smooth_levels(3, 0, boxes=[((2, 2, 2), (1, 2, 1))], n=(5, 6, 5))),
]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", [hydro.HLL, hydro.HLLC])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_levels_match_oracle(name, make, solver, prec):
    lv = make()
    print(f"fmr parity {name} solver={solver} fp{prec}", flush=True)
    F = hydro.Fmr(lv, precision=prec)
    f = oracle_fmr(lv, solver)
    Us = [F.get_state(l, hydro.CONSERVED) for l in range(F.nlev)]
    # the deepest level's time step: the oracle's CFL step of the start state
    dtf = oracle.cfl_dt(f.levels[-1], Us[-1], 0.4)
    for k in range(3):
        Us, dt_o = oracle.fmr_step(f, Us, dt_fixed=dtf)
        dt_g = F.step(dt_fixed=dtf, solver=solver)
        assert dt_g == pytest.approx(dt_o, rel=1e-15)
        compare(F, f, Us, prec, f"{name} step {k}")
    F.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_cfl_time_steps_match_oracle(prec):
    """With the deepest level's CFL step taken on each side from its own
    state, the coarse steps agree to the state's precision."""
    lv = wl.sedov_levels(2, 32, 3)
    F = hydro.Fmr(lv, precision=prec)
    f = oracle_fmr(lv, hydro.HLLC)
    Us = [F.get_state(l, hydro.CONSERVED) for l in range(F.nlev)]
    for k in range(3):
        Us, dt_o = oracle.fmr_step(f, Us, cfl=0.4)
        dt_g = F.step(cfl=0.4, solver=hydro.HLLC)
        assert dt_g == pytest.approx(dt_o, rel=1e-13 if prec == 64 else 1e-5)
    compare(F, f, Us, prec, "cfl")
    F.close()


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("nd,n0,nlev", [(1, 64, 4), (2, 32, 3), (3, 16, 3)])
def test_leaf_totals_conserved(nd, n0, nlev, prec):
    lv = wl.sedov_levels(nd, n0, nlev, bc=wl.BC_PERIODIC)
    F = hydro.Fmr(lv, precision=prec)
    f = oracle_fmr(lv, hydro.HLLC)
    T0 = F.totals()
    want = oracle.fmr_totals(f, [F.get_state(l, hydro.CONSERVED) for l in range(F.nlev)])
    pm = math.sqrt(2 * T0[0] * T0[4])
    sc = np.array([T0[0], pm, pm, pm, T0[4]])
    assert np.all(np.abs(T0 - want) <= 1e-13 * sc)
    for _ in range(10):
        F.step(cfl=0.4, solver=hydro.HLLC)
    T1 = F.totals()
    tol = 1e-12 if prec == 64 else 2e-6
    assert np.all(np.abs(T1 - T0) <= tol * sc), (T1 - T0) / sc
    F.close()


def test_single_level_equals_patch_step():
    """One level is the single-patch update: the same kernels, bitwise."""
    lv = wl.smooth_levels(2, 32, 1)
    F = hydro.Fmr(lv, precision=32)
    P = hydro.Patch(lv.base, precision=32)
    for _ in range(3):
        F.step(dt_fixed=2e-3, solver=hydro.HLLC)
        P.step(2e-3, hydro.HLLC)
    assert np.array_equal(F.get_state(0), P.get_state())
    F.close()
    P.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_graph_replays_match_eager_launches(prec):
    """The captured global step, replayed several times with reads of the
    state in between and a change of cfl (a recapture), gives bit for bit the
    states of the same step launched kernel by kernel."""
    lv = wl.sedov_levels(2, 32, 3)
    G = hydro.Fmr(lv, precision=prec)
    E = hydro.Fmr(lv, precision=prec)
    E.set_graph(False)
    for k, cfl in enumerate([0.4, 0.4, 0.4, 0.3, 0.3]):
        dg = G.step(cfl=cfl, solver=hydro.HLLC)
        de = E.step(cfl=cfl, solver=hydro.HLLC)
        assert dg == de, k
        for l in range(3):
            assert np.array_equal(G.get_state(l), E.get_state(l)), (k, l)
        assert np.array_equal(G.totals(), E.totals())
        if k == 2:
            # a new state on every level between replays: the captured step
            # reads whatever the levels hold
            for l in range(3):
                W = lv.W[l].reshape(4, -1).copy()
                W[0] *= 1.1
                G.set_state(l, W, hydro.PRIMITIVE)
                E.set_state(l, W, hydro.PRIMITIVE)
    G.close()
    E.close()


def test_autotune_changes_no_result():
    """Tiles never change a result; the tuned shapes are among the supported
    ones, and a step after tuning matches a step without it."""
    lv = wl.sedov_levels(3, 16, 2)
    A = hydro.Fmr(lv, precision=32)
    B = hydro.Fmr(lv, precision=32)
    shapes = B.autotune(hydro.HLL, 2)
    assert len(shapes) == 2 and all(s[0] in (32, 64) for s in shapes)
    for F in (A, B):
        F.step(dt_fixed=1e-3, solver=hydro.HLL)
    for l in range(2):
        a, b = A.get_state(l), B.get_state(l)
        s = scale(a)
        assert np.max(np.abs(a - b) / s) < 1e-6
    A.close()
    B.close()


def test_blast_symmetry_fp64():
    lv = wl.sedov_levels(2, 32, 3)
    F = hydro.Fmr(lv, precision=64)
    for _ in range(6):
        F.step(cfl=0.4, solver=hydro.HLLC)
    for l in range(F.nlev):
        A = F.get_state(l).reshape(4, 32, 32)
        scl = np.abs(A).max(axis=(1, 2))[:, None, None]
        mir = A[:, :, ::-1].copy()
        mir[1] = -mir[1]
        assert np.all(np.abs(mir - A) <= 1e-11 * scl)
        tr = A.transpose(0, 2, 1)[[0, 2, 1, 3]]
        assert np.all(np.abs(tr - A) <= 1e-11 * scl)
    F.close()


def test_host_checks():
    lv = wl.sedov_levels(2, 16, 2)
    with pytest.raises(hydro.HydroError) as e:
        hydro.Fmr(wl.sedov_levels(2, 16, 2, boxes=[((1, 4, 0), (8, 8, 1))]))
    assert e.value.status == hydro.HY_EINVAL
    with pytest.raises(hydro.HydroError) as e:
        hydro.Fmr(wl.sedov_levels(2, 16, 2, boxes=[((4, 4, 0), (11, 8, 1))]))
    assert e.value.status == hydro.HY_EINVAL
    F = hydro.Fmr(lv, precision=32)
    for bad in [dict(solver=hydro.HLLC_SWITCH), dict(cfl=0.0), dict(cfl=float("nan"))]:
        args = dict(cfl=0.4, dt_fixed=0.0, solver=hydro.HLLC)
        args.update(bad)
        with pytest.raises(hydro.HydroError) as e:
            F.step(**args)
        assert e.value.status == hydro.HY_EINVAL
    out = np.zeros(4 * 16 * 16)
    for level in (-1, 2):
        assert hydro.lib().hy_fmr_get_state(F.handle, level, hydro.CONSERVED, hydro._dptr(out)) == hydro.HY_EINVAL
    F.close()


def test_multilevel_blast_tracks_the_single_level_run():
    """Sec. 4.2.3 compares multilevel Sedov runs with a single level at the
    finest resolution: the shock positions are similar.  Here the 2D blast on
    three levels (64^2 each, finest 1/256) runs until its shock has crossed
    the finest level's boundary; its shock radius along +x (the density
    maximum in the leaf cells of level 1) lies within two level-1 cells of a
    single-level 256^2 run's at the same time, both near the dimensional
    estimate R = (E t^2 / rho)^(1/4)."""
    lv = wl.sedov_levels(2, 64, 3, bc=wl.BC_OUTFLOW)
    F = hydro.Fmr(lv, precision=32)
    T0 = F.totals()
    t = 0.0
    while t < 0.03:
        t += F.step(cfl=0.4, solver=hydro.HLL)
    T = F.totals()
    W1 = F.get_state(1, hydro.PRIMITIVE).reshape(4, 64, 64)  # level 1: [-0.25, 0.25]^2, dx 1/128
    x1 = -0.25 + (np.arange(64) + 0.5) / 128
    row = W1[0, 31]  # y just below 0
    leaf = x1 > 0.125  # outside level 2
    r_fmr = x1[leaf][np.argmax(row[leaf])]

    single = wl.sedov_levels(2, 256, 1, bc=wl.BC_OUTFLOW)  # one level at the finest spacing
    P = hydro.Patch(single.base, precision=32)
    while P.time() < t * (1 - 1e-12):
        P.advance(50, 0.4, t_end=t, solver=hydro.HLL)
    assert P.time() == pytest.approx(t, rel=1e-9)
    Ws = P.get_state(hydro.PRIMITIVE).reshape(4, 256, 256)
    xs = -0.5 + (np.arange(256) + 0.5) / 256
    rs = Ws[0, 127]
    r_single = xs[xs > 0][np.argmax(rs[xs > 0])]
    print(f"t={t:.4f} r_fmr={r_fmr:.4f} r_single={r_single:.4f} estimate={t ** 0.5:.4f}")
    assert abs(r_fmr - r_single) <= 2.0 / 128
    for r in (r_fmr, r_single):
        assert abs(r - t ** 0.5) < 0.15 * t ** 0.5
    # nothing has reached the outer boundary yet: totals as at the start
    assert abs(T[0] - T0[0]) < 1e-6 * T0[0] and abs(T[4] - T0[4]) < 1e-5 * T0[4]
    F.close()
    P.close()


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("solver", [hydro.HLL, hydro.HLLC])
def test_uniform_flow_stays_uniform(prec, solver):
    """A uniform moving flow over nested levels (prolongation of a uniform
    parent, coarse/fine replacement of equal fluxes, restriction of equal
    children) stays uniform through three global steps to a few roundings."""
    eps = 2.0 ** -52 if prec == 64 else 2.0 ** -23
    for lv in (wl.smooth_levels(2, 32, 3, uniform=True), wl.smooth_levels(3, 16, 2, uniform=True)):
        F = hydro.Fmr(lv, precision=prec)
        U0 = [F.get_state(l, hydro.CONSERVED) for l in range(F.nlev)]
        for _ in range(3):
            F.step(0.4, solver=solver)
        for l in range(F.nlev):
            U = F.get_state(l, hydro.CONSERVED)
            s = np.max(np.abs(U0[l]), axis=1, keepdims=True)
            assert np.max(np.abs(U - U0[l]) / s) <= 8 * eps, (lv.base.ndim, l, np.max(np.abs(U - U0[l]) / s))
        F.close()
