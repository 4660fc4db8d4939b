"""Pins of the oracle's fixed multilevel refinement (Sec. 2 prolongation and
restriction; Sec. 3.6, Algs. Evolve, EvolveLevel and StepLevel; Sec. 4.2.3,
conservation of mass, momentum and energy over the leaf cells to numerical
precision).  Each check comes from outside the oracle: brute-force NumPy
averages, exact linear data, the single-level step, symmetry of the initial
data, closed-form translation of a smooth wave, and a planted mistake (the
flux replacement switched off) that must break conservation."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1207_3392_amd import workloads as wl


def build(lv, solver=O.HLL, theta=1.4, no_reflux=False):
    b = lv.base
    d = O.Desc(b.ndim, b.n, b.lo, b.hi, b.gamma, b.bc, solver, theta)
    f = O.FmrDesc(d, lv.boxes, no_reflux)
    Us = [O.prim_to_cons(f.levels[l], W.reshape(b.nv, -1)) for l, W in enumerate(lv.W)]
    return f, Us


def scale(T):
    """(mass, momentum, momentum, momentum, energy) scales of totals T."""
    pm = math.sqrt(2.0 * abs(T[0]) * abs(T[4]))
    return np.array([abs(T[0]), pm, pm, pm, abs(T[4])])


def test_geometry_of_levels():
    lv = wl.sedov_levels(2, 16, 3)
    f, _ = build(lv)
    assert [d.n[:2] for d in f.levels] == [(16, 16)] * 3
    assert f.levels[1].lo[:2] == pytest.approx((-0.25, -0.25)) and f.levels[1].hi[:2] == pytest.approx((0.25, 0.25))
    assert f.levels[2].lo[:2] == pytest.approx((-0.125, -0.125))
    for l in range(3):
        n, lo, hi = lv.level_geometry(l)
        assert n == f.levels[l].n and lo == pytest.approx(f.levels[l].lo) and hi == pytest.approx(f.levels[l].hi)


def test_invalid_boxes_rejected():
    base = O.Desc(2, (16, 16, 1), (0, 0, 0), (1, 1, 1), 1.4, ((0, 0), (0, 0), (0, 0)), O.HLL, 1.4)
    for box in [((1, 4, 0), (8, 8, 1)), ((4, 4, 0), (11, 8, 1)), ((4, 4, 1), (8, 8, 1)), ((4, 4, 0), (0, 8, 1))]:
        with pytest.raises(O.OracleError):
            O.FmrDesc(base, [box])
    sw = O.Desc(2, (16, 16, 1), (0, 0, 0), (1, 1, 1), 1.4, ((0, 0), (0, 0), (0, 0)), O.HLLC_SWITCH, 1.4)
    with pytest.raises(O.OracleError):
        O.FmrDesc(sw, [((4, 4, 0), (8, 8, 1))])


def _ghost_prims(f, l, ext):
    """Primitive values of the prolonged exterior of level l, as a dict from
    ghosted (i, j, k) of level l (interior-relative) to the primitive vector."""
    d = f.levels[l]
    m = f.ghosted_shape(l)
    g = [O.NG if q < d.ndim else 0 for q in range(3)]
    out = {}
    for k in range(m[2]):
        for j in range(m[1]):
            for i in range(m[0]):
                c = (k * m[1] + j) * m[0] + i
                if np.isnan(ext[0, c]):
                    continue
                u = ext[:, c]
                rho = u[0]
                v = u[1:1 + d.ndim] / rho
                p = (d.gamma - 1.0) * (u[d.ndim + 1] - 0.5 * rho * np.dot(v, v))
                out[(i - g[0], j - g[1], k - g[2])] = np.concatenate([[rho], v, [p]])
    return out


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_prolongation_exact_on_linear_data(nd):
    """Linear primitive fields have equal one-sided differences, so the
    limited slope is the exact gradient and every child takes the linear
    function's value at its own centre."""
    n0 = 8
    base = O.Desc(nd, tuple(n0 if q < nd else 1 for q in range(3)), (0, 0, 0), (1, 1, 1), 1.4,
                  tuple((1, 1) for _ in range(3)), O.HLLC, 1.4)
    box = (tuple(2 if q < nd else 0 for q in range(3)), tuple(4 if q < nd else 1 for q in range(3)))
    f = O.FmrDesc(base, [box])
    grad = [(0.3, -0.2, 0.1), (0.05, 0.1, -0.07), (-0.04, 0.02, 0.03), (0.01, -0.02, 0.05), (0.2, 0.1, -0.1)]

    def lin(v, x):
        return [2.0, 0.3, -0.2, 0.1, 3.0][v] + sum(grad[v][q] * x[q] for q in range(nd))

    pd = f.levels[0]
    W = np.zeros((nd + 2, pd.ncell))
    for c in range(pd.ncell):
        idx = (c % pd.n[0], (c // pd.n[0]) % pd.n[1], c // (pd.n[0] * pd.n[1]))
        x = [pd.lo[q] + (idx[q] + 0.5) * (pd.hi[q] - pd.lo[q]) / pd.n[q] for q in range(3)]
        for v in range(nd + 1):
            W[v, c] = lin(v, x)
        W[nd + 1, c] = lin(4, x)
    U = O.prim_to_cons(pd, W)
    ext = O.fmr_prolong(f, 1, U)
    cd = f.levels[1]
    got = _ghost_prims(f, 1, ext)
    assert len(got) == np.prod(f.ghosted_shape(1)) - cd.ncell
    for (i, j, k), w in got.items():
        idx = (i, j, k)
        x = [cd.lo[q] + (idx[q] + 0.5) * (cd.hi[q] - cd.lo[q]) / cd.n[q] for q in range(3)]
        want = [lin(v, x) for v in range(nd + 1)] + [lin(4, x)]
        assert np.allclose(w, want, rtol=0, atol=1e-13), (idx, w, want)


def test_prolongation_children_mean_and_extremum():
    """The 2^d children of a parent average to the parent's primitives (the
    offsets are +-1/4 symmetric), and a parent that is a local extremum along
    every dimension has zero slopes, so its children equal it."""
    lv = wl.smooth_levels(2, 16, 2, amp=0.3)
    f, Us = build(lv)
    pd = f.levels[0]
    rng = np.random.default_rng(5)
    Wp = O.cons_to_prim(pd, Us[0]).copy()
    Wp *= 1.0 + 0.2 * rng.uniform(-1, 1, size=Wp.shape) * np.array([1, 0, 0, 1])[:, None]
    Wp[1:3] += 0.3 * rng.uniform(-1, 1, size=Wp[1:3].shape)
    # parent (3, 6): a strict local maximum of every variable
    c = 6 * 16 + 3
    for v in range(4):
        nb = [Wp[v, c - 1], Wp[v, c + 1], Wp[v, c - 16], Wp[v, c + 16]]
        Wp[v, c] = max(nb) + 0.5
    U = O.prim_to_cons(pd, Wp)
    got = _ghost_prims(f, 1, O.fmr_prolong(f, 1, U))
    lo = lv.boxes[0][0]
    for pj in range(lo[1] - 1, lo[1] + 9):
        for pi in range(lo[0] - 1, lo[0] + 9):
            ch = [(2 * (pi - lo[0]) + a, 2 * (pj - lo[1]) + b, 0) for a in (0, 1) for b in (0, 1)]
            if not all(k in got for k in ch):
                continue
            mean = np.mean([got[k] for k in ch], axis=0)
            assert np.allclose(mean, Wp[:, pj * 16 + pi], rtol=1e-13, atol=1e-13)
            if (pi, pj) == (3, 6):
                for k in ch:
                    assert np.allclose(got[k], Wp[:, c], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_restriction_is_mean_of_children(nd):
    lv = wl.smooth_levels(nd, 8, 2)
    f, Us = build(lv)
    rng = np.random.default_rng(7)
    cd, pd = f.levels[1], f.levels[0]
    Uc = Us[1] * (1.0 + 0.1 * rng.uniform(-1, 1, size=Us[1].shape))
    Up = O.fmr_restrict(f, 1, Uc, Us[0])
    shape_c = tuple(reversed(cd.n[:nd]))
    blocks = Uc.reshape((nd + 2,) + shape_c)
    for ax in range(nd):
        s = list(blocks.shape)
        s[1 + ax:2 + ax] = [s[1 + ax] // 2, 2]
        blocks = blocks.reshape(s).mean(axis=2 + ax)
    lo, n = lv.boxes[0]
    P = Up.reshape((nd + 2,) + tuple(reversed(pd.n[:nd])))
    sl = tuple(slice(lo[q], lo[q] + n[q]) for q in reversed(range(nd)))
    assert np.allclose(P[(slice(None),) + sl], blocks, rtol=1e-14, atol=0)
    # cells outside the box keep their values
    mask = f.covered(0)
    assert np.array_equal(Up[:, ~mask], Us[0][:, ~mask])


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_single_level_reduces_to_step(nd):
    lv = wl.smooth_levels(nd, 8, 1)
    f, Us = build(lv, O.HLLC, 2.0)
    d = f.levels[0]
    (U1,), dt = O.fmr_step(f, Us, dt_fixed=1e-3)
    assert dt == 1e-3
    assert np.array_equal(U1, O.step(d, Us[0], 1e-3))
    (U2,), dt2 = O.fmr_step(f, Us, cfl=0.4)
    assert dt2 == O.cfl_dt(d, Us[0], 0.4)
    assert np.array_equal(U2, O.step(d, Us[0], dt2))


def test_subcycling_time_steps():
    """With the deepest step fixed, the coarse step is 2^(L-1) of it."""
    lv = wl.smooth_levels(2, 16, 3)
    f, Us = build(lv)
    _, dt = O.fmr_step(f, Us, dt_fixed=1e-4)
    assert dt == pytest.approx(4e-4, rel=1e-15)


@pytest.mark.parametrize("nd,n0,nlev,solver", [(1, 32, 4, O.HLL), (2, 16, 3, O.HLL), (2, 16, 3, O.HLLC),
                                               (3, 8, 2, O.HLLC)])
def test_leaf_totals_conserved(nd, n0, nlev, solver):
    """Sec. 4.2.3: mass, momentum and energy over the leaf cells stay constant
    to numerical precision once the blast has crossed level boundaries
    (periodic outer boundary, so nothing leaves the box)."""
    lv = wl.sedov_levels(nd, n0, nlev, bc=wl.BC_PERIODIC)
    f, Us = build(lv, solver)
    T0 = O.fmr_totals(f, Us)
    for _ in range(12):
        Us, _ = O.fmr_step(f, Us, 0.4)
    T1 = O.fmr_totals(f, Us)
    assert np.all(np.abs(T1 - T0) <= 1e-13 * scale(T0)), (T1 - T0) / scale(T0)
    # the blast has reached the coarse/fine boundaries by now: dropping the
    # flux replacement must be visible
    fb, Ub = build(lv, solver, no_reflux=True)
    for _ in range(12):
        Ub, _ = O.fmr_step(fb, Ub, 0.4)
    Tb = O.fmr_totals(fb, Ub)
    assert np.max(np.abs(Tb - T0) / scale(T0)) > 1e-6


def test_uniform_flow_stays_uniform():
    lv = wl.smooth_levels(2, 16, 3, uniform=True)
    f, Us = build(lv, O.HLLC, 2.0)
    U0 = [U.copy() for U in Us]
    for _ in range(3):
        Us, _ = O.fmr_step(f, Us, 0.4)
    for a, b in zip(Us, U0):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13)


def test_blast_keeps_its_symmetry():
    """The centred blast on centred boxes is symmetric under x -> -x and
    under x <-> y; a wrong index or a transposed operand anywhere in the
    multilevel step would break either."""
    lv = wl.sedov_levels(2, 16, 3)
    f, Us = build(lv, O.HLLC)
    for _ in range(10):
        Us, _ = O.fmr_step(f, Us, 0.4)
    for l, U in enumerate(Us):
        n = f.levels[l].n[0]
        A = U.reshape(4, n, n)  # (v, y, x)
        scl = np.abs(A).max(axis=(1, 2))[:, None, None] + 1e-300
        mir = A[:, :, ::-1].copy()
        mir[1] = -mir[1]
        assert np.all(np.abs(mir - A) <= 1e-12 * scl)
        tr = A.transpose(0, 2, 1)[[0, 2, 1, 3]]
        assert np.all(np.abs(tr - A) <= 1e-12 * scl)


@pytest.mark.parametrize("nd", [1, 2])
def test_smooth_wave_accuracy(nd):
    """A density wave carried through a refined box: the refined level is
    markedly more accurate than one level alone there, and the coarse leaf
    cells are no worse than the single level's (closed-form translation as
    the reference)."""
    n0 = 32
    lv = wl.smooth_levels(nd, n0, 2)
    f, Us = build(lv, O.HLLC, 1.4)
    d = f.levels[0]
    U1 = Us[0].copy()
    dtf = 0.4 / n0 / 4.0
    steps = 40
    for _ in range(steps):
        Us, _ = O.fmr_step(f, Us, dt_fixed=dtf)
        U1 = O.step(d, U1, 2 * dtf)
    ex = wl.smooth_levels(nd, n0, 2, t=steps * 2 * dtf)
    e_fine = np.abs(Us[1][0] - ex.W[1][0].ravel()).mean()
    leaf = ~f.covered(0)
    e_leaf = np.abs(Us[0][0] - ex.W[0][0].ravel())[leaf].mean()
    s_leaf = np.abs(U1[0] - ex.W[0][0].ravel())[leaf].mean()
    s_cov = np.abs(U1[0] - ex.W[0][0].ravel())[~leaf].mean()
    assert e_fine < 0.5 * s_cov
    assert e_leaf < 1.05 * s_leaf
