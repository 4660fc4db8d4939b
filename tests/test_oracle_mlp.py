"""Pins of the oracle's learned-limiter pieces: the hand-written backward pass
against central finite differences, the C forward against the NumPy forward,
the TVD clamp region, bf16 rounding, and the training-data targets on data
whose slopes are known in closed form."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from oracle import training_data as td


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    P = mlp.init_params(3) + 0.05 * rng.normal(size=mlp.NPARAM)
    X = rng.uniform(-1, 1, size=(64, 4))
    T = rng.normal(size=64)
    loss, g = mlp.loss_and_grad(P, X, T)
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, size=120, replace=False)
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (mlp.loss_and_grad(Pp, X, T)[0] - mlp.loss_and_grad(Pm, X, T)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9), i


def test_c_forward_matches_numpy_forward():
    rng = np.random.default_rng(1)
    P = mlp.init_params(7) + 0.1 * rng.normal(size=mlp.NPARAM)
    X = rng.uniform(-1, 1, size=(200, 4))
    for bf16 in (False, True):
        y, _ = mlp.forward(P, X, bf16)
        yc = np.array([oracle.mlp_forward(P, x, bf16) for x in X])
        assert np.allclose(yc, y, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_is_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7  # bf16 spacing at 1
    vals = np.array([one + ulp / 2, one + 3 * ulp / 2, one + ulp / 4, -(one + 3 * ulp / 2), 1e-3])
    r = mlp.bf16_round(vals)
    assert r[0] == one            # tie to even (mantissa 0)
    assert r[1] == one + 2 * ulp  # tie to even (mantissa 2)
    assert r[2] == one
    assert r[3] == -(one + 2 * ulp)
    assert abs(r[4] - 1e-3) <= 1e-3 * 2 ** -8


def test_learned_slope_stays_in_tvd_region():
    rng = np.random.default_rng(2)
    P = mlp.init_params(11) + 0.5 * rng.normal(size=mlp.NPARAM)
    for _ in range(3000):
        w = rng.normal(size=5) * 10.0 ** rng.uniform(-3, 2)
        s = oracle.limiter_learned(P, w)
        dm, dp = w[2] - w[1], w[3] - w[2]
        if dm * dp <= 0:
            assert s == 0.0
        else:
            assert 0.0 <= np.sign(dp) * s <= 2 * min(abs(dm), abs(dp)) * (1 + 1e-15)


def test_learned_limiter_scheme_is_conservative():
    from paper_1207_3392_amd import workloads as wl
    prob = wl.random_smooth_patch(2, (12, 10), seed=3, bc=wl.BC_PERIODIC)
    P = mlp.init_params(5)
    d = oracle.Desc.from_problem(prob, limiter=oracle.LIM_LEARNED, mlp=P, mlp_bf16=True)
    U0 = oracle.prim_to_cons(d, prob.flat())
    U1 = oracle.run_steps(d, U0, 3, 0.4)
    t0, t1 = oracle.totals(d, U0), oracle.totals(d, U1)
    assert np.allclose(t0, t1, rtol=1e-13, atol=1e-14)


def _linear_field(n, ndim, slope):
    """Conserved state of rho = 1 + slope x, v = 0, p = 1 on a periodic box
    of cell width 1/n: a ramp that wraps at the boundary."""
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + slope * x
    if ndim == 1:
        R = rho
    else:
        R = np.broadcast_to(rho, (n, n))
    nv = ndim + 2
    U = np.zeros((nv,) + R.shape)
    U[0] = R
    U[-1] = 1.0 / 0.4
    return U.reshape(nv, -1)


def test_training_targets_on_linear_data():
    """Away from the wrap of a periodic ramp, the sub-cell averages of a
    linear density lie on a line: the least-squares slope is the coarse
    difference, the stencil inputs are all equal, so x = (1, 1, 1, 1) and the
    target is exactly 1; across x the ramp wraps, and along y nothing varies."""
    n = 64
    for ndim in (1, 2):
        U = _linear_field(n, ndim, 0.3)
        x, t = td.samples(U, ndim, (n, n if ndim == 2 else 1, 1), 1.4)
        nc = (n // 4) ** ndim
        xr, tr = x[:nc], t[:nc]  # q = 0, variable rho
        cx = np.arange(nc) % (n // 4)
        inner = (cx >= 2) & (cx <= n // 4 - 3)
        assert np.allclose(xr[inner], 1.0, atol=1e-12)
        assert np.allclose(tr[inner], 1.0, rtol=1e-9)
        if ndim == 2:
            qy = slice(4 * nc, 5 * nc)  # q = 1, variable rho: constant along y
            assert np.all(x[qy] == 0.0) and np.all(t[qy] == 0.0)


def test_flat_stencils_give_zero_inputs_and_slope():
    """A flat stencil (all differences zero, including a field of exact zeros
    such as the velocity of fluid at rest) normalises to the zero input and a
    zero slope; the floor term of s keeps the division defined."""
    P = mlp.init_params(5)
    for c in (0.0, 1.0, -3.5, 1e-20):
        w = np.full(5, c)
        assert oracle.limiter_learned(P, w) == 0.0
        x, s, _ = mlp.stencil_features(w[None, :])
        assert s[0] > 0.0 and np.all(x == 0.0)


# ------------------------------------------------------------- Adam ----
# Kingma & Ba, "Adam: a method for stochastic optimization" (2015), Alg. 1:
# m_t = b1 m + (1 - b1) g, v_t = b2 v + (1 - b2) g^2, mh = m_t / (1 - b1^t),
# vh = v_t / (1 - b2^t), p -= lr mh / (sqrt(vh) + eps).


def test_adam_first_step_from_zero_moments_is_normalised_gradient():
    """From zero moments the bias corrections give mh = g and vh = g^2, so the
    first update is -lr g / (|g| + eps) element by element."""
    rng = np.random.default_rng(21)
    P = rng.normal(size=mlp.NPARAM)
    g = rng.normal(size=mlp.NPARAM) * 10.0 ** rng.uniform(-6, 2, size=mlp.NPARAM)
    lr = 3e-3
    P1, m, v = mlp.adam(P, g, np.zeros_like(P), np.zeros_like(P), 1, lr=lr)
    assert np.allclose(P1 - P, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_moves_every_step_by_the_same_amount():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step t, so each step moves by -lr g / (|g| + eps); a wrong
    step count in the bias correction breaks this from the second step on."""
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    P = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    for t in range(1, 30):
        P2, m, v = mlp.adam(P, g, m, v, t, lr=1e-2)
        assert np.allclose(P2 - P, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-10), t
        P = P2


def test_adam_two_steps_hand_computed():
    """Gradients 1 then -2 on one parameter, lr 0.1: m2 = 0.9 * 0.1 - 0.2 =
    -0.11, v2 = 0.999 * 0.001 + 0.004 = 0.004999, mh = -0.11 / 0.19,
    vh = 0.004999 / 0.001999; the two updates are -0.1 / (1 + 1e-8) and
    0.1 * (0.11 / 0.19) / (sqrt(0.004999 / 0.001999) + 1e-8)."""
    from fractions import Fraction as F
    import math

    m1, v1 = F(1, 10), F(1, 1000)
    m2 = F(9, 10) * m1 + F(1, 10) * (-2)
    v2 = F(999, 1000) * v1 + F(1, 1000) * 4
    assert m2 == F(-11, 100) and v2 == F(4999, 1000000)
    mh = m2 / (1 - F(9, 10) ** 2)
    vh = v2 / (1 - F(999, 1000) ** 2)
    step1 = -0.1 / (1.0 + 1e-8)
    step2 = -0.1 * float(mh) / (math.sqrt(float(vh)) + 1e-8)
    P = np.array([0.5])
    P1, m, v = mlp.adam(P, np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=0.1)
    assert P1[0] == pytest.approx(0.5 + step1, rel=1e-15)
    P2, m, v = mlp.adam(P1, np.array([-2.0]), m, v, 2, lr=0.1)
    assert m[0] == pytest.approx(-0.11, rel=1e-14) and v[0] == pytest.approx(0.004999, rel=1e-14)
    assert P2[0] == pytest.approx(0.5 + step1 + step2, rel=1e-14)
    assert step2 > 0.0  # the second gradient reverses the motion
