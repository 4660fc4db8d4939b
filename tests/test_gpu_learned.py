"""The learned limiter on the GPU: MFMA inference and training kernels against
the FP64 oracle (bf16 operand rounding emulated there), the TVD clamp, the
training data, a learned-limiter step, and a short training run."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from oracle import training_data as td
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

import torch  # noqa: E402


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return (mlp.init_params(seed) + scale * rng.normal(size=mlp.NPARAM)).astype(np.float32)


def test_mfma_inference_matches_oracle():
    P = random_params(1)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(10000, 4)).astype(np.float32)
    tr = hydro.Trainer(P)
    y = tr.eval(torch.from_numpy(X).cuda()).cpu().numpy()
    ref, _ = mlp.forward(P.astype(np.float64), X.astype(np.float64), bf16=True)
    err = np.abs(y - ref)
    # FP32 accumulation against FP64: rare bf16 ties of the hidden layer differ by one bf16 ulp
    assert np.quantile(err, 0.999) < 1e-4 * (1 + np.abs(ref).max())
    assert err.max() < 2e-2 * (1 + np.abs(ref).max())
    # ragged batch sizes (tails of a wave)
    for b in (1, 63, 65, 257):
        yb = tr.eval(torch.from_numpy(X[:b]).cuda()).cpu().numpy()
        assert np.array_equal(yb, y[:b])
    tr.close()


def test_mfma_inference_is_exactly_homogeneous_under_power_of_two_scaling():
    """The network is positively homogeneous: scaling W1 and every bias by 2^j
    scales the output by 2^j.  With bf16 operands and FP32 accumulation this
    holds bit for bit (powers of two commute with rounding), also when the
    weights' bound moves the kernel's internal power-of-two shift (j up to 40)
    and when it is zero (all weights tiny)."""
    P = random_params(17)
    rng = np.random.default_rng(18)
    X = rng.uniform(-1, 1, size=(4096, 4)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    W1, b1, W2, b2, w3, b3 = mlp.unpack(P)
    tr = hydro.Trainer(P)
    y0 = tr.eval(Xd).cpu().numpy()
    tr.close()
    assert np.any(y0 != 0)
    for j in (1, 7, 40, -20):
        Pj = mlp.pack(W1 * 2.0 ** j, b1 * 2.0 ** j, W2, b2 * 2.0 ** j, w3, b3 * 2.0 ** j).astype(np.float32)
        tr = hydro.Trainer(Pj)
        yj = tr.eval(Xd).cpu().numpy()
        tr.close()
        assert np.array_equal(yj, (y0.astype(np.float64) * 2.0 ** j).astype(np.float32)), j


def _abs_gradient(P, X, T, bf16=True):
    """Per-parameter sum over the batch of the magnitudes of the terms that
    make up the oracle's gradient (the backward pass on |.| of every factor,
    the ReLU masks kept).  Each term of the GPU's sum carries at most a few
    bf16 roundings of its factors (relative 2^-9 each), so a per-element
    error bound is a small multiple of 2^-9 times this."""
    y, (Xb, W1, W2, w3, z1, h1, z2, h2) = mlp.forward(P, X, bf16)
    r = np.abs(2.0 * (y - T) / len(T))
    dz2 = np.outer(r, np.abs(w3)) * (z2 > 0)
    dz1 = (dz2 @ np.abs(W2)) * (z1 > 0)
    return mlp.pack(dz1.T @ np.abs(Xb), dz1.sum(axis=0), dz2.T @ np.abs(h1), dz2.sum(axis=0),
                    np.abs(h2).T @ r, np.array([r.sum()]))


def _training_batch(seed, n=5000, batch=3000):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)
    T = rng.normal(scale=0.5, size=n).astype(np.float32)
    idx = rng.choice(n, size=batch, replace=False).astype(np.int32)
    return X, T, idx


def test_training_gradient_matches_oracle_per_element():
    P = random_params(3)
    X, T, idx = _training_batch(4)
    tr = hydro.Trainer(P)
    g, loss = tr.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), torch.from_numpy(idx).cuda())
    Xb, Tb = X[idx].astype(np.float64), T[idx].astype(np.float64)
    lref, gref = mlp.loss_and_grad(P.astype(np.float64), Xb, Tb, bf16=True)
    assert loss == pytest.approx(lref, rel=2e-3)
    # every element: the GPU rounds dZ2, dZ1, H1, X, W2 (and H2, w3) to bf16
    # as backward operands; a few roundings of 2^-9 per term, summed over the
    # batch, bound the difference by 2^-6 of the sum of the term magnitudes
    A = _abs_gradient(P.astype(np.float64), Xb, Tb)
    err = np.abs(g - gref)
    bound = 2.0 ** -6 * A + 1e-7 * np.abs(gref).max()
    worst = int(np.argmax(err / bound))
    assert np.all(err <= bound), (worst, err[worst], bound[worst], g[worst], gref[worst])
    # and most elements far inside it
    assert np.median(err / (A + 1e-30)) < 2.0 ** -9
    tr.close()


def test_adam_steps_match_oracle_adam():
    """Three hy_trainer_step calls on one batch: after each, every master
    weight equals the oracle's Adam (bias corrections with the step count
    1, 2, 3) applied to the gradient the device step used (read before the
    step with hy_trainer_gradient, same fixed-order reduction), to FP32
    rounding; the first update also matches Adam on the oracle's own
    gradient wherever the two gradients agree in sign."""
    P = random_params(13)
    X, T, idx = _training_batch(14)
    tr = hydro.Trainer(P)
    Xd, Td, Id = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), torch.from_numpy(idx).cuda()
    Pref = tr.params().astype(np.float64)
    assert np.array_equal(Pref, P.astype(np.float64))
    m = np.zeros(mlp.NPARAM)
    v = np.zeros(mlp.NPARAM)
    lr = 2e-3
    for t in (1, 2, 3):
        g, _ = tr.gradient(Xd, Td, Id)
        tr.step(Xd, Td, Id, lr=lr)
        got = tr.params().astype(np.float64)
        Pref, m, v = mlp.adam(Pref, g.astype(np.float64), m, v, t, lr=lr)
        # FP32 master weights: the update itself (<= lr) is formed in FP32
        assert np.all(np.abs(got - Pref) <= 4e-7 * np.abs(Pref) + 2e-6 * lr), t
        Pref = got  # carry the device weights so rounding does not accumulate
        if t == 1:
            gref = mlp.loss_and_grad(P.astype(np.float64), X[idx].astype(np.float64),
                                     T[idx].astype(np.float64), bf16=True)[1]
            P1_oracle = mlp.adam(P.astype(np.float64), gref, np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), 1,
                                 lr=lr)[0]
            same = (np.sign(g) == np.sign(gref)) & (np.abs(gref) > 1e-6)
            assert same.mean() > 0.95
            d_dev, d_orc = got - P, P1_oracle - P
            assert np.all(np.abs(d_dev[same] - d_orc[same]) <= 0.05 * lr)
    tr.close()


def test_learned_slopes_match_oracle_and_stay_in_tvd_region():
    P = random_params(5, scale=0.5)
    for bc in (wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT):
        prob = wl.random_smooth_patch(2, (70, 21), seed=6 + bc, bc=bc)
        p = hydro.Patch(prob, precision=32, limiter=hydro.LIM_LEARNED, set_initial=False)
        p.set_mlp(P)
        p.set_state(prob.W)
        S = p.learned_slopes().cpu().numpy()
        W = p.get_state(hydro.PRIMITIVE).reshape(4, 21, 70)
        nv = 4
        worst = 0.0
        for q in range(2):
            ax = 1 - q
            for v in range(nv):
                w = W[v]
                st = np.stack([np.roll(w, 2 - k, axis=ax) for k in range(5)], axis=-1)
                sl = S[q * nv + v].reshape(21, 70)
                dm = st[..., 2] - st[..., 1]
                dp = st[..., 3] - st[..., 2]
                interior = np.ones_like(w, dtype=bool)
                if bc != wl.BC_PERIODIC:  # oracle stencils below use periodic wrap; skip 2 cells at walls
                    if ax == 1:
                        interior[:, :2] = interior[:, -2:] = False
                    else:
                        interior[:2, :] = interior[-2:, :] = False
                # clamp invariant; the primitives read back here can differ from the
                # kernel's own by an ulp, so differences within FP32 noise are tolerated
                noise = 4e-7 * np.max(np.abs(st), axis=-1)
                lim = 2 * np.minimum(np.abs(dm), np.abs(dp))
                ok = np.where(dm * dp <= 0, np.abs(sl) <= 2 * noise + lim,
                              (np.sign(dp) * sl >= -2 * noise) & (np.abs(sl) <= lim * (1 + 1e-5) + 2 * noise))
                assert np.all(ok[interior]), (bc, q, v)
                idx = np.argwhere(interior)[::7]
                for (j, i) in idx[:200]:
                    ref = oracle.limiter_learned(P.astype(np.float64), st[j, i].astype(np.float64), bf16=True)
                    scale = np.max(np.abs(np.diff(st[j, i]))) + 1e-30
                    worst = max(worst, abs(sl[j, i] - ref) / scale)
        assert worst < 2e-2, worst
        p.close()


def test_learned_limiter_step_matches_oracle():
    P = random_params(8, scale=0.2)
    for ndim, n in ((1, (200,)), (2, (40, 24)), (3, (20, 12, 10))):
        prob = wl.random_smooth_patch(ndim, n, seed=9 + ndim, bc=wl.BC_PERIODIC)
        d = oracle.Desc.from_problem(prob, solver=oracle.HLLC, limiter=oracle.LIM_LEARNED,
                                     mlp=P.astype(np.float64), mlp_bf16=True)
        p = hydro.Patch(prob, precision=32, limiter=hydro.LIM_LEARNED, set_initial=False)
        p.set_mlp(P)
        p.set_state(prob.W)
        U0 = p.get_state(hydro.CONSERVED)
        dt = oracle.cfl_dt(d, U0, 0.3)
        p.step(dt, hydro.HLLC)
        U1 = p.get_state(hydro.CONSERVED)
        ref = oracle.step(d, U0, dt)
        s = np.max(np.abs(ref), axis=1, keepdims=True)
        err = np.abs(U1 - ref) / s
        # slopes of bf16 networks: rare operand ties shift a slope by a bf16 ulp
        assert np.mean(err) < 2e-5, (ndim, np.mean(err))
        assert err.max() < 2e-3, (ndim, err.max())
        p.close()


@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT])
def test_learned_limiter_on_the_smallest_patches(bc):
    """The learned limiter's 5-cell stencil on patches of two to five cells
    along a dimension: every stencil reaches ghost cells, whose slopes come
    from the boundary map (periodic source, zero for outflow, mirrored for a
    reflecting wall), against the oracle's step."""
    P = random_params(8, scale=0.2)
    for k, n in enumerate(((2,), (5,), (2, 3), (5, 2), (2, 2, 2), (3, 2, 5))):
        prob = wl.random_smooth_patch(len(n), n, seed=70 + 10 * bc + k, bc=bc)
        d = oracle.Desc.from_problem(prob, solver=oracle.HLLC, limiter=oracle.LIM_LEARNED,
                                     mlp=P.astype(np.float64), mlp_bf16=True)
        p = hydro.Patch(prob, precision=32, limiter=hydro.LIM_LEARNED, set_initial=False)
        p.set_mlp(P)
        p.set_state(prob.W)
        U0 = p.get_state(hydro.CONSERVED)
        dt = oracle.cfl_dt(d, U0, 0.3)
        p.step(dt, hydro.HLLC)
        U1 = p.get_state(hydro.CONSERVED)
        p.close()
        ref = oracle.step(d, U0, dt)
        s = np.max(np.abs(ref), axis=1, keepdims=True)
        err = np.abs(U1 - ref) / s
        assert np.mean(err) < 2e-5 and err.max() < 2e-3, (n, np.mean(err), err.max())


def test_training_samples_match_oracle():
    prob = wl.kelvin_helmholtz(64)
    p = hydro.Patch(prob, precision=32)
    p.advance(20, 0.4, solver=hydro.HLLC)
    U = p.get_state(hydro.CONSERVED)
    x, t = p.make_samples()
    x, t = x.cpu().numpy(), t.cpu().numpy()
    xr, tr, sr, wr = td.samples(U, 2, prob.n, prob.gamma, return_scale=True)
    assert x.shape == xr.shape and t.shape == tr.shape
    # x = d / s carries the FP32 rounding of the coarse averages amplified by
    # |w| / s (about 1e-7 |w| / s); compare the samples with s > 1e-3 |w|
    good = sr > 1e-3 * (np.abs(wr) + 1e-3)
    assert good.mean() > 0.2
    ex = np.abs(x - xr).max(axis=1)[good]
    et = np.abs(t - tr)[good]
    assert np.quantile(ex, 0.999) < 1e-3 and np.quantile(et, 0.999) < 1e-2, (np.quantile(ex, 0.999), np.quantile(et, 0.999))
    assert np.median(ex) < 1e-5
    p.close()


def test_short_training_reduces_the_loss():
    from paper_1207_3392_amd import limiter
    x, t = limiter.fine_samples(256, times=(0.2, 0.4))
    x, t = limiter.augment(x, t)
    params, losses = limiter.train(x, t, steps=300, batch=16384, lr=2e-3, log_every=50)
    assert np.all(np.isfinite(params))
    first, last = losses[0][1], losses[-1][1]
    assert last < 0.6 * first, losses


def _learned_run_vs_oracle(prob, P, steps):
    d = oracle.Desc.from_problem(prob, solver=oracle.HLLC, limiter=oracle.LIM_LEARNED,
                                 mlp=P.astype(np.float64), mlp_bf16=True)
    p = hydro.Patch(prob, precision=32, limiter=hydro.LIM_LEARNED, set_initial=False)
    p.set_mlp(P)
    p.set_state(prob.W)
    U = p.get_state(hydro.CONSERVED)
    worst_mean, worst_max = 0.0, 0.0
    for _ in range(steps):
        dt = oracle.cfl_dt(d, U, prob.cfl)
        ref = oracle.step(d, U, dt)
        p.set_state(U, hydro.CONSERVED)
        p.step(dt, hydro.HLLC)
        G = p.get_state(hydro.CONSERVED)
        # per-variable scale; a momentum component is measured against the
        # flow's momentum scale sqrt(2 rho E), since one that starts at zero
        # (v_x, v_y of Rayleigh-Taylor) carries the FP32 cancellation error of
        # the pressure flux while its own maximum is still tiny
        s = np.max(np.abs(ref), axis=1, keepdims=True)
        s[1:-1] = np.maximum(s[1:-1], np.sqrt(2.0 * s[0] * s[-1]))
        err = np.abs(G - ref) / s
        assert np.all(np.isfinite(G))
        worst_mean = max(worst_mean, float(err.mean()))
        worst_max = max(worst_max, float(err.max()))
        U = ref
    p.close()
    return worst_mean, worst_max


def test_learned_limiter_on_discontinuities_and_flat_zero_stencils():
    """Sod (1D, outflow) and the implosion (2D, reflecting walls): fluid at rest
    gives flat stencils of exact zeros, whose normalisation must stay finite;
    before that was guarded, a NaN input of one lane reached the other lanes of
    its MFMA column and zeroed their slopes.  Each step starts from the
    oracle's state, so errors do not accumulate."""
    P = random_params(11, scale=0.3)
    for prob, steps in ((wl.sod(128, theta=2.0, cfl=0.4), 12), (wl.implosion(48), 6)):
        mean, mx = _learned_run_vs_oracle(prob, P, steps)
        # bf16 rounding of inputs that differ by FP32 rounding can move a slope
        # by a bf16 ulp (0.4 %) next to a jump
        assert mean < 1e-4 and mx < 1e-2, (prob.name, mean, mx)


def test_training_samples_finite_on_flat_zero_stencils():
    n = 64
    x = (np.arange(n) + 0.5) / n
    W = np.zeros((4, n, n))
    W[0] = 1.0 + 0.1 * np.sin(2 * np.pi * x)[None, :]
    W[3] = 1.0
    prob = wl.Problem(2, (n, n, 1), (0, 0, 0), (1, 1, 1), 1.4, ((0, 0), (0, 0), (0, 0)), W)
    p = hydro.Patch(prob, precision=32)
    xs, ts = p.make_samples()
    xs, ts = xs.cpu().numpy(), ts.cpu().numpy()
    assert np.all(np.isfinite(xs)) and np.all(np.isfinite(ts))
    xr, tr = td.samples(p.get_state(hydro.CONSERVED), 2, prob.n, prob.gamma)
    flat = np.all(xr == 0, axis=1)
    assert flat.mean() > 0.5  # velocity stencils and every stencil along y
    assert np.all(xs[flat] == 0) and np.all(ts[flat] == 0)
    p.close()


def test_learned_limiter_rayleigh_taylor_small():
    """3D, gravity source, reflecting z walls, periodic x and y, v_x = v_y = 0."""
    P = random_params(12, scale=0.3)
    mean, mx = _learned_run_vs_oracle(wl.rayleigh_taylor_3d(16), P, 3)
    assert mean < 1e-4 and mx < 1e-2, (mean, mx)
