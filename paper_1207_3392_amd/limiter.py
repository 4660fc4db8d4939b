"""Learned slope limiter: training data from fine GPU runs and GPU training.

The network replaces the generalised minmod of eq. MinMod.  Training data come
from runs of the plain method (HLLC, monotonized central) on a fine periodic
grid, restricted 4x by the library (hy_lim_make_samples); the training loop
draws minibatches on the device and calls the library's forward/backward and
Adam kernels (hy_trainer_step).  Augmentation enforces the limiter's odd
symmetries: flipping the sign of the data flips inputs and target; mirroring
the stencil reverses and negates the inputs and negates the target.
"""
from __future__ import annotations

import numpy as np

from . import hydro
from . import workloads as wl

IN, H = 4, 32


def trained_params() -> np.ndarray:
    """The shipped network: trained on plain-method Kelvin-Helmholtz runs at
    2048^2 restricted to 512^2 (three sharp-layer seeds and two smooth layer
    widths), by ``python -m paper_1207_3392_amd.limiter_study train``; its
    training and evaluation record is data/kh_limiter_study.json."""
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "kh_limiter.npy")
    w = np.load(path, allow_pickle=False).astype(np.float32)
    assert w.shape == (1249,)
    return w


def init_params(seed: int = 1207) -> np.ndarray:
    """He initialisation (seeded), flat in the library's parameter order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [
        rng.normal(0.0, np.sqrt(2.0 / IN), size=H * IN),
        np.zeros(H),
        rng.normal(0.0, np.sqrt(2.0 / H), size=H * H),
        np.zeros(H),
        rng.normal(0.0, np.sqrt(1.0 / H), size=H),
        np.zeros(1),
    ]
    return np.concatenate(parts).astype(np.float32)


def fine_samples(n_fine: int = 1024, times=(0.3, 0.6, 0.9), seed: int = wl.DEFAULT_SEED, cfl: float = 0.4,
                 gamma: float = 5.0 / 3.0, width: float = 0.0):
    """Kelvin-Helmholtz (shear-layer half-width ``width``, 0 = sharp) on an
    n_fine^2 periodic grid (plain HLLC, MC limiter, FP32) sampled at the given
    times; returns device tensors x (n, 4), t (n)."""
    import torch

    prob = wl.kelvin_helmholtz(n_fine, seed=seed, gamma=gamma, width=width)
    p = hydro.Patch(prob, precision=32)
    xs, ts = [], []
    for T in times:
        while p.time() < T * (1 - 1e-12):
            p.advance(200, cfl, t_end=T, solver=hydro.HLLC)
        x, t = p.make_samples()
        xs.append(x)
        ts.append(t)
    p.close()
    return torch.cat(xs), torch.cat(ts)


def augment(x, t):
    """Add the sign-flipped, mirrored and mirrored-flipped copies."""
    import torch

    rev = torch.flip(x, dims=[1])
    return torch.cat([x, -x, -rev, rev]), torch.cat([t, -t, -t, t])


def train(x, t, steps: int = 3000, batch: int = 65536, lr: float = 1e-3, seed: int = wl.DEFAULT_SEED,
          params=None, log_every: int = 0, log=None, cosine: bool = False):
    """Adam on the device (rate lr, or lr (1 + cos(pi k / steps)) / 2 at step k
    with cosine); returns (params (1249,) float32, list of (step, minibatch
    loss) every log_every steps, also passed to log)."""
    import math

    import torch

    tr = hydro.Trainer(init_params(seed) if params is None else params, device=str(x.device))
    gen = torch.Generator(device=x.device)
    gen.manual_seed(seed)
    n = x.shape[0]
    if n >= 2 ** 31:
        raise ValueError(f"{n} samples: minibatch indices are int32, at most 2^31 - 1 samples")
    losses = []
    for k in range(steps):
        idx = torch.randint(0, n, (batch,), device=x.device, dtype=torch.int32, generator=gen)
        tr.step(x, t, idx, lr * 0.5 * (1.0 + math.cos(math.pi * k / steps)) if cosine else lr)
        if log_every and (k % log_every == 0 or k == steps - 1):
            losses.append((k, tr.loss()))
            if log is not None:
                log(f"step {k}: loss {losses[-1][1]:.5g}")
    out = tr.params()
    tr.close()
    return out, losses


def coarse_reference(n_coarse: int, t_end: float, seed: int = wl.DEFAULT_SEED, cfl: float = 0.4,
                     gamma: float = 5.0 / 3.0, refine: int = 4):
    """Plain-method run at refine x n_coarse, restricted (block-averaged
    conserved variables) to n_coarse^2; returns the coarse density."""
    prob = wl.kelvin_helmholtz(n_coarse * refine, seed=seed, gamma=gamma)
    p = hydro.Patch(prob, precision=32)
    while p.time() < t_end * (1 - 1e-12):
        p.advance(200, cfl, t_end=t_end, solver=hydro.HLLC)
    U = p.get_state(hydro.CONSERVED)
    p.close()
    nf = n_coarse * refine
    D = U[0].reshape(n_coarse, refine, n_coarse, refine).mean(axis=(1, 3))
    return D


def coarse_run(n: int, t_end: float, params=None, seed: int = wl.DEFAULT_SEED, cfl: float = 0.4,
               gamma: float = 5.0 / 3.0):
    """KH at n^2 with the learned limiter (params given) or the MC limiter;
    returns (density, wall seconds, steps)."""
    import time

    import torch

    prob = wl.kelvin_helmholtz(n, seed=seed, gamma=gamma)
    lim = hydro.LIM_LEARNED if params is not None else hydro.LIM_THETA
    p = hydro.Patch(prob, precision=32, limiter=lim, set_initial=params is None)
    if params is not None:
        p.set_mlp(params)
        p.set_state(prob.W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while p.time() < t_end * (1 - 1e-12):
        p.advance(50, cfl, t_end=t_end, solver=hydro.HLLC)
        steps += 50
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    U = p.get_state(hydro.CONSERVED)
    p.close()
    return U[0].reshape(n, n), wall, steps
