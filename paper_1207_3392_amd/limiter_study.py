"""Train the learned slope limiter and measure what it buys at matched error.

Training data come from plain-method Kelvin-Helmholtz runs (HLLC, monotonized
central limiter, FP32; the Sec. 4.3.1 setup) on fine periodic grids, restricted
4x by the library; several seeds of the initial random perturbation give
independent runs, and one more seed is held out for validation.

The evaluation is a posteriori: the same problem is run with the plain and
the learned limiter at a ladder of resolutions N and compared, through the L1
norm of the density error (the norm of the paper's convergence tables), with
a plain run at the finest resolution restricted to each N by block averages
of the conserved density.  "Matched L1" then reads, from the plain method's
L1(N) curve, the resolution the plain method needs to reach the learned
limiter's error (log-log interpolation), and the wall time either needs.
Two 1D problems complete the picture: the Sod shock tube (Sec. 4.2.1) and
the smooth density wave (Sec. 4.1.1), also against fine plain runs.

Usage:
    python -m paper_1207_3392_amd.limiter_study train --out weights.npy
    python -m paper_1207_3392_amd.limiter_study eval --weights weights.npy --json out.json
    python -m paper_1207_3392_amd.limiter_study c3 --json out.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import diagnostics, hydro, limiter
from . import workloads as wl

HELD_OUT_SEED = 4242


# ---------------------------------------------------------------------------
# training


def training_set(n_fine: int, runs, times, cfl: float = 0.4, log=None):
    """Samples (x, t) on the device from fine KH runs, one per (seed, width)."""
    import torch

    xs, ts = [], []
    for seed, width in runs:
        t0 = time.perf_counter()
        x, t = limiter.fine_samples(n_fine, times=times, seed=seed, cfl=cfl, width=width)
        xs.append(x)
        ts.append(t)
        if log:
            log(f"run seed {seed} width {width}: {x.shape[0]} samples at {n_fine}^2 ({time.perf_counter() - t0:.1f} s)")
    return torch.cat(xs), torch.cat(ts)


def mc_normalised(x):
    """The monotonized-central slope (theta = 2) in the sample's normalised
    units, from the two central differences of the stencil."""
    import torch

    dm, dp = x[:, 1], x[:, 2]
    a, b, c = 2 * dm, 0.5 * (dm + dp), 2 * dp
    s = torch.sign(b)
    m = torch.minimum(torch.minimum(a.abs(), b.abs()), c.abs())
    ok = (torch.sign(a) == s) & (torch.sign(c) == s)
    return torch.where(ok, s * m, torch.zeros_like(m))


def tvd_clamp_normalised(x, y):
    import torch

    dm, dp = x[:, 1], x[:, 2]
    sg = torch.where(dp > 0, torch.ones_like(dp), -torch.ones_like(dp))
    lim = 2 * torch.minimum(dm.abs(), dp.abs())
    c = sg * torch.minimum(torch.clamp(sg * y, min=0.0), lim)
    return torch.where(dm * dp > 0, c, torch.zeros_like(c))


def a_priori(params, x, t):
    """Mean squared error, in normalised slope units, of the clamped network,
    of the monotonized-central limiter and of minmod against the sub-cell
    target slopes of the samples."""
    import torch

    tr = hydro.Trainer(params, device=str(x.device))
    y = torch.empty_like(t)
    chunk = 1 << 22
    for i in range(0, x.shape[0], chunk):
        y[i:i + chunk] = tr.eval(x[i:i + chunk].contiguous())
    tr.close()
    net = tvd_clamp_normalised(x, y)
    mc = mc_normalised(x)
    dm, dp = x[:, 1], x[:, 2]
    mm = torch.where(dm * dp > 0, torch.sign(dp) * torch.minimum(dm.abs(), dp.abs()), torch.zeros_like(dp))
    return {
        "mse_learned": float(torch.mean((net - t) ** 2)),
        "mse_mc": float(torch.mean((mc - t) ** 2)),
        "mse_minmod": float(torch.mean((mm - t) ** 2)),
        "samples": int(x.shape[0]),
    }


TRAIN_RUNS = ((1207, 0.0), (1208, 0.0), (1209, 0.0), (1207, 0.01), (1208, 0.05))
EVAL_WIDTH = 0.025


def train_limiter(n_fine: int = 8192, runs=TRAIN_RUNS, times=(0.25, 0.5, 1.0),
                  steps: int = 40000, batch: int = 65536, lr: float = 1e-3, log=print):
    """Runs are (seed, shear-layer half-width) pairs; the held-out validation
    run is the sharp setup with another seed."""
    t0 = time.perf_counter()
    x, t = training_set(n_fine, runs, times, log=log)
    x, t = limiter.augment(x, t)
    log(f"training samples: {x.shape[0]} from {len(runs)} runs at {n_fine}^2 ({time.perf_counter() - t0:.1f} s)")
    t1 = time.perf_counter()
    params, losses = limiter.train(x, t, steps=steps, batch=batch, lr=lr, log_every=max(steps // 20, 1), log=log,
                                   cosine=True)
    log(f"trained {steps} steps in {time.perf_counter() - t1:.1f} s; loss {losses[0][1]:.4g} -> {losses[-1][1]:.4g}")
    del x, t
    xv, tv = training_set(n_fine, ((HELD_OUT_SEED, 0.0),), times, log=log)
    val = a_priori(params, xv, tv)
    log(f"held-out seed {HELD_OUT_SEED}: " + json.dumps(val))
    info = {"n_fine": n_fine, "runs": [list(r) for r in runs], "times": list(times), "steps": steps,
            "batch": batch, "lr": lr, "schedule": "cosine", "losses": losses, "validation": val}
    return params, info


# ---------------------------------------------------------------------------
# evaluation


def restrict(a: np.ndarray, n: int) -> np.ndarray:
    """Block average of a 1D or 2D field onto n cells per dimension."""
    r = a.shape[-1] // n
    if a.ndim == 1:
        return a.reshape(n, r).mean(axis=1)
    return a.reshape(n, r, n, r).mean(axis=(1, 3))


def run_to_times(prob, times, params=None, cfl: float = None, chunk: int = 64, diag=None, progress=None):
    """Density at each requested time (plain limiter if params is None),
    with the wall time of the whole run.  With a dict ``diag`` (2D), also
    E_kin,y at each time (diag["ekin_y"]) and the kinetic-energy spectrum at
    the last time (diag["spectrum"] = (k, e)); their cost is outside the wall
    time.  ``progress`` (a callable) hears the simulation time every ~10 s."""
    import torch

    cfl = prob.cfl if cfl is None else cfl
    lim = hydro.LIM_LEARNED if params is not None else hydro.LIM_THETA
    p = hydro.Patch(prob, precision=32, limiter=lim, set_initial=params is None)
    if params is not None:
        p.set_mlp(params)
        p.set_state(prob.W)
    out = {}
    wall = 0.0
    last = time.perf_counter()
    for T in times:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while p.time() < T * (1 - 1e-12):
            p.advance(chunk, cfl, t_end=T, solver=hydro.HLLC)
            if progress is not None and time.perf_counter() - last > 10.0:
                last = time.perf_counter()
                progress(f"{prob.name} {prob.n[0]}: t = {p.time():.4f}")
        U = p.get_state(hydro.CONSERVED)
        wall += time.perf_counter() - t0
        shape = (prob.n[1], prob.n[0]) if prob.ndim == 2 else (prob.n[0],)
        out[T] = U[0].reshape(shape).copy()
        if diag is not None:
            diag.setdefault("ekin_y", []).append(float(p.kinetic_energy()[1]))
            if T == times[-1]:
                diag["spectrum"] = diagnostics.kinetic_spectrum(p)
    p.close()
    return out, wall


def loglog_resolution(ns, errs, target):
    """Resolution at which the piecewise log-log interpolant of (ns, errs)
    reaches target (extrapolated from the end segments if outside)."""
    ln, le = np.log(np.asarray(ns, float)), np.log(np.asarray(errs, float))
    lt = math.log(target)
    for i in range(len(ns) - 1):
        lo, hi = sorted((le[i], le[i + 1]))
        if lo <= lt <= hi:
            break
    else:
        i = 0 if lt > le[0] else len(ns) - 2
    slope = (le[i + 1] - le[i]) / (ln[i + 1] - ln[i])
    if slope == 0:
        return float("nan")
    return float(math.exp(ln[i] + (lt - le[i]) / slope))


def spectral_error(k, e, kr, er, n, level: float = 1e-9):
    """Mean |ln(e / e_ref)| over the shells 1 .. n/4 (the well-resolved part of
    an n-cell run's spectrum) on which the reference carries more than
    ``level`` (below it the reference spectrum is roundoff)."""
    m = max(1, n // 4)
    keep = np.nonzero(er[1:m + 1] > level)[0] + 1
    if keep.size == 0:
        return float("nan")
    return float(np.mean(np.abs(np.log(e[keep] / er[keep]))))


def ladder(name, make, ns, n_ref, times, params, log=print, diagnose=False, progress=None):
    """L1 of plain and learned runs at each N against the restricted fine plain
    run; with ``diagnose`` (2D) also E_kin,y(t) of every run and the kinetic
    energy spectra at the last time (Sec. 4.3.1's yardsticks)."""
    dref = {} if diagnose else None
    ref, ref_wall = run_to_times(make(n_ref), times, diag=dref, progress=progress)
    log(f"{name}: reference {n_ref} in {ref_wall:.1f} s")
    rows = []
    spectra = {}
    for n in ns:
        dp = {} if diagnose else None
        dl = {} if diagnose else None
        pl, wp = run_to_times(make(n), times, diag=dp, progress=progress)
        le, wlr = run_to_times(make(n), times, params=params, diag=dl, progress=progress)
        if diagnose:
            kr, er = dref["spectrum"]
            spectra[n] = {
                "spectral_error_plain": spectral_error(*dp["spectrum"], kr, er, n),
                "spectral_error_learned": spectral_error(*dl["spectrum"], kr, er, n),
                "cutoff_1e-9_plain": diagnostics.spectral_cutoff(*dp["spectrum"], 1e-9),
                "cutoff_1e-9_learned": diagnostics.spectral_cutoff(*dl["spectrum"], 1e-9)}
        for i, T in enumerate(times):
            r = restrict(ref[T], n)
            row = {"n": n, "t": T, "l1_plain": float(np.mean(np.abs(pl[T] - r))),
                   "l1_learned": float(np.mean(np.abs(le[T] - r))), "wall_plain": wp, "wall_learned": wlr}
            if diagnose:
                row.update({"ekin_y_plain": dp["ekin_y"][i], "ekin_y_learned": dl["ekin_y"][i],
                            "ekin_y_reference": dref["ekin_y"][i]})
            rows.append(row)
        log(f"{name}: N={n} " + " ".join(f"t={r['t']}: plain {r['l1_plain']:.3e} learned {r['l1_learned']:.3e}"
                                             for r in rows[-len(times):]))
    matched = []
    for T in times:
        sub = [r for r in rows if r["t"] == T]
        nsub = [r["n"] for r in sub]
        lp = [r["l1_plain"] for r in sub]
        for r in sub:
            n_eq = loglog_resolution(nsub, lp, r["l1_learned"])
            matched.append({"t": T, "n_learned": r["n"], "l1_learned": r["l1_learned"],
                            "plain_n_for_same_l1": n_eq, "resolution_gain": n_eq / r["n"]})
    out = {"problem": name, "n_ref": n_ref, "times": list(times), "rows": rows, "matched": matched}
    if diagnose:
        out["spectra_at_last_time"] = {str(n): v for n, v in spectra.items()}
        out["cutoff_1e-9_reference"] = diagnostics.spectral_cutoff(*dref["spectrum"], 1e-9)
    return out


def evaluate(params, kh_ns=(128, 256, 512, 1024), kh_ref=4096, kh_times=(0.5, 1.0, 1.5), seed=HELD_OUT_SEED,
             log=print):
    """Ladders on the well-posed KH variant (tanh shear layers of half-width
    0.025, single-mode perturbation, a width no training run used), the Sod
    tube and the smooth density wave."""
    res = {"kelvin_helmholtz": ladder("kelvin_helmholtz",
                                      lambda n: wl.kelvin_helmholtz(n, seed=seed, width=EVAL_WIDTH, random_amp=0.0),
                                      kh_ns, kh_ref, kh_times, params, log, diagnose=True)}
    res["sod"] = ladder("sod", lambda n: wl.sod(n, theta=2.0, cfl=0.4, t_end=0.2), (128, 256, 512, 1024),
                        16384, (0.2,), params, log)
    res["advection_1d"] = ladder("advection_1d", lambda n: wl.advection_1d(n, theta=2.0),
                                 (32, 64, 128, 256), 8192, (1.0,), params, log)
    return res


def c3(params, ns=(512, 1024, 2048), n_ref=8192, T=1.5, log=print):
    """The Kelvin-Helmholtz comparison at its full size: plain and learned
    runs at 2048^2 (and 512^2, 1024^2 for the matched-L1 reading) to t = 1.5
    against a plain 8192^2 run restricted to each N, for the sharp shear
    layers of the Sec. 4.3.1 setup (seed 1207; no convergence in N is
    expected there, so E_kin,y and the spectrum are the yardsticks) and for
    the smooth-layer variant of the ladders above.  Records L1, E_kin,y at
    t = 0.5, 1, 1.5, the spectral error at t = 1.5, the wall times, and the
    time the learned run takes over the time the plain method needs for the
    same L1 (a 2D run costs N^3)."""
    out = {}
    times = (0.5, 1.0, T)
    for key, make in (("sharp_layers", lambda n: wl.kelvin_helmholtz(n, seed=1207)),
                      ("smooth_layers", lambda n: wl.kelvin_helmholtz(n, seed=HELD_OUT_SEED, width=EVAL_WIDTH,
                                                                       random_amp=0.0))):
        r = ladder(key, make, ns, n_ref, times, params, log=log, diagnose=True, progress=log)
        last = [x for x in r["rows"] if x["t"] == T]
        wall = {x["n"]: (x["wall_plain"], x["wall_learned"]) for x in last}
        for m in r["matched"]:
            if m["t"] != T:
                continue
            n = m["n_learned"]
            n_eq = m["plain_n_for_same_l1"]
            # plain wall time at the resolution with the same L1, from the
            # measured plain wall time at N scaled as N^3
            if n_eq == n_eq:
                m["time_ratio_learned_over_plain"] = wall[n][1] / (wall[n][0] * (n_eq / n) ** 3)
        out[key] = r
        log(f"{key}: " + json.dumps([{k: v for k, v in m.items()} for m in r["matched"] if m["t"] == T]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-fine", type=int, default=8192)
    t.add_argument("--runs", default=",".join(f"{s}:{w}" for s, w in TRAIN_RUNS),
                   help="seed:width pairs of the training runs")
    t.add_argument("--times", default="0.25,0.5,1.0")
    t.add_argument("--steps", type=int, default=40000)
    t.add_argument("--batch", type=int, default=65536)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True, help="weights (.npy, float32, 1249 values)")
    t.add_argument("--json", default="", help="training record")
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--kh-ns", default="128,256,512,1024")
    e.add_argument("--kh-ref", type=int, default=4096)
    e.add_argument("--json", default="")
    c = sub.add_parser("c3", help="the 2048^2 Kelvin-Helmholtz comparison to t = 1.5 against 8192^2")
    c.add_argument("--weights", default="", help="weights (.npy); default: the shipped network")
    c.add_argument("--n-ref", type=int, default=8192)
    c.add_argument("--ns", default="512,1024,2048")
    c.add_argument("--json", default="")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if a.cmd == "train":
        runs = tuple((int(r.split(":")[0]), float(r.split(":")[1])) for r in a.runs.split(","))
        params, info = train_limiter(a.n_fine, runs,
                                     tuple(float(s) for s in a.times.split(",")), a.steps, a.batch, a.lr, log)
        np.save(a.out, params.astype(np.float32))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(info, f, indent=1)
    elif a.cmd == "c3":
        params = (np.load(a.weights, allow_pickle=False).astype(np.float32) if a.weights
                  else limiter.trained_params())
        res = c3(params, tuple(int(s) for s in a.ns.split(",")), a.n_ref, log=log)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
    else:
        params = np.load(a.weights, allow_pickle=False).astype(np.float32)
        res = evaluate(params, tuple(int(s) for s in a.kh_ns.split(",")), a.kh_ref, log=log)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
