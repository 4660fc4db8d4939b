"""FP64 statement of the learned limiter's training data (test infrastructure).

TEST INFRASTRUCTURE ONLY.  From a fine conserved state on a periodic grid:
restriction to a grid 4x coarser by averaging the conserved variables over
each coarse cell (the averaging step of restriction, Sec. 2), primitives of
those averages; for each (dimension q, variable v, coarse cell) the inputs are
the four one-sided differences of the coarse 5-cell stencil along q over
s = max|d| + 1e-12 (|w_c| + 1e-30), and the target is the least-squares slope
of the four quarter-slab averages (conserved averages over the slab, then
primitives) at positions -3/8, -1/8, 1/8, 3/8, clamped to the TVD region and
divided by s.  Sample order: (q * nv + v) * ncoarse + coarse cell.
"""
from __future__ import annotations

import numpy as np

from .mlp import tvd_clamp


def _prim(U, ndim, gamma):
    rho = U[0]
    v = U[1:1 + ndim] / rho
    p = (gamma - 1.0) * (U[ndim + 1] - 0.5 * np.sum(U[1:1 + ndim] * v, axis=0))
    return np.concatenate([rho[None], v, p[None]], axis=0)


def samples(U, ndim, n, gamma, return_scale=False):
    """U: (nv, ncell) FP64 conserved fine state; n: fine cells per dim (x, y, z).
    Returns x (ns, 4), t (ns) and, with return_scale, also s (ns) and the
    stencil centre value w_c (ns)."""
    nv = ndim + 2
    shape = tuple(int(n[q]) for q in reversed(range(ndim)))  # (nz, ny, nx) active
    Uf = np.asarray(U, dtype=np.float64).reshape((nv,) + shape)
    # block views: axis order per variable is (z, y, x) -> (cz, 4, cy, 4, cx, 4)
    blk = []
    for q in reversed(range(ndim)):
        blk += [shape[ndim - 1 - q] // 4, 4]
    Ub = Uf.reshape((nv,) + tuple(blk))
    sub_axes = tuple(2 + 2 * i for i in range(ndim))  # the "4" axes
    Uc = Ub.mean(axis=sub_axes)
    Wc = _prim(Uc.reshape(nv, -1), ndim, gamma).reshape(Uc.shape)
    nc = Wc[0].size
    xs, ts, ss, ws = [], [], [], []
    for q in range(ndim):
        ax = ndim - 1 - q  # array axis of dimension q in the coarse field
        sub_ax = 2 + 2 * ax
        others = tuple(a for a in sub_axes if a != sub_ax)
        slabs = Ub.mean(axis=others)  # (nv, ..., 4 along q, ...)
        # move the q sub-axis to the end
        slabs = np.moveaxis(slabs, 1 + 2 * ax + 1 - sum(1 for a in others if a < sub_ax), -1)
        Ws = _prim(slabs.reshape(nv, -1), ndim, gamma).reshape(slabs.shape)
        for v in range(nv):
            w = Wc[v]
            st = np.stack([np.roll(w, 2 - k, axis=ax) for k in range(5)], axis=0)  # cells c-2 .. c+2
            d = np.diff(st, axis=0)
            s = np.max(np.abs(d), axis=0) + 1e-12 * (np.abs(w) + 1e-30)
            xs.append(np.stack([(d[k] / s).ravel() for k in range(4)], axis=1))
            ss.append(s.ravel())
            ws.append(w.ravel())
            wsub = Ws[v]
            target = 0.4 * (-3 * wsub[..., 0] - wsub[..., 1] + wsub[..., 2] + 3 * wsub[..., 3])
            tc = tvd_clamp(target, d[1], d[2])
            ts.append((tc / s).ravel())
    if return_scale:
        return (np.concatenate(xs, axis=0), np.concatenate(ts, axis=0), np.concatenate(ss), np.concatenate(ws))
    return np.concatenate(xs, axis=0), np.concatenate(ts, axis=0)
