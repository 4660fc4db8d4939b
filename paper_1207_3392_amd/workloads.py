"""Seeded synthetic inputs shared by the GPU path, the oracle, tests and the bench.

Every generator returns *primitive* fields only (mass density, velocity
components, pressure) as float64 NumPy arrays, plus the patch description the
problem needs.  Nothing here performs any arithmetic of the numerical method
(no equation of state, no conserved variables, no fluxes): the two
implementations each convert primitives themselves.

Field layout: ``W`` has shape ``(nv, nz, ny, nx)`` squeezed to the active
dimensions, i.e. ``(nv, nx)`` in 1D, ``(nv, ny, nx)`` in 2D and
``(nv, nz, ny, nx)`` in 3D, x fastest.  The primitive order is
``rho, v_x[, v_y[, v_z]], p`` (``nv = ndim + 2``).

Initial conditions are point values at cell centres (the paper's tests are
specified pointwise; Sec. 4).  Random numbers come from NumPy's PCG64 with an
explicit seed (default 1207).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

DEFAULT_SEED = 1207

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
HLL, HLLC = 0, 1
LIM_THETA, LIM_LEARNED = 0, 1


@dataclasses.dataclass
class Problem:
    """A patch description plus its initial primitive fields."""

    ndim: int
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    gamma: float
    bc: Tuple[Tuple[int, int], Tuple[int, int], Tuple[int, int]]
    W: np.ndarray
    theta: float = 2.0
    cfl: float = 0.4
    t_end: float = 0.0
    accel: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    name: str = ""

    @property
    def ncell(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nv(self) -> int:
        return self.ndim + 2

    def flat(self) -> np.ndarray:
        """Primitive fields as a contiguous ``(nv, ncell)`` float64 array."""
        return np.ascontiguousarray(self.W.reshape(self.nv, -1), dtype=np.float64)


def _cell_centres(n: int, lo: float, hi: float) -> np.ndarray:
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx


def _pad3(v, fill):
    v = list(v)
    while len(v) < 3:
        v.append(fill)
    return tuple(v)


def riemann_tube(n: int, left, right, x0: float = 0.5, gamma: float = 1.4,
                 lo: float = 0.0, hi: float = 1.0, bc=BC_OUTFLOW, theta: float = 2.0,
                 cfl: float = 0.4, t_end: float = 0.2, name: str = "riemann") -> Problem:
    """1D Riemann problem: ``left``/``right`` are (rho, v, p); cells whose centre
    lies left of ``x0`` take the left state."""
    x = _cell_centres(n, lo, hi)
    W = np.empty((3, n))
    m = x < x0
    for k in range(3):
        W[k] = np.where(m, left[k], right[k])
    return Problem(1, (n, 1, 1), (lo, 0.0, 0.0), (hi, 1.0, 1.0), gamma,
                   ((bc, bc), (BC_PERIODIC, BC_PERIODIC), (BC_PERIODIC, BC_PERIODIC)),
                   W, theta=theta, cfl=cfl, t_end=t_end, name=name)


SOD_LEFT = (1.0, 0.0, 1.0)
SOD_RIGHT = (0.125, 0.0, 0.1)          # standard Sod right state
SOD_RIGHT_AS_PRINTED = (0.1, 0.0, 0.125)  # right state as printed in the paper's Sod setup (Sec. 4.2.1)


def sod(n: int = 400, theta: float = 1.0, cfl: float = 0.4, t_end: float = 0.2,
        as_printed: bool = False) -> Problem:
    """Sod shock tube on [0,1], interface at x=0.5, gamma=1.4, outflow ends."""
    right = SOD_RIGHT_AS_PRINTED if as_printed else SOD_RIGHT
    return riemann_tube(n, SOD_LEFT, right, 0.5, 1.4, theta=theta, cfl=cfl, t_end=t_end, name="sod")


def contact(n: int = 128, vc: float = 0.0, t_end: float = 2.0) -> Problem:
    """Isolated contact (Sec. 4.2.1): [1.4, vc, 1] | [1.0, vc, 1]."""
    return riemann_tube(n, (1.4, vc, 1.0), (1.0, vc, 1.0), 0.5, 1.4, theta=1.4, cfl=0.5,
                        t_end=t_end, name="contact")


def double_rarefaction(n: int = 128) -> Problem:
    """Einfeldt 1-2-0-3 (Sec. 4.2.1): [1,-2,0.4] | [1,2,0.4] to t=0.15."""
    return riemann_tube(n, (1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.5, 1.4, theta=1.4, cfl=0.5,
                        t_end=0.15, name="double_rarefaction")


def blast_waves(n: int = 400) -> Problem:
    """Interacting blast waves (Sec. 4.2.2): reflecting [0,1], rho=1 at rest,
    p=1000 for x<0.1, 100 for x>0.9, 0.01 elsewhere."""
    x = _cell_centres(n, 0.0, 1.0)
    W = np.empty((3, n))
    W[0] = 1.0
    W[1] = 0.0
    W[2] = np.where(x < 0.1, 1000.0, np.where(x > 0.9, 100.0, 0.01))
    return Problem(1, (n, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 1.4,
                   ((BC_REFLECT, BC_REFLECT), (0, 0), (0, 0)), W, theta=1.4, cfl=0.5,
                   t_end=0.038, name="blast_waves")


def advection_1d(n: int, mach: float = 0.6, t_end: float = 1.0, theta: float = 1.4) -> Problem:
    """1D density-wave advection (Sec. 4.1.1): rho=1+0.1 sin(2 pi x), v=1,
    p = rho0 v^2/(gamma Ma^2), periodic [0,1], gamma=1.4."""
    x = _cell_centres(n, 0.0, 1.0)
    gamma = 1.4
    W = np.empty((3, n))
    W[0] = 1.0 + 0.1 * np.sin(2 * np.pi * x)
    W[1] = 1.0
    W[2] = 1.0 * 1.0 / (gamma * mach * mach)
    return Problem(1, (n, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), gamma,
                   ((0, 0), (0, 0), (0, 0)), W, theta=theta, cfl=0.5, t_end=t_end,
                   name="advection_1d")


def advection_2d(n: int, mach: float = 0.6, t_end: float = 1.0, theta: float = 1.4) -> Problem:
    """Oblique 2D advection (Sec. 4.1.1): Lx = 2 Ly, Ly = sqrt(5)/2, n x n cells,
    wave along (1/Lx, 1/Ly), returns to its start at t=1."""
    ly = math.sqrt(5.0) / 2.0
    lx = 2.0 * ly
    gamma = 1.4
    x = _cell_centres(n, 0.0, lx)
    y = _cell_centres(n, 0.0, ly)
    X, Y = np.meshgrid(x, y)  # shape (ny, nx)
    norm = math.sqrt(lx ** -2 + ly ** -2)
    W = np.empty((4, n, n))
    W[0] = 1.0 + 0.1 * np.sin(2 * np.pi * (X / lx + Y / ly))
    W[1] = (1.0 / lx) / norm
    W[2] = (1.0 / ly) / norm
    W[3] = 1.0 / (gamma * mach * mach)
    return Problem(2, (n, n, 1), (0.0, 0.0, 0.0), (lx, ly, 1.0), gamma,
                   ((0, 0), (0, 0), (0, 0)), W, theta=theta, cfl=0.5, t_end=t_end,
                   name="advection_2d")


def linear_wave(n: int, kind: str = "sound", amp: float = 1e-6) -> Problem:
    """Linear sound / shear waves (Sec. 4.1.2), 1D periodic [0,1], rho0=1,
    p0=3/5, gamma=5/3 (c0=1).  The sound wave is a 1D problem.  The shear
    wave carries v_y and v_z, so it is posed on an n x 2 x 2 periodic 3D patch
    whose fields are constant across y and z."""
    gamma = 5.0 / 3.0
    x = _cell_centres(n, 0.0, 1.0)
    s = np.sin(2 * np.pi * x)
    if kind == "sound":
        W = np.empty((3, n))
        W[0] = 1.0 + amp * 1.0 * s
        W[1] = 0.0 + amp * 1.0 * s
        W[2] = 0.6 + amp * 1.0 * s
        return Problem(1, (n, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), gamma,
                       ((0, 0), (0, 0), (0, 0)), W, theta=1.4, cfl=0.5, t_end=1.0,
                       name="sound_wave")
    if kind == "shear":
        W = np.empty((5, 2, 2, n))
        W[0] = 1.0
        W[1] = 0.5
        W[2] = amp * s
        W[3] = amp * s
        W[4] = 0.6
        return Problem(3, (n, 2, 2), (0.0, 0.0, 0.0), (1.0, 2.0 / n, 2.0 / n), gamma,
                       ((0, 0), (0, 0), (0, 0)), W, theta=1.4, cfl=0.3, t_end=2.0,
                       name="shear_wave")
    raise ValueError(kind)


def implosion(n: int = 64) -> Problem:
    """2D implosion (Sec. 4.2.1): [0,0.3]^2, reflecting walls, rho=0.125,
    p=0.14 where x+y<=0.15 (cell centres), else 1, 1; fluid at rest."""
    x = _cell_centres(n, 0.0, 0.3)
    X, Y = np.meshgrid(x, x)
    inner = (X + Y) <= 0.15
    W = np.zeros((4, n, n))
    W[0] = np.where(inner, 0.125, 1.0)
    W[3] = np.where(inner, 0.14, 1.0)
    return Problem(2, (n, n, 1), (0.0, 0.0, 0.0), (0.3, 0.3, 1.0), 1.4,
                   ((2, 2), (2, 2), (0, 0)), W, theta=1.4, cfl=0.5, t_end=0.045,
                   name="implosion")


def planar_shock(nx: int = 200, ny: int = 20, mach: float = 6.0, gamma: float = 1.4, x0: float = 0.1,
                 amp: float = 1e-3, ndim: int = 2) -> Problem:
    """A grid-aligned shock of Mach number ``mach`` moving along +x into gas at
    rest (rho = 1, p = 1/gamma, so c = 1), the post-shock state behind it from
    the Rankine-Hugoniot relations, in a channel [0, 1] x [0, ny/nx] (and the
    same depth in z for ndim = 3): outflow at both x ends (the inflow behind
    the shock is supersonic), reflecting side walls.  The pre-shock density of
    the middle row of cells is raised by the relative amount ``amp``, the seed
    of odd-even decoupling (Sec. 3.2)."""
    r1, p1 = 1.0, 1.0 / gamma
    m2 = mach * mach
    r2 = r1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    u2 = mach * (1.0 - r1 / r2)  # shock speed mach * c1 = mach
    x = _cell_centres(nx, 0.0, 1.0)
    nz = ny if ndim == 3 else 1
    post = np.broadcast_to(x[None, None, :] < x0, (nz, ny, nx))
    nv = ndim + 2
    W = np.zeros((nv, nz, ny, nx))
    W[0] = np.where(post, r2, r1)
    W[1] = np.where(post, u2, 0.0)
    W[nv - 1] = np.where(post, p2, p1)
    W[0][:, ny // 2, :] *= np.where(post[0, 0], 1.0, 1.0 + amp)
    depth = ny / nx
    bc = ((BC_OUTFLOW, BC_OUTFLOW), (BC_REFLECT, BC_REFLECT),
          (BC_REFLECT, BC_REFLECT) if ndim == 3 else (BC_PERIODIC, BC_PERIODIC))
    if ndim == 2:
        W = W[:, 0]
    return Problem(ndim, (nx, ny, nz), (0.0, 0.0, 0.0), (1.0, depth, depth if ndim == 3 else 1.0), gamma,
                   bc, W, theta=2.0, cfl=0.4, t_end=0.1, name="planar_shock")


def _mode_set(dim: int, kmax: int = 4) -> np.ndarray:
    """All integer wave vectors k with 1 <= |k| <= kmax in ``dim`` dimensions."""
    r = range(-kmax, kmax + 1)
    if dim == 3:
        ks = [(a, b, c) for a in r for b in r for c in r]
    else:
        ks = [(a, b) for a in r for b in r]
    ks = [k for k in ks if 1 <= math.sqrt(sum(q * q for q in k)) <= kmax]
    return np.array(ks, dtype=np.float64)


def smooth_periodic_3d(n: int = 256, seed: int = DEFAULT_SEED, ny: int = None, nz: int = None,
                       gamma: float = 5.0 / 3.0, cfl: float = 0.4) -> Problem:
    """3D periodic smooth flow on the unit cube: rho = 1 + 0.2 * mean of 8
    random-phase Fourier modes with 1 <= |k| <= 4, p = 1, each velocity
    component 0.1 * mean of its own 8 random modes; gamma = 5/3.

    The sums are separable per mode, evaluated as outer products so that a
    512^3 field is generated in seconds.  ``ny``/``nz`` allow non-cubic
    patches with the same physical unit cube."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = _mode_set(3)
    x = _cell_centres(n, 0.0, 1.0)
    y = _cell_centres(ny, 0.0, 1.0)
    z = _cell_centres(nz, 0.0, 1.0)

    def field(amp):
        idx = rng.choice(len(modes), size=8, replace=False)
        ph = rng.uniform(0.0, 2 * np.pi, size=8)
        out = np.zeros((nz, ny, n))
        for j in range(8):
            k = modes[idx[j]]
            # cos(a+b+c+phi) expanded via complex exponentials (separable)
            ex = np.exp(1j * (2 * np.pi * k[0] * x))
            ey = np.exp(1j * (2 * np.pi * k[1] * y))
            ez = np.exp(1j * (2 * np.pi * k[2] * z + ph[j]))
            out += np.real(ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
        return amp * out / 8.0

    W = np.empty((5, nz, ny, n))
    W[0] = 1.0 + field(0.2)
    W[1] = field(0.1)
    W[2] = field(0.1)
    W[3] = field(0.1)
    W[4] = 1.0
    return Problem(3, (n, ny, nz), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), gamma,
                   ((0, 0), (0, 0), (0, 0)), W, theta=2.0, cfl=cfl, name="smooth_periodic_3d")


def kelvin_helmholtz(n: int = 2048, seed: int = DEFAULT_SEED, gamma: float = 5.0 / 3.0,
                     random_amp: float = 1e-3, lattice: int = 64, width: float = 0.0) -> Problem:
    """2D Kelvin-Helmholtz on the periodic unit square (Sec. 4.3.1 setup):
    p = 2.5; rho = 2, v_x = +0.5 for |y-0.5| < 0.25, else rho = 1, v_x = -0.5;
    v_y = [0.01 sin(2 pi x) + A_R(x, y)] psi(y) with
    psi = exp(-0.5 (cos(2 pi y) / (2 pi 0.1))^2).

    The random part A_R is uniform in [-random_amp, random_amp] on a fixed
    ``lattice x lattice`` grid (seeded) and sampled piecewise-constantly, so
    every resolution sees the same initial condition.

    width = 0 gives the paper's sharp shear layers, whose growth rate rises
    without bound with the wavenumber, so runs at different resolutions do not
    converge to one solution.  width > 0 replaces the steps in rho and v_x by
    tanh profiles of that half-width, e.g. rho = 1 + [tanh((y - 0.25)/width)
    - tanh((y - 0.75)/width)] / 2, a well-posed variant for convergence
    studies."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lat = rng.uniform(-random_amp, random_amp, size=(lattice, lattice))
    x = _cell_centres(n, 0.0, 1.0)
    y = _cell_centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    if width > 0.0:
        inner = 0.5 * (np.tanh((Y - 0.25) / width) - np.tanh((Y - 0.75) / width))
    else:
        inner = (np.abs(Y - 0.5) < 0.25).astype(np.float64)
    ix = np.minimum((x * lattice).astype(np.int64), lattice - 1)
    iy = np.minimum((y * lattice).astype(np.int64), lattice - 1)
    AR = lat[iy[:, None], ix[None, :]]
    psi = np.exp(-0.5 * (np.cos(2 * np.pi * Y) / (2 * np.pi * 0.1)) ** 2)
    W = np.empty((4, n, n))
    W[0] = 1.0 + inner
    W[1] = -0.5 + inner
    W[2] = (0.01 * np.sin(2 * np.pi * X) + AR) * psi
    W[3] = 2.5
    return Problem(2, (n, n, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), gamma,
                   ((0, 0), (0, 0), (0, 0)), W, theta=2.0, cfl=0.4, t_end=1.5,
                   name="kelvin_helmholtz")


def rayleigh_taylor_3d(n: int = 512, seed: int = DEFAULT_SEED, g: float = 0.1,
                       gamma: float = 1.4, amp: float = 0.01) -> Problem:
    """3D Rayleigh-Taylor on [-0.5,0.5]^3: periodic x, y; reflecting z;
    rho = 2 for z > 0 else 1; p = 2.5 - rho g z (hydrostatic for a = -g z_hat);
    v_z = amp * mean_j cos(2 pi (kx x + ky y) + phi_j) * (1 + cos 2 pi z)/2 with 8
    seeded modes 1 <= |k| <= 4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = _mode_set(2)
    idx = rng.choice(len(modes), size=8, replace=False)
    ph = rng.uniform(0.0, 2 * np.pi, size=8)
    c = _cell_centres(n, -0.5, 0.5)
    z = c[:, None, None]
    y = c[None, :, None]
    x = c[None, None, :]
    W = np.empty((5, n, n, n))
    rho = np.where(z > 0, 2.0, 1.0) * np.ones((n, n, n))
    W[0] = rho
    W[1] = 0.0
    W[2] = 0.0
    pert = np.zeros((1, n, n))
    for j in range(8):
        k = modes[idx[j]]
        pert = pert + np.cos(2 * np.pi * (k[0] * x + k[1] * y) + ph[j])
    W[3] = amp * (pert / 8.0) * 0.5 * (1.0 + np.cos(2 * np.pi * z))
    W[4] = 2.5 - rho * g * z
    return Problem(3, (n, n, n), (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5), gamma,
                   ((0, 0), (0, 0), (2, 2)), W, theta=2.0, cfl=0.3,
                   accel=(0.0, 0.0, -g), name="rayleigh_taylor_3d")


@dataclasses.dataclass
class Tube:
    n: int
    left: Tuple[float, float, float]
    right: Tuple[float, float, float]
    x0: float


def batched_tubes(count: int = 512, seed: int = DEFAULT_SEED, nmin: int = 128,
                  nmax: int = 4096) -> List[Tube]:
    """Independent 1D Riemann problems: N ~ U{nmin..nmax}; rho, p log-uniform
    in [0.1, 10]; v uniform in [-1, 1]; interface at the cell face nearest 0.5
    (x0 = floor(N/2)/N)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        rl, rr = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=2))
        pl, pr = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=2))
        vl, vr = rng.uniform(-1.0, 1.0, size=2)
        out.append(Tube(n, (float(rl), float(vl), float(pl)), (float(rr), float(vr), float(pr)),
                        (n // 2) / n))
    return out


def tube_problem(t: Tube, gamma: float = 1.4, theta: float = 2.0, cfl: float = 0.4,
                 t_end: float = 0.1) -> Problem:
    return riemann_tube(t.n, t.left, t.right, t.x0, gamma, theta=theta, cfl=cfl,
                        t_end=t_end, name="tube")


def random_states(count: int, seed: int = DEFAULT_SEED, ndim: int = 3,
                  vmax: float = 2.0) -> np.ndarray:
    """Random primitive states (rho, v[ndim], p) with rho, p log-uniform in
    [0.1, 10] and velocities uniform in [-vmax, vmax]; shape (ndim+2, count)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = np.empty((ndim + 2, count))
    W[0] = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=count))
    for d in range(ndim):
        W[1 + d] = rng.uniform(-vmax, vmax, size=count)
    W[ndim + 1] = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=count))
    return W


def random_smooth_patch(ndim: int, n: Sequence[int], seed: int = DEFAULT_SEED,
                        bc=BC_PERIODIC, amp: float = 0.2, gamma: float = 1.4,
                        theta: float = 2.0) -> Problem:
    """A small random patch for parity tests: smooth background plus a random
    per-cell perturbation of relative size ``amp`` (so limiters are exercised),
    on the unit box with the given boundary kind on every face."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n3 = _pad3(list(n), 1)
    shape = tuple(reversed(n3[:ndim]))
    W = np.empty((ndim + 2,) + shape)
    W[0] = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    for d in range(ndim):
        W[1 + d] = 0.5 * rng.uniform(-1, 1, size=shape)
    W[ndim + 1] = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    bcs = tuple((bc, bc) if q < ndim else (0, 0) for q in range(3))
    return Problem(ndim, n3, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), gamma, bcs, W,
                   theta=theta, name="random_smooth")


@dataclasses.dataclass
class Levels:
    """A nested multilevel configuration: ``base`` is level 0 (box, boundary
    kinds, its initial fields in ``base.W``); ``boxes[l - 1] = (lo, n)`` names
    the cells of level l - 1 that level l refines by two per active dimension
    (unused dimensions: lo 0, n 1); ``W[l]`` are level l's initial primitive
    fields, point values at its own cell centres."""

    base: Problem
    boxes: List[Tuple[Tuple[int, int, int], Tuple[int, int, int]]]
    W: List[np.ndarray]

    @property
    def nlev(self) -> int:
        return 1 + len(self.boxes)

    def level_geometry(self, l: int):
        """(n, lo, hi) of level l."""
        n = list(self.base.n)
        lo = list(self.base.lo)
        hi = list(self.base.hi)
        for k in range(1, l + 1):
            blo, bn = self.boxes[k - 1]
            for q in range(self.base.ndim):
                dq = (hi[q] - lo[q]) / n[q]
                lo[q] = lo[q] + blo[q] * dq
                hi[q] = lo[q] + bn[q] * dq
                n[q] = 2 * bn[q]
        return tuple(n), tuple(lo), tuple(hi)


def _nested_boxes(ndim: int, n0: int, nlev: int):
    """Each level covers the central half of its parent: box lo n/4, n/2."""
    boxes = []
    for _ in range(1, nlev):
        lo = tuple(n0 // 4 if q < ndim else 0 for q in range(3))
        n = tuple(n0 // 2 if q < ndim else 1 for q in range(3))
        boxes.append((lo, n))
    return boxes


def _level_fields(lv: Levels, fn) -> List[np.ndarray]:
    out = []
    for l in range(lv.nlev):
        n, lo, hi = lv.level_geometry(l)
        out.append(fn(n, lo, hi))
    return out


def sedov_levels(ndim: int = 2, n0: int = 64, nlev: int = 3, gamma: float = 1.4, rho0: float = 1.0,
                 p0: float = 1e-5, e_d: float = 1.0, r_cells: float = 3.5, sub: int = 20,
                 bc: int = BC_OUTFLOW, theta: float = 1.4, cfl: float = 0.4, boxes=None) -> Levels:
    """Sedov-Taylor blast (Sec. 4.2.3): fluid at rest, density rho0, pressure p0
    on [-0.5, 0.5]^d, with the energy e_d released as the pressure
    3 (gamma - 1) e_d / ((alpha + 1) pi R_d^alpha) inside r <= R_d (alpha = d;
    in 1D the slab |x| <= R_d holds e_d as (gamma - 1) e_d / (2 R_d)).  R_d is
    r_cells finest-level cells; every cell cut by the sphere takes the volume
    average of the pressure over a sub^d subgrid.  Levels: nested boxes, each
    the central half of its parent, n0 cells per dimension on every level, or
    the given ``boxes``.  theta = 1.4, the value the paper often uses."""
    lo3 = tuple(-0.5 if q < ndim else 0.0 for q in range(3))
    hi3 = tuple(0.5 if q < ndim else 1.0 for q in range(3))
    n3 = tuple(n0 if q < ndim else 1 for q in range(3))
    bcs = tuple((bc, bc) if q < ndim else (0, 0) for q in range(3))
    if boxes is not None:
        nlev = 1 + len(boxes)
    dx_fine = 1.0 / (n0 * 2 ** (nlev - 1))
    r_d = r_cells * dx_fine
    if ndim == 1:
        p_d = (gamma - 1.0) * e_d / (2.0 * r_d)
    else:
        p_d = 3.0 * (gamma - 1.0) * e_d / ((ndim + 1) * math.pi * r_d ** ndim)

    def fields(n, lo, hi):
        axes = [_cell_centres(n[q], lo[q], hi[q]) for q in range(ndim)]
        widths = [(hi[q] - lo[q]) / n[q] for q in range(ndim)]
        grids = np.meshgrid(*reversed(axes), indexing="ij")  # (z, y, x) order
        r = np.sqrt(sum(g ** 2 for g in grids))
        half_diag = 0.5 * math.sqrt(sum(w ** 2 for w in widths))
        frac = (r <= r_d).astype(np.float64)
        cut = np.abs(r - r_d) <= half_diag
        if np.any(cut):
            offs = (np.arange(sub) + 0.5) / sub - 0.5
            sg = np.meshgrid(*([offs] * ndim), indexing="ij")
            for idx in zip(*np.nonzero(cut)):
                rr2 = 0.0
                for a, g in enumerate(grids):
                    w = widths[ndim - 1 - a]
                    rr2 = rr2 + (g[idx] + sg[a] * w) ** 2
                frac[idx] = float(np.mean(np.sqrt(rr2) <= r_d))
        W = np.empty((ndim + 2,) + r.shape)
        W[0] = rho0
        W[1:ndim + 1] = 0.0
        W[ndim + 1] = p0 + (p_d - p0) * frac
        return W

    base = Problem(ndim, n3, lo3, hi3, gamma, bcs, None, theta=theta, cfl=cfl, name="sedov_levels")
    lv = Levels(base, _nested_boxes(ndim, n0, nlev) if boxes is None else list(boxes), [])
    lv.W = _level_fields(lv, fields)
    base.W = lv.W[0]
    return lv


def smooth_levels(ndim: int = 2, n0: int = 32, nlev: int = 2, seed: int = DEFAULT_SEED, amp: float = 0.2,
                  vel=(0.6, 0.3, 0.2), gamma: float = 1.4, theta: float = 2.0, cfl: float = 0.4,
                  uniform: bool = False, t: float = 0.0, boxes=None, n=None) -> Levels:
    """Periodic unit box with a smooth density wave (random phases, modes 1 and
    2 per dimension) carried by a uniform velocity at uniform pressure; with
    ``uniform`` the density is 1 everywhere.  ``t`` > 0 gives the exact
    solution at time t (the wave translated by vel * t).  Levels as in
    sedov_levels; ``n`` (cells per dimension of level 0) overrides n0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(ndim, 2))
    n3 = tuple((n0 if n is None else n[q]) if q < ndim else 1 for q in range(3))
    bcs = tuple((BC_PERIODIC, BC_PERIODIC) for _ in range(3))

    def fields(n, lo, hi):
        axes = [_cell_centres(n[q], lo[q], hi[q]) - vel[q] * t for q in range(ndim)]
        grids = list(reversed(np.meshgrid(*reversed(axes), indexing="ij")))  # grids[q] varies along q
        rho = np.ones(grids[0].shape)
        if not uniform:
            for q in range(ndim):
                rho = rho + amp / ndim * (np.sin(2 * math.pi * grids[q] + ph[q, 0])
                                          + 0.5 * np.sin(4 * math.pi * grids[q] + ph[q, 1]))
        W = np.empty((ndim + 2,) + rho.shape)
        W[0] = rho
        for q in range(ndim):
            W[1 + q] = vel[q]
        W[ndim + 1] = 1.0
        return W

    base = Problem(ndim, n3, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), gamma, bcs, None, theta=theta, cfl=cfl,
                   name="smooth_levels")
    lv = Levels(base, _nested_boxes(ndim, n0, nlev) if boxes is None else list(boxes), [])
    lv.W = _level_fields(lv, fields)
    base.W = lv.W[0]
    return lv
