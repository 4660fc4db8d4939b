"""FP64 CPU oracle for the finite-volume hydrodynamics hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it and shares no code with it.

The arithmetic lives in ``hydro_oracle.c`` (plain C, double precision); this
module only marshals NumPy arrays through ctypes, plus three plain helpers
written here in Python: exact conserved totals (``math.fsum``), the time
loop of Alg. 2 (single level) and the relative L1 norm of eq. L1ErrorNorm.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ESTATE = 0, -1, -4
HLL, HLLC, HLLC_SWITCH = 0, 1, 2
SHOCK_EPS = 0.5
LIM_THETA, LIM_LEARNED = 0, 1
MLP_IN, MLP_H = 4, 32
MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


class OracleError(RuntimeError):
    def __init__(self, status, what=""):
        super().__init__(f"oracle {what} returned status {status}")
        self.status = status


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no FP contraction; OpenMP over
    independent loops, bitwise the same result on any thread count)."""
    src = os.path.join(_HERE, "hydro_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fopenmp", "-Wall", "-shared", "-fPIC",
               "-o", LIB_PATH, src, "-lm"]
        subprocess.check_call(cmd)
    return LIB_PATH


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("bc", (ctypes.c_int * 2) * 3),
        ("solver", ctypes.c_int),
        ("limiter", ctypes.c_int),
        ("theta", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("mlp", ctypes.POINTER(ctypes.c_double)),
        ("mlp_bf16", ctypes.c_int),
        ("shock_fp32", ctypes.c_int),
    ]


FMR_MAXLEV = 8
NG = 2


class _FmrDesc(ctypes.Structure):
    _fields_ = [
        ("base", _Desc),
        ("nlev", ctypes.c_int),
        ("box_lo", (ctypes.c_int64 * 3) * FMR_MAXLEV),
        ("box_n", (ctypes.c_int64 * 3) * FMR_MAXLEV),
        ("no_reflux", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_Desc)
        dp = ctypes.POINTER(ctypes.c_double)
        for name, args, res in [
            ("orc_prim_to_cons", [P, dp, dp], ctypes.c_int),
            ("orc_cons_to_prim", [P, dp, dp], ctypes.c_int),
            ("orc_rhs", [P, dp, dp], ctypes.c_int),
            ("orc_step", [P, dp, ctypes.c_double], ctypes.c_int),
            ("orc_cfl_dt", [P, dp, ctypes.c_double, dp], ctypes.c_int),
            ("orc_limiter_theta", [ctypes.c_double, ctypes.c_double, ctypes.c_double], ctypes.c_double),
            ("orc_limiter_learned", [dp, ctypes.c_int, dp], ctypes.c_double),
            ("orc_mlp_forward", [dp, ctypes.c_int, dp], ctypes.c_double),
            ("orc_flux", [P, ctypes.c_int, dp, dp, dp], None),
            ("orc_physical", [P, ctypes.c_int, dp, dp, dp, dp, dp], None),
            ("orc_hllc_star", [P, ctypes.c_int, dp, dp, dp], None),
            ("orc_shock_bits", [P, dp, ctypes.POINTER(ctypes.c_ubyte)], ctypes.c_int),
            ("orc_fmr_level", [ctypes.POINTER(_FmrDesc), ctypes.c_int, P], ctypes.c_int),
            ("orc_fmr_prolong", [ctypes.POINTER(_FmrDesc), ctypes.c_int, dp, dp], ctypes.c_int),
            ("orc_fmr_restrict", [ctypes.POINTER(_FmrDesc), ctypes.c_int, dp, dp], ctypes.c_int),
            ("orc_fmr_step", [ctypes.POINTER(_FmrDesc), ctypes.POINTER(dp), ctypes.c_double, ctypes.c_double, dp],
             ctypes.c_int),
            ("orc_set_threads", [ctypes.c_int], ctypes.c_int),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Host threads the oracle's parallel loops use (n <= 0 keeps the current
    setting); returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Desc:
    """Patch description for the oracle (mirrors a workloads.Problem)."""

    def __init__(self, ndim, n, lo, hi, gamma, bc, solver=HLLC, theta=2.0,
                 limiter=LIM_THETA, accel=(0.0, 0.0, 0.0), mlp: Optional[np.ndarray] = None,
                 mlp_bf16: bool = False, shock_fp32: bool = False):
        self.ndim = ndim
        self.n = tuple(int(v) for v in n)
        self.lo, self.hi = tuple(lo), tuple(hi)
        self.gamma = float(gamma)
        self.bc = tuple(tuple(b) for b in bc)
        self.solver = solver
        self.theta = float(theta)
        self.limiter = limiter
        self.accel = tuple(accel)
        self.mlp = None if mlp is None else np.ascontiguousarray(mlp, dtype=np.float64)
        if self.mlp is not None:
            assert self.mlp.size == MLP_NPARAM
        self.mlp_bf16 = bool(mlp_bf16)
        self.shock_fp32 = bool(shock_fp32)

    @classmethod
    def from_problem(cls, prob, solver=HLLC, theta=None, limiter=LIM_THETA, mlp=None,
                     mlp_bf16=False, shock_fp32=False):
        return cls(prob.ndim, prob.n, prob.lo, prob.hi, prob.gamma, prob.bc, solver,
                   prob.theta if theta is None else theta, limiter, prob.accel, mlp, mlp_bf16, shock_fp32)

    @property
    def nv(self):
        return self.ndim + 2

    @property
    def ncell(self):
        return self.n[0] * self.n[1] * self.n[2]

    def dV(self):
        v = 1.0
        for q in range(self.ndim):
            v *= (self.hi[q] - self.lo[q]) / self.n[q]
        return v

    def c(self) -> _Desc:
        d = _Desc()
        d.ndim = self.ndim
        for q in range(3):
            d.n[q] = self.n[q]
            d.lo[q] = self.lo[q]
            d.hi[q] = self.hi[q]
            d.accel[q] = self.accel[q]
            d.bc[q][0] = self.bc[q][0]
            d.bc[q][1] = self.bc[q][1]
        d.gamma = self.gamma
        d.solver = self.solver
        d.limiter = self.limiter
        d.theta = self.theta
        d.mlp = _dp(self.mlp) if self.mlp is not None else ctypes.POINTER(ctypes.c_double)()
        d.mlp_bf16 = int(self.mlp_bf16)
        d.shock_fp32 = int(self.shock_fp32)
        self._keep = d
        return d


def _flat(desc: Desc, a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(desc.nv, desc.ncell))


def prim_to_cons(desc: Desc, W) -> np.ndarray:
    W = _flat(desc, W)
    U = np.empty_like(W)
    st = lib().orc_prim_to_cons(ctypes.byref(desc.c()), _dp(W), _dp(U))
    if st != OK:
        raise OracleError(st, "prim_to_cons")
    return U


def cons_to_prim(desc: Desc, U, check: bool = True) -> np.ndarray:
    U = _flat(desc, U)
    W = np.empty_like(U)
    st = lib().orc_cons_to_prim(ctypes.byref(desc.c()), _dp(U), _dp(W))
    if check and st != OK:
        raise OracleError(st, "cons_to_prim")
    return W


def rhs(desc: Desc, U) -> np.ndarray:
    U = _flat(desc, U)
    L = np.empty_like(U)
    st = lib().orc_rhs(ctypes.byref(desc.c()), _dp(U), _dp(L))
    if st != OK:
        raise OracleError(st, "rhs")
    return L


def kinetic_energy(desc: Desc, U) -> np.ndarray:
    """Integral of rho v_q^2 / 2 over the patch per component q (Sec. 4.3.1,
    the y component is E_kin,y): dV times the exactly rounded sum over cells
    of S_q^2 / (2 D)."""
    U = _flat(desc, U)
    out = np.zeros(3)
    for q in range(desc.ndim):
        out[q] = math.fsum(0.5 * U[1 + q] ** 2 / U[0]) * desc.dV()
    return out


def shock_bits(desc: Desc, U) -> np.ndarray:
    """Per interior cell, bit q set where the switch's detector flags a shock
    moving along q (see orc_shock_bits)."""
    U = _flat(desc, U)
    out = np.zeros(U.shape[1], dtype=np.uint8)
    st = lib().orc_shock_bits(ctypes.byref(desc.c()), _dp(U), out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    if st not in (OK, ESTATE):
        raise OracleError(st, "shock_bits")
    return out


def step(desc: Desc, U, dt: float) -> np.ndarray:
    """One full two-stage step; returns a new array."""
    U = _flat(desc, U).copy()
    st = lib().orc_step(ctypes.byref(desc.c()), _dp(U), float(dt))
    if st != OK:
        raise OracleError(st, "step")
    return U


def cfl_dt(desc: Desc, U, cfl: float) -> float:
    U = _flat(desc, U)
    out = np.zeros(1)
    st = lib().orc_cfl_dt(ctypes.byref(desc.c()), _dp(U), float(cfl), _dp(out))
    if st != OK:
        raise OracleError(st, "cfl_dt")
    return float(out[0])


def totals(desc: Desc, U) -> np.ndarray:
    """Exactly rounded sums of U_k over the cells times the cell volume,
    returned as (D, S_x, S_y, S_z, G) with zeros for absent components."""
    U = _flat(desc, U)
    out = np.zeros(5)
    dv = desc.dV()
    nd = desc.ndim
    out[0] = math.fsum(U[0].tolist()) * dv
    for r in range(nd):
        out[1 + r] = math.fsum(U[1 + r].tolist()) * dv
    out[4] = math.fsum(U[nd + 1].tolist()) * dv
    return out


def run(desc: Desc, U, t_end: float, cfl: float, max_steps: int = 10 ** 7):
    """Single-level time loop (Alg. 2 with one level): dt = C dt_CFL, the
    last step clipped to end exactly at t_end.  Returns (U, steps)."""
    U = _flat(desc, U).copy()
    t = 0.0
    nsteps = 0
    while t < t_end and nsteps < max_steps:
        dt = min(cfl_dt(desc, U, cfl), t_end - t)
        U = step(desc, U, dt)
        t += dt
        nsteps += 1
    return U, nsteps


def run_steps(desc: Desc, U, nsteps: int, cfl: float):
    """``nsteps`` steps, each of size C dt_CFL of the state it starts from."""
    U = _flat(desc, U).copy()
    for _ in range(nsteps):
        U = step(desc, U, cfl_dt(desc, U, cfl))
    return U


def l1_error(num, exact) -> float:
    """Relative L1 norm, eq. L1ErrorNorm: sum|num - exact| / sum|exact|."""
    num = np.asarray(num, dtype=np.float64).ravel()
    exact = np.asarray(exact, dtype=np.float64).ravel()
    return float(np.sum(np.abs(num - exact)) / np.sum(np.abs(exact)))


def convergence_rate(l1_a: float, n_a: int, l1_b: float, n_b: int) -> float:
    """-p from eq. convergenceRate: log(L1_a / L1_b) / log(N_a / N_b)."""
    return math.log(l1_a / l1_b) / math.log(n_a / n_b)


# ---- pointwise pieces ----

def limiter_theta(dm: float, dp: float, theta: float) -> float:
    return lib().orc_limiter_theta(float(dm), float(dp), float(theta))


def limiter_learned(params: np.ndarray, w5, bf16: bool = False) -> float:
    p = np.ascontiguousarray(params, dtype=np.float64)
    w = np.ascontiguousarray(w5, dtype=np.float64)
    return lib().orc_limiter_learned(_dp(p), int(bf16), _dp(w))


def mlp_forward(params: np.ndarray, x, bf16: bool = False) -> float:
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_mlp_forward(_dp(p), int(bf16), _dp(xx))


def flux(desc: Desc, q: int, wl, wr) -> np.ndarray:
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(desc.nv)
    lib().orc_flux(ctypes.byref(desc.c()), int(q), _dp(wl), _dp(wr), _dp(f))
    return f


def physical(desc: Desc, q: int, w):
    w = np.ascontiguousarray(w, dtype=np.float64)
    U = np.zeros(desc.nv)
    F = np.zeros(desc.nv)
    lm = np.zeros(1)
    lp = np.zeros(1)
    lib().orc_physical(ctypes.byref(desc.c()), int(q), _dp(w), _dp(U), _dp(F), _dp(lm), _dp(lp))
    return U, F, float(lm[0]), float(lp[0])


def hllc_star(desc: Desc, q: int, wl, wr) -> dict:
    nv = desc.nv
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = np.zeros(3 + 4 * nv)
    lib().orc_hllc_star(ctypes.byref(desc.c()), int(q), _dp(wl), _dp(wr), _dp(out))
    return {
        "alpha_m": out[0], "p_star_L": out[1], "p_star_R": out[2],
        "U_star_L": out[3:3 + nv], "U_star_R": out[3 + nv:3 + 2 * nv],
        "F_star_L": out[3 + 2 * nv:3 + 3 * nv], "F_star_R": out[3 + 3 * nv:3 + 4 * nv],
    }


# ---- fixed multilevel refinement (Sec. 2 prolongation / restriction, Sec. 3.6 Algs. Evolve..StepLevel) ----

class FmrDesc:
    """Nested levels: ``base`` is level 0; ``boxes[l - 1] = (lo, n)`` is the
    box of level l - 1 cells that level l refines by two (unused dimensions:
    lo 0, n 1)."""

    def __init__(self, base: Desc, boxes, no_reflux: bool = False):
        self.base = base
        self.boxes = [(tuple(int(v) for v in lo), tuple(int(v) for v in n)) for lo, n in boxes]
        self.nlev = 1 + len(self.boxes)
        assert self.nlev <= FMR_MAXLEV
        self.no_reflux = bool(no_reflux)
        self.levels = [self.level(l) for l in range(self.nlev)]

    def c(self) -> _FmrDesc:
        f = _FmrDesc()
        f.base = self.base.c()
        f.nlev = self.nlev
        for l, (lo, n) in enumerate(self.boxes, start=1):
            for q in range(3):
                f.box_lo[l][q] = lo[q]
                f.box_n[l][q] = n[q]
        f.no_reflux = int(self.no_reflux)
        self._keep = (f, self.base._keep)
        return f

    def level(self, l: int) -> Desc:
        out = _Desc()
        st = lib().orc_fmr_level(ctypes.byref(self.c()), int(l), ctypes.byref(out))
        if st != OK:
            raise OracleError(st, "fmr_level")
        b = self.base
        return Desc(b.ndim, tuple(out.n), tuple(out.lo), tuple(out.hi), b.gamma,
                    tuple((out.bc[q][0], out.bc[q][1]) for q in range(3)), b.solver, b.theta, b.limiter, b.accel)

    def ghosted_shape(self, l: int):
        d = self.levels[l]
        return tuple(d.n[q] + (2 * NG if q < d.ndim else 0) for q in range(3))

    def covered(self, l: int) -> np.ndarray:
        """Boolean (ncell,) of level l: True where level l + 1 covers the cell."""
        d = self.levels[l]
        m = np.zeros((d.n[2], d.n[1], d.n[0]), dtype=bool)
        if l + 1 < self.nlev:
            lo, n = self.boxes[l]
            m[lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]] = True
        return m.ravel()


def fmr_prolong(f: FmrDesc, l: int, Uparent) -> np.ndarray:
    """Level l's exterior from its parent: (nv, ghosted cells) with NaN in
    the interior cells, which prolongation does not write."""
    Up = _flat(f.levels[l - 1], Uparent)
    m = f.ghosted_shape(l)
    ext = np.full((f.base.nv, m[0] * m[1] * m[2]), np.nan)
    st = lib().orc_fmr_prolong(ctypes.byref(f.c()), int(l), _dp(Up), _dp(ext))
    if st != OK:
        raise OracleError(st, "fmr_prolong")
    return ext


def fmr_restrict(f: FmrDesc, l: int, Uchild, Uparent) -> np.ndarray:
    Uc = _flat(f.levels[l], Uchild)
    Up = _flat(f.levels[l - 1], Uparent).copy()
    st = lib().orc_fmr_restrict(ctypes.byref(f.c()), int(l), _dp(Uc), _dp(Up))
    if st != OK:
        raise OracleError(st, "fmr_restrict")
    return Up


def fmr_step(f: FmrDesc, Us, cfl: float = 0.4, dt_fixed: float = 0.0):
    """One global step of every level; returns (new level states, coarse dt)."""
    Us = [_flat(f.levels[l], U).copy() for l, U in enumerate(Us)]
    ptrs = (ctypes.POINTER(ctypes.c_double) * f.nlev)(*[_dp(U) for U in Us])
    out = np.zeros(1)
    st = lib().orc_fmr_step(ctypes.byref(f.c()), ptrs, float(cfl), float(dt_fixed), _dp(out))
    if st != OK:
        raise OracleError(st, "fmr_step")
    return Us, float(out[0])


def fmr_totals(f: FmrDesc, Us) -> np.ndarray:
    """Conserved totals over the leaf cells (cells no finer level covers),
    each level's cells weighted by its cell volume; exactly rounded sums."""
    nd = f.base.ndim
    parts = [[] for _ in range(5)]
    for l, U in enumerate(Us):
        d = f.levels[l]
        U = _flat(d, U)
        leaf = ~f.covered(l)
        dv = d.dV()
        comps = [0] + [1 + r for r in range(nd)] + [nd + 1]
        slots = [0] + [1 + r for r in range(nd)] + [4]
        for c, s in zip(comps, slots):
            parts[s].extend((U[c][leaf] * dv).tolist())
    return np.array([math.fsum(p) for p in parts])
