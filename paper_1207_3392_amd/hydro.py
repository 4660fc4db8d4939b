"""Python binding of libhydro.so (include/hydro.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch supplies
device memory (the workspace is a uint8 tensor) and the HIP stream (torch's
current stream).  If the library is not built this module raises; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydro.so")

HY_OK, HY_EINVAL, HY_ENOMEM, HY_EDEVICE, HY_ESTATE, HY_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
HLL, HLLC, HLLC_SWITCH = 0, 1, 2
LIM_THETA, LIM_LEARNED = 0, 1
PRIMITIVE, CONSERVED = 0, 1
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
MLP_NPARAM = 1249


class HydroError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hydro status {status}: {msg}")
        self.status = status


class LaunchCfg(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int), ("by", ctypes.c_int), ("zchunk", ctypes.c_int)]


class PatchDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("bc", (ctypes.c_int * 2) * 3),
        ("precision", ctypes.c_int),
        ("limiter", ctypes.c_int),
        ("theta", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
    ]


FMR_MAXLEV = 8


class FmrDesc(ctypes.Structure):
    _fields_ = [
        ("base", PatchDesc),
        ("nlev", ctypes.c_int),
        ("box_lo", (ctypes.c_int64 * 3) * FMR_MAXLEV),
        ("box_n", (ctypes.c_int64 * 3) * FMR_MAXLEV),
    ]


_P = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)

SIGNATURES = {
    "hy_patch_workspace_bytes": [ctypes.POINTER(PatchDesc), ctypes.POINTER(ctypes.c_size_t)],
    "hy_init_patch": [ctypes.POINTER(PatchDesc), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "hy_set_state": [_P, ctypes.c_int, _dp],
    "hy_get_state": [_P, ctypes.c_int, _dp],
    "hy_step": [_P, ctypes.c_double, ctypes.c_int],
    "hy_cfl_dt": [_P, ctypes.c_double, _dp],
    "hy_advance": [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int],
    "hy_advance_graph_prepare": [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int],
    "hy_advance_graph": [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int],
    "hy_get_time": [_P, _dp],
    "hy_conserved_totals": [_P, _dp],
    "hy_kinetic_energy": [_P, _dp],
    "hy_spectrum_workspace_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "hy_kinetic_spectrum": [_P, ctypes.c_void_p, ctypes.c_size_t, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "hy_set_mlp": [_P, _fp, ctypes.c_size_t],
    "hy_set_timing": [_P, ctypes.c_int],
    "hy_kernel_times": [_P, _dp, _i64p],
    "hy_kernel_config": [_P, ctypes.c_char_p, ctypes.c_size_t],
    "hy_get_launch_cfg": [_P, ctypes.POINTER(LaunchCfg)],
    "hy_set_launch_cfg": [_P, ctypes.POINTER(LaunchCfg)],
    "hy_autotune": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(LaunchCfg), _dp],
    "hy_destroy": [_P],
}

_lib = None


def lib():
    """Load libhydro.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1207_3392_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.hy_last_error.argtypes = []
        L.hy_last_error.restype = ctypes.c_char_p
        _extra_signatures(L)
        _lib = L
    return _lib


def _extra_signatures(L):
    """Signatures of the batched-launch and training entry points."""
    for name, args in EXTRA_SIGNATURES.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int


EXTRA_SIGNATURES = {
    "hy_batch_workspace_bytes": [ctypes.POINTER(PatchDesc), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "hy_batch_init": [ctypes.POINTER(PatchDesc), ctypes.c_int, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "hy_batch_set_state": [_P, ctypes.c_int, ctypes.c_int, _dp],
    "hy_batch_run_to": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int],
    "hy_batch_last_ms": [_P, _dp],
    "hy_batch_set_block": [_P, ctypes.c_int],
    "hy_batch_get_block": [_P, ctypes.POINTER(ctypes.c_int)],
    "hy_batch_autotune": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp],
    "hy_batch_get_state": [_P, ctypes.c_int, ctypes.c_int, _dp],
    "hy_batch_status": [_P, ctypes.c_int, _i64p, _dp],
    "hy_batch_destroy": [_P],
    "hy_lim_sample_count": [_P, _i64p],
    "hy_lim_samples_scratch_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "hy_lim_make_samples": [_P, _P, ctypes.c_size_t, _P, _P],
    "hy_lim_make_samples_noalloc": [_P, _P, _P],
    "hy_lim_slopes": [_P, _P],
    "hy_trainer_workspace_bytes": [ctypes.POINTER(ctypes.c_size_t)],
    "hy_trainer_init": [_P, ctypes.c_size_t, _fp, _P, ctypes.POINTER(_P)],
    "hy_trainer_step": [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float],
    "hy_trainer_gradient": [_P, _P, _P, _P, ctypes.c_int64, _fp, _fp],
    "hy_trainer_loss": [_P, _fp],
    "hy_trainer_get_params": [_P, _fp],
    "hy_mlp_eval": [_P, _P, _P, ctypes.c_int64],
    "hy_trainer_destroy": [_P],
    "hy_fmr_workspace_bytes": [ctypes.POINTER(FmrDesc), ctypes.POINTER(ctypes.c_size_t)],
    "hy_fmr_init": [ctypes.POINTER(FmrDesc), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "hy_fmr_set_state": [_P, ctypes.c_int, ctypes.c_int, _dp],
    "hy_fmr_get_state": [_P, ctypes.c_int, ctypes.c_int, _dp],
    "hy_fmr_step": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp],
    "hy_fmr_conserved_totals": [_P, _dp],
    "hy_fmr_autotune": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(LaunchCfg)],
    "hy_fmr_set_graph": [_P, ctypes.c_int],
    "hy_fmr_destroy": [_P],
}


def check(status: int, what: str = ""):
    if status != HY_OK:
        msg = lib().hy_last_error().decode(errors="replace")
        raise HydroError(status, f"{what}: {msg}")


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def make_desc(ndim, n, lo, hi, gamma, bc, precision=32, limiter=LIM_THETA, theta=2.0,
              accel=(0.0, 0.0, 0.0)) -> PatchDesc:
    d = PatchDesc()
    d.ndim = int(ndim)
    for q in range(3):
        d.n[q] = int(n[q])
        d.lo[q] = float(lo[q])
        d.hi[q] = float(hi[q])
        d.bc[q][0] = int(bc[q][0])
        d.bc[q][1] = int(bc[q][1])
        d.accel[q] = float(accel[q])
    d.gamma = float(gamma)
    d.precision = int(precision)
    d.limiter = int(limiter)
    d.theta = float(theta)
    return d


class Patch:
    """One Cartesian patch in GPU memory.

    ``problem`` is a workloads.Problem (or any object with ndim, n, lo, hi,
    gamma, bc, theta, accel).  The workspace is allocated as a torch uint8
    tensor on ``device``; work is enqueued on torch's current stream there."""

    def __init__(self, problem, precision: int = 32, limiter: int = LIM_THETA,
                 theta: Optional[float] = None, device: str = "cuda", set_initial: bool = True):
        import torch

        self.problem = problem
        self.ndim = problem.ndim
        self.n = tuple(int(v) for v in problem.n)
        self.nv = self.ndim + 2
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        self.precision, self.limiter = int(precision), int(limiter)
        self.desc = make_desc(problem.ndim, problem.n, problem.lo, problem.hi, problem.gamma,
                              problem.bc, precision, limiter,
                              problem.theta if theta is None else theta, problem.accel)
        nbytes = ctypes.c_size_t(0)
        check(lib().hy_patch_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)),
              "workspace_bytes")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _P()
        check(lib().hy_init_patch(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                                  nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "init_patch")
        self.handle = h
        if set_initial and getattr(problem, "W", None) is not None:
            self.set_state(problem.W, PRIMITIVE)

    # ---- state ----
    def set_state(self, arr, kind: int = PRIMITIVE):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(self.nv, self.ncell))
        check(lib().hy_set_state(self.handle, int(kind), _dptr(a)), "set_state")

    def get_state(self, kind: int = CONSERVED, check_state: bool = True) -> np.ndarray:
        out = np.empty((self.nv, self.ncell), dtype=np.float64)
        st = lib().hy_get_state(self.handle, int(kind), _dptr(out))
        if check_state or st != HY_ESTATE:
            check(st, "get_state")
        return out

    # ---- stepping ----
    def step(self, dt: float, solver: int = HLLC):
        check(lib().hy_step(self.handle, float(dt), int(solver)), "step")

    def cfl_dt(self, cfl: float) -> float:
        out = ctypes.c_double(0.0)
        check(lib().hy_cfl_dt(self.handle, float(cfl), ctypes.byref(out)), "cfl_dt")
        return out.value

    def advance(self, nsteps: int, cfl: float, t_end: float = float("inf"), solver: int = HLLC):
        check(lib().hy_advance(self.handle, int(nsteps), float(cfl), float(t_end), int(solver)), "advance")

    def advance_graph(self, nsteps: int, cfl: float, t_end: float = float("inf"), solver: int = HLLC,
                      prepare_only: bool = False):
        """hy_advance as one replay of a captured HIP graph (prepare_only:
        capture without running)."""
        fn = lib().hy_advance_graph_prepare if prepare_only else lib().hy_advance_graph
        check(fn(self.handle, int(nsteps), float(cfl), float(t_end), int(solver)), "advance_graph")

    def time(self) -> float:
        out = ctypes.c_double(0.0)
        check(lib().hy_get_time(self.handle, ctypes.byref(out)), "get_time")
        return out.value

    def totals(self) -> np.ndarray:
        out = np.zeros(5)
        check(lib().hy_conserved_totals(self.handle, _dptr(out)), "conserved_totals")
        return out

    def kinetic_energy(self) -> np.ndarray:
        """Integral of rho v_q^2 / 2 per component q (FP64 reduction)."""
        out = np.zeros(3)
        check(lib().hy_kinetic_energy(self.handle, _dptr(out)), "kinetic_energy")
        return out

    def kinetic_spectrum(self):
        """Kinetic-energy spectrum of a 2D N x N patch on the device: (k, e)
        with k = 2 pi s / L for the shells s = 0, 1, ... (hy_kinetic_spectrum)."""
        import torch

        nb = ctypes.c_size_t(0)
        check(lib().hy_spectrum_workspace_bytes(self.handle, ctypes.byref(nb)), "spectrum_workspace_bytes")
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        n = int(self.desc.n[0])
        cap = int(math.floor(math.sqrt(2.0) * (n // 2) + 0.5)) + 1
        e = np.zeros(cap)
        ns = ctypes.c_int(0)
        check(lib().hy_kinetic_spectrum(self.handle, ctypes.c_void_p(ws.data_ptr()), nb, _dptr(e), cap,
                                        ctypes.byref(ns)), "kinetic_spectrum")
        del ws
        box = float(self.desc.hi[0] - self.desc.lo[0])
        return 2.0 * math.pi / box * np.arange(ns.value), e[:ns.value]

    def set_mlp(self, params):
        w = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        check(lib().hy_set_mlp(self.handle, w.ctypes.data_as(_fp), ctypes.c_size_t(w.size)), "set_mlp")

    # ---- timing ----
    def set_timing(self, on: bool):
        check(lib().hy_set_timing(self.handle, int(bool(on))), "set_timing")

    def kernel_times(self):
        ms = np.zeros(2)
        n = np.zeros(2, dtype=np.int64)
        check(lib().hy_kernel_times(self.handle, _dptr(ms), n.ctypes.data_as(_i64p)), "kernel_times")
        return ms, n

    def make_samples(self):
        """Training samples of the learned limiter from this (fine, periodic)
        patch: returns device tensors x (n, 4) and t (n) (float32)."""
        import torch

        ns = ctypes.c_int64(0)
        check(lib().hy_lim_sample_count(self.handle, ctypes.byref(ns)), "lim_sample_count")
        nb = ctypes.c_size_t(0)
        check(lib().hy_lim_samples_scratch_bytes(self.handle, ctypes.byref(nb)), "lim_samples_scratch_bytes")
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        x = torch.empty((ns.value, 4), dtype=torch.float32, device=self.device)
        t = torch.empty((ns.value,), dtype=torch.float32, device=self.device)
        check(lib().hy_lim_make_samples(self.handle, ctypes.c_void_p(scratch.data_ptr()), nb,
                                        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr())),
              "lim_make_samples")
        torch.cuda.current_stream(self.device).synchronize()
        del scratch
        return x, t

    def make_samples_noalloc(self, x, t):
        """make_samples into caller tensors x (n, 4), t (n) (float32, on this
        patch's device), staged in the library's static device array (no
        allocation; raises HY_ENOMEM beyond its 64 MiB)."""
        check(lib().hy_lim_make_samples_noalloc(self.handle, ctypes.c_void_p(x.data_ptr()),
                                                ctypes.c_void_p(t.data_ptr())), "lim_make_samples_noalloc")

    def sample_count(self) -> int:
        ns = ctypes.c_int64(0)
        check(lib().hy_lim_sample_count(self.handle, ctypes.byref(ns)), "lim_sample_count")
        return int(ns.value)

    def learned_slopes(self):
        """Clamped learned slopes of the current state, (ndim * nv, ncell) on the device."""
        import torch

        out = torch.empty((self.ndim * self.nv, self.ncell), dtype=torch.float32, device=self.device)
        check(lib().hy_lim_slopes(self.handle, ctypes.c_void_p(out.data_ptr())), "lim_slopes")
        torch.cuda.current_stream(self.device).synchronize()
        return out

    def kernel_config(self) -> str:
        buf = ctypes.create_string_buffer(256)
        check(lib().hy_kernel_config(self.handle, buf, 256), "kernel_config")
        return buf.value.decode()

    def launch_cfg(self):
        """(bx, by, zchunk) of the stage kernels' launch shape."""
        c = LaunchCfg()
        check(lib().hy_get_launch_cfg(self.handle, ctypes.byref(c)), "get_launch_cfg")
        return (c.bx, c.by, c.zchunk)

    def set_launch_cfg(self, bx: int, by: int, zchunk: int):
        c = LaunchCfg(bx, by, zchunk)
        check(lib().hy_set_launch_cfg(self.handle, ctypes.byref(c)), "set_launch_cfg")

    def autotune(self, solver: int = HLLC, reps: int = 5, cache: Optional[str] = None):
        """Pick the fastest launch shape for this patch (see hy_autotune).

        With ``cache`` (a JSON file path) a shape already tuned for the same
        device architecture, dimensions, precision, limiter, solver and size
        is applied without timing, and a new result is added to the file.
        Returns (bx, by, zchunk, ms per first-stage launch or None if cached)."""
        key = None
        if cache:
            import torch

            arch = torch.cuda.get_device_properties(torch.device(self.device)).gcnArchName.split(":")[0]
            key = (f"{arch}|nd{self.ndim}|fp{self.precision}|lim{self.limiter}|"
                   f"{'hllc' if solver == HLLC else 'hll'}|{'x'.join(str(int(v)) for v in self.n)}")
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            if key in table:
                e = table[key]
                self.set_launch_cfg(e["bx"], e["by"], e["zchunk"])
                return (e["bx"], e["by"], e["zchunk"], None)
        best, ms = LaunchCfg(), ctypes.c_double()
        check(lib().hy_autotune(self.handle, int(solver), int(reps), ctypes.byref(best), ctypes.byref(ms)),
              "autotune")
        if key:
            table[key] = {"bx": best.bx, "by": best.by, "zchunk": best.zchunk, "ms": ms.value}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return (best.bx, best.by, best.zchunk, ms.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().hy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- loops ----
    def run(self, t_end: float, cfl: float, solver: int = HLLC, max_steps: int = 10 ** 8) -> int:
        """Host-driven single-level loop: dt = min(C dt_CFL, t_end - t)."""
        t, k = 0.0, 0
        while t < t_end and k < max_steps:
            dt = min(self.cfl_dt(cfl), t_end - t)
            self.step(dt, solver)
            t += dt
            k += 1
        return k


class Batch:
    """Independent 1D tubes advanced together in one persistent launch.

    ``problems`` is a sequence of 1D workloads.Problem objects (FP32,
    generalised minmod, no source)."""

    def __init__(self, problems, device: str = "cuda", theta: Optional[float] = None):
        import torch

        self.problems = list(problems)
        n = len(self.problems)
        arr = (PatchDesc * n)()
        for i, pr in enumerate(self.problems):
            arr[i] = make_desc(pr.ndim, pr.n, pr.lo, pr.hi, pr.gamma, pr.bc, 32, LIM_THETA,
                               pr.theta if theta is None else theta, pr.accel)
        self.descs = arr
        nbytes = ctypes.c_size_t(0)
        check(lib().hy_batch_workspace_bytes(arr, n, ctypes.byref(nbytes)), "batch_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=torch.device(device))
        self.stream = torch.cuda.current_stream(self.workspace.device)
        h = _P()
        check(lib().hy_batch_init(arr, n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "batch_init")
        self.handle = h
        for i, pr in enumerate(self.problems):
            self.set_state(i, pr.W, PRIMITIVE)

    def set_state(self, i: int, arr, kind: int = PRIMITIVE):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(3, -1))
        check(lib().hy_batch_set_state(self.handle, int(i), int(kind), _dptr(a)), "batch_set_state")

    def run_to(self, t_end: float, cfl: float, solver: int = HLLC):
        check(lib().hy_batch_run_to(self.handle, float(t_end), float(cfl), int(solver)), "batch_run_to")

    def block(self) -> int:
        """Threads per workgroup of the batched kernel."""
        v = ctypes.c_int()
        check(lib().hy_batch_get_block(self.handle, ctypes.byref(v)), "batch_get_block")
        return v.value

    def set_block(self, threads: int):
        check(lib().hy_batch_set_block(self.handle, int(threads)), "batch_set_block")

    def autotune(self, t_end: float, cfl: float, solver: int = HLLC):
        """Time the whole run with each workgroup size, keep the fastest, leave
        the state as it was; returns (threads, ms)."""
        bt, ms = ctypes.c_int(), ctypes.c_double()
        check(lib().hy_batch_autotune(self.handle, float(t_end), float(cfl), int(solver), ctypes.byref(bt),
                                      ctypes.byref(ms)), "batch_autotune")
        return bt.value, ms.value

    def last_ms(self) -> float:
        out = ctypes.c_double(0.0)
        check(lib().hy_batch_last_ms(self.handle, ctypes.byref(out)), "batch_last_ms")
        return out.value

    def get_state(self, i: int, kind: int = PRIMITIVE) -> np.ndarray:
        n = int(self.problems[i].n[0])
        out = np.empty((3, n), dtype=np.float64)
        check(lib().hy_batch_get_state(self.handle, int(i), int(kind), _dptr(out)), "batch_get_state")
        return out

    def status(self, i: int):
        steps = ctypes.c_int64(0)
        t = ctypes.c_double(0.0)
        check(lib().hy_batch_status(self.handle, int(i), ctypes.byref(steps), ctypes.byref(t)), "batch_status")
        return steps.value, t.value

    def close(self):
        if getattr(self, "handle", None):
            lib().hy_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trainer:
    """Device-side trainer of the learned limiter (FP32 master weights, Adam)."""

    def __init__(self, params, device: str = "cuda"):
        import torch

        nb = ctypes.c_size_t(0)
        check(lib().hy_trainer_workspace_bytes(ctypes.byref(nb)), "trainer_workspace_bytes")
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=torch.device(device))
        self.stream = torch.cuda.current_stream(self.workspace.device)
        w = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        assert w.size == MLP_NPARAM
        h = _P()
        check(lib().hy_trainer_init(ctypes.c_void_p(self.workspace.data_ptr()), nb, w.ctypes.data_as(_fp),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "trainer_init")
        self.handle = h

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr())

    def step(self, x, t, idx, lr: float = 1e-3):
        """x (n, 4), t (n) float32 and idx (batch) int32 device tensors."""
        check(lib().hy_trainer_step(self.handle, self._ptr(x), self._ptr(t), self._ptr(idx),
                                    int(idx.numel()), float(lr)), "trainer_step")

    def gradient(self, x, t, idx):
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        check(lib().hy_trainer_gradient(self.handle, self._ptr(x), self._ptr(t), self._ptr(idx),
                                        int(idx.numel()), g.ctypes.data_as(_fp), loss.ctypes.data_as(_fp)),
              "trainer_gradient")
        return g, float(loss[0])

    def loss(self) -> float:
        out = np.zeros(1, dtype=np.float32)
        check(lib().hy_trainer_loss(self.handle, out.ctypes.data_as(_fp)), "trainer_loss")
        return float(out[0])

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        check(lib().hy_trainer_get_params(self.handle, out.ctypes.data_as(_fp)), "trainer_get_params")
        return out

    def eval(self, x):
        """Network output (the limiter's MFMA inference kernel) on x (n, 4)."""
        import torch

        y = torch.empty((x.shape[0],), dtype=torch.float32, device=x.device)
        check(lib().hy_mlp_eval(self.handle, self._ptr(x), self._ptr(y), int(x.shape[0])), "mlp_eval")
        return y

    def close(self):
        if getattr(self, "handle", None):
            lib().hy_trainer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fmr:
    """Nested levels stepped with subcycling and coarse/fine flux replacement
    (include/hydro.h, hy_fmr_*).  ``levels`` is a workloads.Levels (base
    problem, boxes, per-level initial primitive fields)."""

    def __init__(self, levels, precision: int = 32, theta: Optional[float] = None, device: str = "cuda",
                 set_initial: bool = True):
        import torch

        b = levels.base
        self.levels = levels
        self.nlev = levels.nlev
        self.ndim = b.ndim
        self.nv = b.ndim + 2
        self.desc = FmrDesc()
        self.desc.base = make_desc(b.ndim, b.n, b.lo, b.hi, b.gamma, b.bc, precision, LIM_THETA,
                                   b.theta if theta is None else theta, b.accel)
        self.desc.nlev = self.nlev
        for l, (lo, n) in enumerate(levels.boxes, start=1):
            for q in range(3):
                self.desc.box_lo[l][q] = int(lo[q])
                self.desc.box_n[l][q] = int(n[q])
        self.ncell = [int(np.prod(levels.level_geometry(l)[0])) for l in range(self.nlev)]
        nbytes = ctypes.c_size_t(0)
        check(lib().hy_fmr_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)), "fmr_workspace_bytes")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _P()
        check(lib().hy_fmr_init(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "fmr_init")
        self.handle = h
        if set_initial:
            for l, W in enumerate(levels.W):
                self.set_state(l, W, PRIMITIVE)

    def set_state(self, level: int, arr, kind: int = PRIMITIVE):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(self.nv, self.ncell[level]))
        check(lib().hy_fmr_set_state(self.handle, int(level), int(kind), _dptr(a)), "fmr_set_state")

    def get_state(self, level: int, kind: int = CONSERVED) -> np.ndarray:
        out = np.empty((self.nv, self.ncell[level]), dtype=np.float64)
        check(lib().hy_fmr_get_state(self.handle, int(level), int(kind), _dptr(out)), "fmr_get_state")
        return out

    def step(self, cfl: float = 0.4, dt_fixed: float = 0.0, solver: int = HLLC) -> float:
        """One global step; returns the coarse time step."""
        out = ctypes.c_double(0.0)
        check(lib().hy_fmr_step(self.handle, float(cfl), float(dt_fixed), int(solver), ctypes.byref(out)),
              "fmr_step")
        return out.value

    def totals(self) -> np.ndarray:
        out = np.zeros(5)
        check(lib().hy_fmr_conserved_totals(self.handle, _dptr(out)), "fmr_conserved_totals")
        return out

    def set_graph(self, on: bool):
        """Replay the global step from a captured HIP graph (default) or launch it kernel by kernel."""
        check(lib().hy_fmr_set_graph(self.handle, int(bool(on))), "fmr_set_graph")

    def autotune(self, solver: int = HLLC, reps: int = 3):
        """Tune every level's stage launch shape; returns [(bx, by, zchunk)] per level."""
        best = (LaunchCfg * self.nlev)()
        check(lib().hy_fmr_autotune(self.handle, int(solver), int(reps), best), "fmr_autotune")
        return [(c.bx, c.by, c.zchunk) for c in best]

    def close(self):
        if getattr(self, "handle", None):
            lib().hy_fmr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
