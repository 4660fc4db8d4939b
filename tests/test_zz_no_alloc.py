"""The allocation-free training-sample entry point (static device staging)
against the entry point with a caller scratch, through the C ABI: bit for bit
on two calls in a row, the second on a smaller patch, and the size limit."""
import ctypes

import numpy as np
import pytest

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


def _samples_both(prob, steps):
    p = hydro.Patch(prob, precision=32)
    if steps:
        p.advance(steps, 0.4, solver=hydro.HLLC)
    ref_x, ref_t = p.make_samples()
    n = p.sample_count()
    x = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
    t = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    p.make_samples_noalloc(x, t)
    torch.cuda.synchronize()
    p.close()
    return ref_x.cpu().numpy(), ref_t.cpu().numpy(), x.cpu().numpy(), t.cpu().numpy()


def test_noalloc_samples_equal_scratch_samples_two_calls():
    # a 2D Kelvin-Helmholtz patch, then a smaller 3D smooth patch: the second
    # call reuses the static array holding the first call's larger staging
    for prob, steps in ((wl.kelvin_helmholtz(128), 10), (wl.random_smooth_patch(3, (24, 20, 28), seed=5), 2)):
        rx, rt, x, t = _samples_both(prob, steps)
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(t))
        assert np.array_equal(x.view(np.uint32), rx.view(np.uint32)), prob.name
        assert np.array_equal(t.view(np.uint32), rt.view(np.uint32)), prob.name


def test_noalloc_samples_reject_patch_beyond_static_size():
    # 3D 264^3: 66^3 coarse cells x 65 floats = 74.8 MB of staging > 64 MiB
    n = 264
    prob = wl.Problem(3, (n, n, n), (0, 0, 0), (1, 1, 1), 5.0 / 3.0, ((0, 0),) * 3, None)
    p = hydro.Patch(prob, precision=32, set_initial=False)
    nb = ctypes.c_size_t(0)
    assert hydro.lib().hy_lim_samples_scratch_bytes(p.handle, ctypes.byref(nb)) == 0
    assert nb.value > 64 << 20
    x = torch.empty((1, 4), dtype=torch.float32, device="cuda")
    t = torch.empty((1,), dtype=torch.float32, device="cuda")
    st = hydro.lib().hy_lim_make_samples_noalloc(p.handle, ctypes.c_void_p(x.data_ptr()),
                                                 ctypes.c_void_p(t.data_ptr()))
    assert st == hydro.HY_ENOMEM
    assert b"64 MiB" in hydro.lib().hy_last_error()
    p.close()
