"""pm_run_noalloc (the whole-simulation entry point that allocates nothing,
its arena in the library's static device scratch) against pm_create +
pm_init_ic + pm_run on a handle of its own, through the C ABI: two calls in a
row, the second on a smaller simulation, each bit for bit in float32 (the
same kernels; paint and projection accumulate in fixed point) and to
round-off in float64; and the refusal of an arena beyond the scratch."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu


def _reference(wl, noise, dtype):
    with new_sim(wl, dtype) as sim:
        k = sim.run(noise, wl.a_grid())
        sim.sync()
        return k.clone()


def _noalloc(wl, noise, dtype):
    from paper_2012_07266_amd.sim import run_noalloc
    k = torch.zeros((len(wl.z_src), wl.npix, wl.npix), dtype=dtype, device="cuda")
    run_noalloc(noise.to("cuda", dtype), wl.a_grid(), k, wl.np_side, wl.nm_side, wl.box, wl.npix,
                wl.fov_deg, wl.z_src, dtype=dtype, omega_m=wl.omega_m, sigma8=wl.sigma8,
                h=wl.h, n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb)
    torch.cuda.synchronize()
    return k


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_run_equals_pm_run(dtype):
    # the largest float32 case the scratch holds (51 MiB), then a smaller one
    big = W.Workload("noalloc_big", 64, 128, 100.0, 0.1, 1.0, 6, 128, 3.0, (1.0, 1.5), seed=21)
    small = W.Workload("noalloc_small", 32, 64, 64.0, 0.2, 1.0, 4, 64, 3.0, (1.0,), seed=22)
    if dtype == torch.float64:
        big = big.with_(np_side=48, nm_side=96)  # float64 arena within the scratch
    for wl in (big, small):
        log(f"noalloc {dtype} {wl.np_side}^3/{wl.nm_side}^3")
        noise = torch.from_numpy(W.white_noise(wl.np_side, wl.seed))
        ref = _reference(wl, noise, dtype)
        got = _noalloc(wl, noise, dtype)
        assert torch.abs(ref).max() > 0
        if dtype == torch.float32:
            assert torch.equal(got, ref)
        else:
            assert rel_rms(to_np(got), to_np(ref)) < 1e-12


def test_noalloc_refuses_an_arena_beyond_the_scratch():
    from paper_2012_07266_amd import _lib
    from paper_2012_07266_amd.sim import footprint, make_lens, make_params
    assert footprint(128, 256, 128.0, 64, 2.0, (1.0,)) > _lib.PM_NOALLOC_MAX_BYTES
    p = make_params(128, 256, 128.0)
    l = make_lens(64, 2.0, (1.0,))
    a = np.linspace(0.1, 1.0, 3)
    noise = torch.zeros((128,) * 3, dtype=torch.float32, device="cuda")
    kap = torch.zeros((1, 64, 64), dtype=torch.float32, device="cuda")
    rc = _lib.lib().pm_run_noalloc(ctypes.byref(p), ctypes.byref(l), None,
                                   ctypes.c_void_p(noise.data_ptr()),
                                   a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2,
                                   ctypes.c_void_p(kap.data_ptr()))
    assert rc == _lib.PM_ETOOBIG
    assert _lib.lib().pm_strerror(rc).decode().startswith("arena larger")
    assert torch.equal(kap, torch.zeros_like(kap))
