"""GPU parity of the sub-evolution projection (pm_set_interpolation) against
the float64 oracle: an image keeps the shell of its end-of-step depth and is
moved along its step's drift to the scale factor of that depth before it is
projected.  Float64 agrees to round-off; float32 within 1e-4 relative RMS of
the maps (the tolerance of the plain projection)."""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import cosmo_of, log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


def _tol(dtype, f64, f32):
    return f64 if dtype == torch.float64 else f32


def _run_wl(np_side, nm, box):
    return W.Workload("sub", np_side, nm, box, 0.3, 1.0, 5, 64, 3.0, (0.5, 1.0), seed=9)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 32, 40.0), (32, 32, 64.0)], ids=lambda s: f"{s[0]}p{s[1]}m")
def test_run_with_interpolation_matches_oracle(dtype, shape):
    from oracle import lens
    np_side, nm, box = shape
    wl = _run_wl(np_side, nm, box)
    log(f"sub-evolution run {dtype} np={np_side} nm={nm}")
    c = cosmo_of(wl)
    noise = W.white_noise(np_side, wl.seed)
    a = wl.a_grid()
    with new_sim(wl, dtype) as sim:
        k_plain = to_np(sim.run(torch.from_numpy(noise), a))
        sim.set_interpolation(True)
        k_sub = to_np(sim.run(torch.from_numpy(noise), a))
        sim.sync()
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    log("oracle run")
    kap, _, _ = lens.run_lensing(noise, c, box, nm, a, geom, interpolation=True)
    e = rel_rms(k_sub, kap)
    moved = rel_rms(k_plain, kap)
    log(f"sub {dtype} {shape}: kappa rel-rms {e:.3e} (plain vs sub-evolved oracle {moved:.3e})")
    assert moved > 1e-3          # the mode changes the maps by far more than the tolerance
    assert e <= _tol(dtype, 1e-10, 1e-4)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_stepwise_equals_fused_with_interpolation(dtype):
    """pm_step + lens_project rebuild the drift momentum as p - K2 f; pm_run
    projects while the momentum is the drift momentum itself.  The two agree
    to the rounding of that reconstruction."""
    wl = _run_wl(32, 64, 64.0)
    noise = torch.from_numpy(W.white_noise(32, wl.seed))
    a = wl.a_grid()
    with new_sim(wl, dtype) as sim:
        sim.set_interpolation(True)
        k1 = to_np(sim.run_stepwise(noise, a).clone())
        k2 = to_np(sim.run(noise, a))
        sim.sync()
    e = rel_rms(k1, k2)
    log(f"sub stepwise vs fused {dtype}: {e:.3e}")
    assert np.abs(k1).max() > 0
    assert e <= _tol(dtype, 1e-12, 2e-5)


THICK = dict(np_side=16, nm=32, box=64.0, a0=0.45, a1=0.6, npix=48, fov=6.0,
             z_src=(0.5, 1.0, 1.5, 2.0))


@functools.lru_cache(maxsize=None)
def _thick_oracle():
    """Oracle maps of one step from the set state, with and without
    sub-evolution (shared by both precisions)."""
    from oracle import lens, pm
    t = THICK
    wl = _thick_wl()
    c = cosmo_of(wl)
    x0, p0 = _thick_state()
    f0 = pm.particle_force(x0, t["np_side"], t["nm"], t["box"])
    x1, _, _, p_h = pm.kdk_step(x0, p0, f0, t["a0"], t["a1"], c, t["np_side"], t["nm"], t["box"],
                                drift_momentum=True)
    geom = lens.MapGeometry(t["npix"], t["fov"], t["z_src"], c)
    ah = 0.5 * (t["a0"] + t["a1"])
    ref = lens.project_shell(x1, t["a0"], t["a1"], c, t["box"], t["np_side"], geom, sub=(p_h, ah))
    plain = lens.project_shell(x1, t["a0"], t["a1"], c, t["box"], t["np_side"], geom)
    return ref, plain


def _thick_wl():
    t = THICK
    return W.Workload("thick", t["np_side"], t["nm"], t["box"], t["a0"], t["a1"], 1, t["npix"],
                      t["fov"], t["z_src"])


def _thick_state():
    t = THICK
    return (W.clustered_positions(t["np_side"], t["nm"], t["box"], seed=51),
            W.random_momenta(t["np_side"] ** 3, 3.0, seed=52))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_thick_shell_step_with_interpolation(dtype):
    """One step from a set state through a thick early shell (many box
    replicas along the line of sight and across a 6 deg field, four source
    planes), then its projection with sub-evolution."""
    t = THICK
    x0, p0 = _thick_state()
    with new_sim(_thick_wl(), dtype) as sim:
        sim.set_interpolation(True)
        sim.set_state(torch.from_numpy(x0), torch.from_numpy(p0), t["a0"])
        sim.step(t["a0"], t["a1"])
        kg = sim.new_maps()
        sim.lens(t["a0"], t["a1"], kg)
        kg = to_np(kg)
        sim.sync()
    log("oracle step and shell")
    ref, plain = _thick_oracle()
    e = rel_rms(kg, ref)
    log(f"thick sub {dtype}: kappa rel-rms {e:.3e}, plain vs sub {rel_rms(plain, ref):.3e}")
    assert rel_rms(plain, ref) > 1e-3
    assert e <= _tol(dtype, 1e-10, 1e-4)


def test_interpolation_error_paths():
    from paper_2012_07266_amd import MadlensError
    from paper_2012_07266_amd._lib import PM_EINVAL, PM_ESTATE
    wl = _run_wl(16, 32, 40.0)
    noise = torch.from_numpy(W.white_noise(16, 3))
    with new_sim(wl) as sim:
        sim.set_interpolation(True)
        kap = sim.new_maps()
        sim.init_ic(noise, 0.2)
        # no step has ended at the shell's end: no drift momentum
        with pytest.raises(MadlensError) as e:
            sim.lens(0.1, 0.2, kap)
        assert e.value.code == PM_ESTATE
        sim.step(0.2, 0.3)
        with pytest.raises(MadlensError) as e:
            sim.lens(0.25, 0.3, kap)    # not the interval of that step
        assert e.value.code == PM_ESTATE
        sim.lens(0.2, 0.3, kap)
        with pytest.raises(MadlensError) as e:
            sim.lens_vjp(0.2, 0.3, torch.ones_like(kap),
                         torch.zeros((3, 16 ** 3), dtype=kap.dtype, device=kap.device),
                         np.zeros(2))
        assert e.value.code == PM_EINVAL
        # off again: the plain projection needs no step
        sim.set_interpolation(False)
        sim.init_ic(noise, 0.2)
        sim.step(0.2, 0.3)
        sim.lens(0.2, 0.3, kap)
        sim.sync()
