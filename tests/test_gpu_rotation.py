"""GPU parity of replica rotation (pm_set_replica_rotation) against the
float64 oracle: every box replica is the box under one of the 48 cube
symmetries, hashed from its offsets and a seed.  Float64 agrees to
round-off; float32 within 1e-4 relative RMS of the maps."""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from paper_2012_07266_amd._lib import PM_MODE_PGD
from tests.gpu_util import cosmo_of, log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
SEED = 0x5EED1234ABCD

# (np, box, npix, fov, z_src, a_far, a_near): a thick early shell with ~13
# replicas along the line of sight and several across the field; a wide
# field through a thin far shell; the last shell, reaching the observer
GEOMETRIES = {
    "thick": (16, 64.0, 48, 6.0, (0.5, 1.0, 1.5, 2.0), 0.45, 0.6),
    "wide": (16, 64.0, 64, 8.0, (1.0, 2.0), 0.33, 0.345),
    "near": (32, 64.0, 48, 6.0, (0.5, 1.0), 0.9, 1.0),
}


def _tol(dtype, f64, f32):
    return f64 if dtype == torch.float64 else f32


@functools.lru_cache(maxsize=None)
def _static_oracle(geometry):
    from oracle import lens
    np_side, box, npix, fov, zs, a_far, a_near = GEOMETRIES[geometry]
    c = cosmo_of(W.Workload("rot", np_side, np_side, box, 0.1, 1.0, 4, npix, fov, zs))
    x = W.clustered_positions(np_side, np_side, box, seed=51)
    rot = lens.project_shell(x, a_far, a_near, c, box, np_side,
                             lens.MapGeometry(npix, fov, zs, c, rotation_seed=SEED))
    plain = lens.project_shell(x, a_far, a_near, c, box, np_side, lens.MapGeometry(npix, fov, zs, c))
    return rot, plain


@pytest.mark.parametrize("geometry", list(GEOMETRIES))
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_rotated_shell_of_static_field(dtype, geometry):
    np_side, box, npix, fov, zs, a_far, a_near = GEOMETRIES[geometry]
    wl = W.Workload("rot", np_side, np_side, box, 0.1, 1.0, 4, npix, fov, zs)
    x = W.clustered_positions(np_side, np_side, box, seed=51)
    log(f"rotated shell {dtype} {geometry}")
    with new_sim(wl, dtype) as sim:
        sim.set_replica_rotation(SEED)
        sim.set_state(torch.from_numpy(x), torch.zeros((3, np_side ** 3), dtype=torch.float64), a_near)
        k = sim.new_maps()
        sim.lens(a_far, a_near, k)
        kg = to_np(k)
        sim.sync()
    log("oracle shell")
    ko, kp = _static_oracle(geometry)
    e = rel_rms(kg, ko)
    log(f"rotated {dtype} {geometry}: kappa rel-rms {e:.2e}, rotated vs not {rel_rms(kp, ko):.2e}")
    assert rel_rms(kp, ko) > 1e-3        # rotation changes the map
    assert e <= _tol(dtype, 1e-10, 1e-4)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_rotated_run_matches_oracle(dtype):
    """A 5-step run with rotation, sub-evolution and PGD all on."""
    from oracle import lens
    wl = W.Workload("rotrun", 16, 32, 40.0, 0.3, 1.0, 5, 64, 3.0, (0.5, 1.0), seed=9)
    c = cosmo_of(wl)
    noise = W.white_noise(16, wl.seed)
    a = wl.a_grid()
    pgd = (0.5, 0.5, 0.05, 1.5)
    log(f"rotated run {dtype}")
    with new_sim(wl, dtype, modes=PM_MODE_PGD) as sim:
        sim.set_replica_rotation(SEED)
        sim.set_interpolation(True)
        sim.set_pgd(*pgd)
        kg = to_np(sim.run(torch.from_numpy(noise), a))
        sim.sync()
    log("oracle run")
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c, rotation_seed=SEED)
    kap, _, _ = lens.run_lensing(noise, c, 40.0, 32, a, geom, interpolation=True, pgd=pgd)
    e = rel_rms(kg, kap)
    log(f"rotated run {dtype}: kappa rel-rms {e:.3e}")
    assert e <= _tol(dtype, 1e-10, 1e-4)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_rotated_lens_vjp(dtype):
    """The lens VJP with rotation: position cotangents against the oracle's
    adjoint (itself pinned against finite differences)."""
    from oracle import adjoint, lens
    wl = W.Workload("rotvjp", 16, 32, 64.0, 0.4, 1.0, 3, 24, 4.0, (1.0, 2.0))
    c = cosmo_of(wl)
    x = W.clustered_positions(16, 32, wl.box, seed=21)
    kbar = np.random.default_rng(22).standard_normal((2, 24, 24))
    a_far, a_near = 0.55, 0.7
    log(f"rotated lens vjp {dtype}")
    with new_sim(wl, dtype) as sim:
        sim.set_replica_rotation(SEED)
        sim.set_state(torch.from_numpy(x), torch.zeros((3, 16 ** 3), dtype=torch.float64), a_near)
        xb = torch.zeros((3, 16 ** 3), dtype=dtype, device="cuda")
        cb = np.zeros(2)
        sim.lens_vjp(a_far, a_near, torch.tensor(kbar, dtype=dtype, device="cuda"), xb, cb)
        xg = to_np(xb)
        sim.sync()
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c, rotation_seed=SEED)
    xo = adjoint.lens_vjp(x, a_far, a_near, kbar, c, wl.box, 16, geom)
    plain = adjoint.lens_vjp(x, a_far, a_near, kbar, c, wl.box, 16,
                             lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c))
    e = rel_rms(xg, xo)
    log(f"rotated lens vjp {dtype}: x rel-rms {e:.2e}, rotated vs not {rel_rms(plain, xo):.2e}")
    assert rel_rms(plain, xo) > 1e-3
    assert e < _tol(dtype, 1e-9, 1e-4)


def test_rotation_off_restores_the_plain_projection():
    np_side, box, npix, fov, zs, a_far, a_near = GEOMETRIES["near"]
    wl = W.Workload("rot", np_side, np_side, box, 0.1, 1.0, 4, npix, fov, zs)
    x = torch.from_numpy(W.clustered_positions(np_side, np_side, box, seed=51))
    with new_sim(wl, torch.float32) as sim:
        sim.set_state(x, torch.zeros_like(x), a_near)
        k0 = sim.new_maps()
        sim.lens(a_far, a_near, k0)
        sim.set_replica_rotation(SEED)
        k1 = sim.new_maps()
        sim.lens(a_far, a_near, k1)
        sim.set_replica_rotation(None)
        k2 = sim.new_maps()
        sim.lens(a_far, a_near, k2)
        sim.sync()
        assert torch.equal(k0, k2)
        assert not torch.equal(k0, k1)
