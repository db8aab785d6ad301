"""GPU parity: the HIP path through the C ABI against the float64 oracle.

Float64 instantiations must agree to round-off (1e-10 relative or better);
float32 ones to the stated tolerances: positions within 1e-4 of a mesh cell,
convergence maps within 1e-4 relative RMS.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import cosmo_of, log, new_sim, periodic_cells, rel_rms, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
# (Np, Nm, box): B = 2 with 2^3 tiles, B = 1, radix-3 lengths (48, 96), and
# 128/256, whose strided passes take the register-resident FFT path
SHAPES = [(16, 32, 40.0), (32, 32, 64.0), (48, 96, 100.0), (128, 256, 128.0)]


def _wl(np_side, nm, box, **kw):
    return W.Workload(f"t{np_side}_{nm}", np_side, nm, box, 0.1, 1.0, 4, 32, 2.0, (1.0,), **kw)


def _tol(dtype, f64, f32):
    return f64 if dtype == torch.float64 else f32


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_background_tables(dtype):
    wl = _wl(16, 32, 40.0)
    c = cosmo_of(wl)
    with new_sim(wl, dtype) as sim:
        for a in (0.01, 0.1, 0.5, 0.97):
            d, g, chi = sim.background(a)
            assert abs(d - c.D(a)) < 1e-12 * c.D(a)
            assert abs(g - c.gp(a)) < 1e-12 * c.gp(a)
            assert abs(chi - c.chi(a)) < 1e-11 * c.chi(a)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}p{s[1]}m")
def test_density_force_readout(dtype, shape):
    from oracle import pm
    np_side, nm, box = shape
    log(f"density/force {shape} {dtype}")
    wl = _wl(np_side, nm, box)
    x = W.clustered_positions(np_side, nm, box, seed=31)
    p = W.random_momenta(np_side ** 3, 1.0, seed=32)
    with new_sim(wl, dtype) as sim:
        sim.set_state(torch.from_numpy(x), torch.from_numpy(p), 0.5)
        rho_g, fm_g, acc_g = (to_np(t) for t in sim.get_force())
        sim.sync()
    rho = pm.density(x, np_side, nm, box)
    f = pm.force_mesh(rho, box)
    acc = np.stack([pm.cic_readout(x, f[j], box) for j in range(3)])
    # float32: positions are rounded to float32 on the way in (about 1e-5 of a
    # cell for coordinates of ~100 cells), which moves each CIC weight by up
    # to that much; clumps of thousands of particles add these up.
    e_rho = np.max(np.abs(rho_g - rho)) / np.max(rho)
    e_f = rel_rms(fm_g, f)
    e_fmax = np.max(np.abs(fm_g - f)) / np.max(np.abs(f))
    e_acc = rel_rms(acc_g, acc)
    log(f"{shape} {dtype}: rho {e_rho:.2e} force rms {e_f:.2e} max {e_fmax:.2e} acc {e_acc:.2e}")
    assert abs(rho_g.sum() - nm ** 3) < _tol(dtype, 1e-9, 1e-3) * nm ** 3
    assert e_rho <= _tol(dtype, 1e-12, 2e-5)
    assert e_f <= _tol(dtype, 1e-12, 2e-5)
    assert e_fmax <= _tol(dtype, 1e-12, 1e-4)
    assert e_acc <= _tol(dtype, 1e-12, 2e-5)


# Radix-3 lengths of the serving sizes and of the 768^3 mesh: meshes of 192
# and 384 (float32 only: the float64 instantiation stops at 256).
RADIX3_SHAPES = [(96, 192, 120.0), (192, 384, 192.0)]


@pytest.mark.parametrize("shape", RADIX3_SHAPES, ids=lambda s: f"{s[0]}p{s[1]}m")
def test_density_force_readout_radix3_lengths(shape):
    test_density_force_readout(torch.float32, shape)


@pytest.mark.parametrize("shape", [(192, 384, 192.0), (384, 768, 384.0)],
                         ids=lambda s: f"{s[0]}p{s[1]}m")
def test_zeldovich_ic_radix3_lengths(shape):
    """Initial conditions transformed on the particle lattice at lengths 192
    and 384 (the 768^3 mesh's lattice), float32."""
    test_zeldovich_ic(torch.float32, shape)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 32, 40.0), (32, 32, 64.0), (48, 96, 100.0)],
                         ids=lambda s: f"{s[0]}p{s[1]}m")
def test_zeldovich_ic(dtype, shape):
    from oracle import pm
    np_side, nm, box = shape
    log(f"ic {shape} {dtype}")
    wl = _wl(np_side, nm, box)
    c = cosmo_of(wl)
    noise = W.white_noise(np_side, 41)
    a0 = 0.2
    with new_sim(wl, dtype) as sim:
        sim.init_ic(torch.from_numpy(noise), a0)
        xg, pg = (to_np(t) for t in sim.get_state())
        sim.sync()
    x, p = pm.zeldovich_ic(noise, c, box, nm, a0)
    err = periodic_cells(xg - x, box, nm)
    log(f"ic {shape} {dtype}: pos max {err.max():.2e} cells, mom rel-rms {rel_rms(pg, p):.2e}")
    # float32 output positions alone carry half an ulp of the box coordinate
    # (1.5e-5 Mpc/h = 3e-5 cells for coordinates in [256, 384) on the 768^3
    # mesh), on top of the displacement's own rounding
    half_ulp = 0.5 * float(np.spacing(np.float32(box))) / (box / nm)
    assert err.max() <= _tol(dtype, 1e-10, max(2e-5, half_ulp + 1e-5))
    assert rel_rms(pg, p) <= _tol(dtype, 1e-12, 1e-5)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_cfg1_positions_and_kappa(dtype):
    """The full 32^3 / 32^3, 5-step run with its 64^2 map at z_s = 1."""
    from oracle import lens
    wl = W.CFG1
    log(f"cfg1 full run {dtype}")
    c = cosmo_of(wl)
    noise = W.white_noise(wl.np_side, wl.seed)
    a = wl.a_grid()
    with new_sim(wl, dtype) as sim:
        kap_g = to_np(sim.run(torch.from_numpy(noise), a))
        xg, pg = (to_np(t) for t in sim.get_state())
        sim.sync()
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    kap, x, p = lens.run_lensing(noise, c, wl.box, wl.nm_side, a, geom)
    err = periodic_cells(xg - x, wl.box, wl.nm_side)
    log(f"cfg1 {dtype}: pos max {err.max():.3e} rms {np.sqrt((err**2).mean()):.3e} cells; "
        f"kappa rel-rms {rel_rms(kap_g, kap):.3e}")
    assert err.max() <= _tol(dtype, 1e-8, 1e-4)
    assert rel_rms(pg, p) <= _tol(dtype, 1e-10, 1e-4)
    assert rel_rms(kap_g, kap) <= _tol(dtype, 1e-10, 1e-4)


LENS_GEOMETRIES = {
    # thick early shell: ~13 box replicas along the line of sight, several
    # across the 6 deg field, four source planes
    "thick": (32, 64.0, 48, 6.0, (0.5, 1.0, 1.5, 2.0), 0.45, 0.6),
    # 8 deg field through a thin shell that straddles z_s = 2 and lies behind
    # z_s = 1: ~8 transverse replicas per axis at the far edge
    "wide": (16, 64.0, 64, 8.0, (1.0, 2.0), 0.33, 0.345),
    # the last shell, reaching the observer
    "near": (32, 64.0, 48, 6.0, (0.5, 1.0), 0.9, 1.0),
    # a 256^2 map: 64 x 64-pixel regions with 1024-thread workgroups
    "regions64": (16, 64.0, 256, 4.0, (1.0, 2.0), 0.5, 0.6),
    # six source planes, one in front of the shell, one inside and four
    # beyond it: those four share two accumulators, which lets the regions
    # grow to 64 x 64 pixels (six accumulators would need 32 x 32)
    "many": (16, 64.0, 256, 4.0, (0.3, 0.6, 1.0, 1.4, 1.8, 2.2), 0.6, 0.7),
    # the same planes, a shell around z_s = 1.8: one plane beyond it, one
    # inside, four in front, so A and B serve one plane
    "many_one_beyond": (16, 64.0, 256, 4.0, (0.3, 0.6, 1.0, 1.4, 1.8, 2.2), 0.35, 0.365),
    # a shell around the farthest plane: none beyond it (A and B unused)
    "many_none_beyond": (16, 64.0, 256, 4.0, (0.3, 0.6, 1.0, 1.4, 1.8, 2.2), 0.305, 0.32),
}


@functools.lru_cache(maxsize=None)
def _lens_oracle(geometry):
    """Oracle maps (with and without the mean term) of a geometry's shell."""
    from oracle import lens
    np_side, box, npix, fov, zs, a_far, a_near = LENS_GEOMETRIES[geometry]
    c = cosmo_of(W.Workload("lens", np_side, np_side, box, 0.1, 1.0, 4, npix, fov, zs))
    x = W.clustered_positions(np_side, np_side, box, seed=51)
    geom = lens.MapGeometry(npix, fov, zs, c)
    return (lens.project_shell(x, a_far, a_near, c, box, np_side, geom),
            lens.project_shell(x, a_far, a_near, c, box, np_side, geom, include_mean=False))


@pytest.mark.parametrize("geometry", list(LENS_GEOMETRIES))
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_lens_shell_of_static_field(dtype, geometry):
    """One shell of a static particle field against the oracle.  Clustered
    particles, so the map is not a cancellation of the particle and mean
    terms; float32 is also held to 1e-5 of the particle term alone (rounding
    of ~10^4 atomic additions per pixel)."""
    np_side, box, npix, fov, zs, a_far, a_near = LENS_GEOMETRIES[geometry]
    wl = W.Workload("lens", np_side, np_side, box, 0.1, 1.0, 4, npix, fov, zs)
    c = cosmo_of(wl)
    x = W.clustered_positions(np_side, np_side, wl.box, seed=51)
    p = np.zeros_like(x)
    log(f"lens static {dtype} {geometry}")
    with new_sim(wl, dtype) as sim:
        sim.set_state(torch.from_numpy(x), torch.from_numpy(p), a_near)
        k = sim.new_maps()
        sim.lens(a_far, a_near, k)
        kg = to_np(k)
        sim.sync()
    ko, kp = _lens_oracle(geometry)
    e_tot = rel_rms(kg, ko)
    e_part = float(np.sqrt(np.mean((kg - ko) ** 2) / np.mean(kp ** 2)))
    log(f"lens static {dtype}: kappa rel-rms {e_tot:.2e}, vs particle term {e_part:.2e}")
    assert e_tot <= _tol(dtype, 1e-10, 1e-4)
    assert e_part <= _tol(dtype, 1e-12, 1e-5)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}p{s[1]}m")
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_fused_run_equals_step_and_lens(dtype, shape):
    """pm_run (each readout also starts the next step; shells projected after
    the paint) gives the maps and state of pm_step + lens_project per
    interval: bit for bit in float32, whose paint and projection accumulate
    in fixed point; to round-off in float64, whose LDS accumulators are
    float64 atomics and so depend on the order of arrival."""
    np_side, nm, box = shape
    wl = W.Workload("fused", np_side, nm, box, 0.2, 1.0, 5, 64, 4.0, (1.0, 1.5), seed=9)
    log(f"fused run vs stepwise {dtype} np={np_side} nm={nm}")
    noise = torch.from_numpy(W.white_noise(np_side, wl.seed))
    a = wl.a_grid()
    with new_sim(wl, dtype) as sim:
        k1 = sim.run_stepwise(noise, a).clone()
        x1, p1 = (t.clone() for t in sim.get_state())
        k2 = sim.run(noise, a)
        x2, p2 = sim.get_state()
        sim.sync()
        assert torch.abs(k1).max() > 0
        if dtype == torch.float32:
            assert torch.equal(k1, k2) and torch.equal(x1, x2) and torch.equal(p1, p2)
        else:
            assert rel_rms(to_np(k2), to_np(k1)) < 1e-12 and rel_rms(to_np(p2), to_np(p1)) < 1e-12
            assert periodic_cells(to_np(x2) - to_np(x1), box, nm).max() < 1e-10


def test_error_paths():
    from paper_2012_07266_amd import MadlensError
    from paper_2012_07266_amd._lib import PM_ESTATE, PM_ENONFINITE
    wl = _wl(16, 32, 40.0)
    with new_sim(wl) as sim:
        with pytest.raises(MadlensError) as e:
            sim.step(0.1, 0.2)          # no state yet
        assert e.value.code == PM_ESTATE
        sim.init_ic(torch.from_numpy(W.white_noise(16, 1)), 0.1)
        with pytest.raises(MadlensError) as e:
            sim.step(0.3, 0.4)          # state is at 0.1
        assert e.value.code == PM_ESTATE
        sim.sync()
        # a non-finite position forced from the host is reported, not hidden
        x = torch.from_numpy(W.random_positions(16 ** 3, 40.0, seed=2))
        x[1, 77] = float("nan")
        sim.set_state(x, torch.zeros_like(x), 0.2)
        with pytest.raises(MadlensError) as e:
            sim.sync()
        assert e.value.code == PM_ENONFINITE


def _off_shell_bounds(x, box, cell, bounds, gap):
    """x with axis-2 coordinates moved, where needed, to at least `gap` from
    every distance in `bounds` modulo the box (the depth of an image is
    x_2 plus a multiple of the box)."""
    x = x.copy()
    for b in bounds:
        zb = np.mod(b, box)
        d = np.mod(x[2] - zb + 0.5 * box, box) - 0.5 * box
        near = np.abs(d) < gap
        x[2, near] = np.mod(zb + np.where(d[near] < 0, -gap, gap), box)
    return x


@pytest.mark.timeout(900)
def test_full_size_step_and_shell():
    """The benchmark's size and launch path: 256^3 particles, 512^3 mesh,
    box 205 Mpc/h, four 2048^2 maps over 5 deg, float32.  Zel'dovich initial
    conditions at a = 0.01 and one pm_run step (a -> 0.03475) against the
    float64 oracle at every particle; then the particles of that state,
    placed at a = 0.51 and kept 0.01 cells off the shell boundaries,
    projected over the thin shell (0.5, 0.51] (just in front of z_s = 1;
    transverse replicas for the farther sources) against the oracle's full
    maps."""
    from oracle import lens, pm
    wl = W.CFG2
    c = cosmo_of(wl)
    a = wl.a_grid()
    noise = W.white_noise(wl.np_side, wl.seed)
    log("full size: GPU IC + one step + shell")
    with new_sim(wl, torch.float32) as sim:
        k = sim.new_maps()
        sim.init_ic(torch.from_numpy(noise), a[0])
        sim.steps(a[:2], k)
        xg, pg = (to_np(t) for t in sim.get_state())
        # shell membership is decided in the kernels' precision: keep every
        # image 0.01 cells off both shell boundaries, so that float32 and the
        # float64 oracle place each one on the same side
        xl = _off_shell_bounds(xg, wl.box, wl.box / wl.nm_side,
                               (c.chi(0.51), c.chi(0.5)), 0.01 * wl.box / wl.nm_side)
        xl = xl.astype(np.float32).astype(np.float64)
        xs = torch.from_numpy(xl)
        sim.set_state(xs, torch.zeros_like(xs), 0.51)
        kl = sim.new_maps()
        sim.lens(0.5, 0.51, kl)
        klg = to_np(kl)
        sim.sync()
    log("full size: oracle IC + step")
    x0, p0 = pm.zeldovich_ic(noise, c, wl.box, wl.nm_side, a[0])
    f0 = pm.particle_force(x0, wl.np_side, wl.nm_side, wl.box)
    x1, p1, _ = pm.kdk_step(x0, p0, f0, a[0], a[1], c, wl.np_side, wl.nm_side, wl.box)
    err = periodic_cells(xg - x1, wl.box, wl.nm_side)
    e_p = rel_rms(pg, p1)
    log(f"full size step: pos max {err.max():.2e} rms {np.sqrt((err ** 2).mean()):.2e} cells, "
        f"mom rel-rms {e_p:.2e}")
    assert np.sqrt((err ** 2).mean()) < 1e-4 and err.max() < 1e-3 and e_p < 1e-4
    log("full size: oracle shell")
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    ko = lens.project_shell(xl, 0.5, 0.51, c, wl.box, wl.np_side, geom)
    e_k = rel_rms(klg, ko)
    log(f"full size shell: kappa rel-rms {e_k:.2e}")
    assert np.abs(ko).max() > 0 and e_k < 1e-4


def test_profile_only_records_one_kernel():
    """pm_profile_only limits the event pairs to one kernel name: a fused
    5-step run records every kernel when unrestricted, and only the paint
    (six launches: the initial force and one per step) when restricted to
    it; the maps are the same either way."""
    wl = W.Workload("prof", 16, 32, 40.0, 0.2, 1.0, 5, 64, 4.0, (1.0,), seed=9)
    log("profile_only: 16^3/32^3, 5 steps")
    noise = torch.from_numpy(W.white_noise(16, wl.seed))
    a = wl.a_grid()
    with new_sim(wl) as sim:
        sim.profile(True)
        k1 = sim.run(noise, a).clone()
        every = sim.profile_read()
        sim.profile_only("paint")
        k2 = sim.run(noise, a)
        only = sim.profile_read()
        sim.profile(False)
        sim.profile_only(None)
        sim.sync()
    assert len(every) > 3 and every["paint"][1] == 6
    assert only.get("paint", (0.0, 0))[1] == 6
    assert all(c == 0 for n, (_, c) in only.items() if n != "paint")
    assert only["paint"][0] > 0.0
    assert torch.equal(k1, k2)
