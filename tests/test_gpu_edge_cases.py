"""GPU parity on degenerate inputs: most of the mass in one point, every
particle on a mesh node (half of them on tile faces), and a lens shell that
holds no particle.  The HIP path through the C ABI against the float64
oracle, to the tolerances of the other parity tests."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import cosmo_of, log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]
# cell sizes 2, 1.25, 2 and 0.5: node positions k * cell are exact in
# float32.  16^3/16^3 is the smallest mesh: one tile, its own neighbour on
# every side.
SHAPES = [(16, 16, 32.0), (16, 32, 40.0), (32, 32, 64.0), (128, 256, 128.0)]


def _tol(dtype, f64, f32):
    return f64 if dtype == torch.float64 else f32


def _field(kind, np_side, nm, box, seed):
    """[3][Np^3] positions in [0, box).

    point: three quarters of the particles at one off-node point (one 2x2x2
    corner set receives most of the mass; one sort key holds most of the
    particles), the rest uniform.
    nodes: every particle exactly on a mesh node, half of them on a tile's
    low face along one axis (tile = 16 cells), some at the origin."""
    n = np_side ** 3
    gen = np.random.Generator(np.random.Philox(key=seed))
    if kind == "point":
        x = gen.uniform(0.0, box, size=(3, n))
        p0 = np.array([0.37, 0.61, 0.83]) * box + 0.3 * box / nm
        x[:, : 3 * n // 4] = np.mod(p0, box)[:, None]
        return x
    cell = box / nm
    k = gen.integers(0, nm, size=(3, n))
    face = gen.random(n) < 0.5
    axis = gen.integers(0, 3, size=n)
    f = np.nonzero(face)[0]
    k[axis[f], f] = 16 * gen.integers(0, nm // 16, size=f.size)
    k[:, :17] = 0
    return k * cell


def _wl(np_side, nm, box):
    return W.Workload(f"e{np_side}_{nm}", np_side, nm, box, 0.1, 1.0, 4, 32, 2.0, (1.0,))


@pytest.mark.parametrize("kind", ["point", "nodes"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}p{s[1]}m")
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_degenerate_density_force_readout(dtype, shape, kind):
    from oracle import pm
    np_side, nm, box = shape
    log(f"edge density/force {kind} {shape} {dtype}")
    x = _field(kind, np_side, nm, box, seed=61)
    p = W.random_momenta(np_side ** 3, 1.0, seed=62)
    with new_sim(_wl(np_side, nm, box), dtype) as sim:
        sim.set_state(torch.from_numpy(x), torch.from_numpy(p), 0.5)
        rho_g, fm_g, acc_g = (to_np(t) for t in sim.get_force())
        sim.sync()
    rho = pm.density(x, np_side, nm, box)
    f = pm.force_mesh(rho, box)
    acc = np.stack([pm.cic_readout(x, f[j], box) for j in range(3)])
    fmax = np.max(np.abs(f))
    e_rho = np.max(np.abs(rho_g - rho)) / np.max(rho)
    e_f = rel_rms(fm_g, f)
    # at the point the eight corner forces largely cancel: measure the
    # readout against the largest force, not against its own size
    e_acc = np.max(np.abs(acc_g - acc)) / fmax
    log(f"edge {kind} {shape} {dtype}: rho {e_rho:.2e} force rms {e_f:.2e} acc max {e_acc:.2e}")
    assert abs(rho_g.sum() - nm ** 3) < _tol(dtype, 1e-9, 1e-3) * nm ** 3
    assert e_rho <= _tol(dtype, 1e-12, 2e-5)
    assert e_f <= _tol(dtype, 1e-12, 2e-5)
    assert e_acc <= _tol(dtype, 1e-12, 1e-4)


@pytest.mark.parametrize("shape", [(16, 16, 32.0), (32, 32, 64.0)], ids=lambda s: f"{s[0]}p{s[1]}m")
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_step_from_node_field(dtype, shape):
    """One KDK step from particles that all sit on mesh nodes (their CIC
    weights are 0 and 1, and a step's first readout is at those nodes)."""
    from oracle import pm
    np_side, nm, box = shape
    wl = _wl(np_side, nm, box)
    c = cosmo_of(wl)
    x = _field("nodes", np_side, nm, box, seed=63)
    p = W.random_momenta(np_side ** 3, 0.05, seed=64)
    a0, a1 = 0.5, 0.55
    log(f"edge step nodes {shape} {dtype}")
    with new_sim(wl, dtype) as sim:
        sim.set_state(torch.from_numpy(x), torch.from_numpy(p), a0)
        sim.step(a0, a1)
        xg, pg = (to_np(t) for t in sim.get_state())
        sim.sync()
    f0 = pm.particle_force(x, np_side, nm, box)
    xo, po, _ = pm.kdk_step(x, p, f0, a0, a1, c, np_side, nm, box)
    d = np.mod(xg - xo + 0.5 * box, box) - 0.5 * box
    err = np.max(np.abs(d)) / (box / nm)
    log(f"edge step nodes {shape} {dtype}: pos max {err:.2e} cells, mom rel-rms {rel_rms(pg, po):.2e}")
    assert err <= _tol(dtype, 1e-10, 1e-4)
    assert rel_rms(pg, po) <= _tol(dtype, 1e-10, 1e-4)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_empty_lens_shell(dtype):
    """A thin shell with no particle in its depth range: every pixel gets
    the mean term alone."""
    from oracle import lens
    np_side, box, npix, fov, zs = 16, 64.0, 48, 6.0, (1.5, 2.0)
    a_far, a_near = 0.5, 0.5005
    wl = W.Workload("empty", np_side, np_side, box, 0.1, 1.0, 4, npix, fov, zs)
    c = cosmo_of(wl)
    chi_near, chi_far = float(c.chi(a_near)), float(c.chi(a_far))
    assert chi_far - chi_near < 0.25 * box
    # depths x_2 + j box avoid [chi_near - 1, chi_far + 1] for every j
    lo = np.mod(chi_far + 1.0, box)
    width = box - (chi_far - chi_near) - 2.0
    x = W.random_positions(np_side ** 3, box, seed=65)
    x[2] = np.mod(lo + np.mod(x[2], width), box)
    geom = lens.MapGeometry(npix, fov, zs, c)
    ko = lens.project_shell(x, a_far, a_near, c, box, np_side, geom)
    kp = lens.project_shell(x, a_far, a_near, c, box, np_side, geom, include_mean=False)
    assert np.all(kp == 0.0) and np.all(ko < 0.0)
    log(f"edge empty shell {dtype}")
    with new_sim(wl, dtype) as sim:
        sim.set_state(torch.from_numpy(x), torch.zeros((3, np_side ** 3), dtype=torch.float64),
                      a_near)
        k = sim.new_maps()
        sim.lens(a_far, a_near, k)
        kg = to_np(k)
        sim.sync()
    e = rel_rms(kg, ko)
    log(f"edge empty shell {dtype}: kappa rel-rms {e:.2e}")
    assert e <= _tol(dtype, 1e-10, 1e-5)
