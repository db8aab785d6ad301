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


def _exact_grid(v, cell):
    """v rounded to a multiple of cell / 64 (for the box and cell below such
    values, their sums with the box and their quotients by the cell are
    exact in float32)."""
    return np.round(v / cell * 64.0) * (cell / 64.0)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("copy", [(205.0, 256, 512), (192.0, 192, 384)],
                         ids=["1024m_from_512m", "768m_from_384m"])
def test_largest_mesh_replicated_configuration(copy):
    """The largest meshes (1024^3 with 512^3 particles; 768^3 with 384^3,
    radix 3), float32, against the path at half their size: a configuration
    repeated 2 x 2 x 2 in a box twice as large has, node for node and
    particle for particle, the density, the force and the step of one copy.
    (The transform of the repeated field lives on even modes, where the
    doubled box's Green's function equals the original's.)  Positions and
    momenta sit on a 1/64-cell grid, so both sides get bit-identical CIC
    weights and differ only in FFT rounding.  The copies (512^3 and 384^3
    meshes) are themselves held against the oracle in test_gpu_parity.py."""
    L, np_s, nm_s = copy
    cell = L / nm_s
    n = np_s ** 3
    x = _exact_grid(W.clustered_positions(np_s, nm_s, L, seed=66), cell)
    x = np.mod(x, L)
    p = _exact_grid(W.random_momenta(n, 1.0, seed=67), cell)
    a0, a1 = 0.5, 0.52
    log(f"edge replicated: {np_s}^3/{nm_s}^3 copy")
    with new_sim(_wl(np_s, nm_s, L), torch.float32) as sim:
        sim.set_state(torch.from_numpy(x.astype(np.float32)),
                      torch.from_numpy(p.astype(np.float32)), a0)
        rho_s, fm_s, acc_s = sim.get_force()
        sim.step(a0, a1)
        xs, ps = sim.get_state()
        sim.sync()
    x32, p32 = x.astype(np.float32), p.astype(np.float32)
    xb = np.empty((3, 8 * n), dtype=np.float32)
    for c in range(8):
        off = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1], dtype=np.float32)[:, None] * L
        xb[:, c * n:(c + 1) * n] = x32 + off
    pb = np.tile(p32, (1, 8))
    log(f"edge replicated: {2 * np_s}^3/{2 * nm_s}^3 repeated")
    with new_sim(_wl(2 * np_s, 2 * nm_s, 2 * L), torch.float32) as sim:
        sim.set_state(torch.from_numpy(xb), torch.from_numpy(pb), a0)
        del xb, pb
        rho_b, fm_b, acc_b = sim.get_force()
        fmax = float(fm_s.abs().max())
        rho_same = True
        e_f = 0.0
        for c in range(8):
            i, j, k = ((c >> 2) & 1) * nm_s, ((c >> 1) & 1) * nm_s, (c & 1) * nm_s
            rho_same &= bool(torch.equal(rho_b[i:i + nm_s, j:j + nm_s, k:k + nm_s], rho_s))
            d = fm_b[:, i:i + nm_s, j:j + nm_s, k:k + nm_s] - fm_s
            e_f = max(e_f, float(d.abs().max()) / fmax)
            del d
        del rho_b, fm_b
        e_acc = max(float((acc_b[:, c * n:(c + 1) * n] - acc_s).abs().max())
                    for c in range(8)) / fmax
        sim.step(a0, a1)
        xb_g, pb_g = sim.get_state()
        sim.sync()
        e_x = 0.0
        e_x_rms = 0.0
        for c in range(8):
            d = torch.remainder(xb_g[:, c * n:(c + 1) * n] - xs + 0.5 * L, L) - 0.5 * L
            e_x = max(e_x, float(d.abs().max()) / cell)
            e_x_rms = max(e_x_rms, float(d.double().pow(2).mean().sqrt()) / cell)
        ps64 = ps.double()
        e_p = max(float((pb_g[:, c * n:(c + 1) * n].double() - ps64).pow(2).mean().sqrt()
                        / ps64.pow(2).mean().sqrt()) for c in range(8))
    log(f"edge replicated: rho bitwise {rho_same}, force max {e_f:.2e}, acc max {e_acc:.2e}, "
        f"step pos max {e_x:.2e} rms {e_x_rms:.2e} cells, mom rel-rms {e_p:.2e}")
    assert rho_same
    assert e_f <= 2e-5
    assert e_acc <= 2e-5
    assert e_x_rms <= 1e-4 and e_x <= 1e-3
    assert e_p <= 1e-4
