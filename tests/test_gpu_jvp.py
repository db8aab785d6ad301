"""GPU forward-mode tangents (pm_init_ic_jvp, pm_set_tangent / pm_get_tangent,
pm_step_jvp, lens_project_jvp) against the oracle's hand-derived tangents (oracle/jvp.py,
pinned by finite differences), and the transpose identity with the GPU
reverse pass at the gradient workload's full size."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2012_07266_amd._lib import PM_MODE_PGD, PM_MODE_TANGENT
from tests.gpu_util import cosmo_of, log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


def _off_node_planes(x, box, nm, gap=1e-3):
    """x moved, where needed, to at least `gap` cells from every mesh-node
    plane: the CIC derivative jumps there, so a position within an ulp of
    one has two valid tangents."""
    u = x * (nm / box)
    r = np.round(u)
    f = u - r
    f = np.where(np.abs(f) < gap, np.where(f < 0, -gap, gap), f)
    return np.mod((r + f) * (box / nm), box)


def _rd(dtype):
    """Rounding of host inputs to the device precision (both sides get the
    same values)."""
    if dtype == torch.float32:
        return lambda v: v.astype(np.float32).astype(np.float64)
    return lambda v: v


PIECE_SHAPES = [(16, 32, 48.0), (48, 96, 100.0), (128, 256, 128.0)]


@pytest.mark.parametrize("shape", PIECE_SHAPES, ids=lambda s: f"{s[0]}p{s[1]}m")
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_force_and_step_tangents_match_oracle(dtype, shape):
    """The force tangent at a state, then one step's tangent (Omega_m part
    on), element by element: meshes of one tile, several tiles with a
    mixed-radix FFT, and the gradient workload's 256^3."""
    from oracle import jvp, pm
    np_side, nm, box = shape
    wl = W.Workload("jvp", np_side, nm, box, 0.4, 1.0, 3, 16, 3.0, (1.0,), seed=11)
    log(f"force/step tangents {dtype} np={np_side} nm={nm}")
    c = cosmo_of(wl)
    a = wl.a_grid()
    rd = _rd(dtype)
    noise = W.white_noise(np_side, wl.seed)
    x0, p0 = pm.zeldovich_ic(noise, c, box, nm, a[0])
    x0 = rd(_off_node_planes(x0, box, nm))
    p0 = rd(p0)
    rng = np.random.default_rng(41)
    xd0 = rd(rng.standard_normal((3, wl.n_particles)))
    pd0 = rd(rng.standard_normal((3, wl.n_particles)))
    om_dot = 0.7
    with new_sim(wl, dtype, modes=PM_MODE_TANGENT) as sim:
        T = lambda v: torch.tensor(v, dtype=dtype, device="cuda")
        sim.set_state(T(x0), T(p0), a[0])
        sim.set_tangent(T(xd0), T(pd0), om_dot)
        f0g = to_np(sim.get_tangent()[2])
        sim.step_jvp(a[0], a[1])
        xg, pg, fg = sim.get_tangent()
        x1g, _ = sim.get_state()
        res = (to_np(xg), to_np(pg), to_np(fg), to_np(x1g))
        sim.sync()
    log("oracle")
    f0 = pm.particle_force(x0, np_side, nm, box)
    f0d = jvp.force_jvp(x0, xd0, np_side, nm, box)
    x1, p1, f1, x1d, p1d, f1d = jvp.step_jvp(x0, p0, f0, xd0, pd0, f0d, a[0], a[1], om_dot, c,
                                            np_side, nm, box)
    tol = 1e-9 if dtype == torch.float64 else 3e-5
    # The step's end positions are the device's own: in float32 they differ
    # from the oracle's by up to ~1e-5 cells, which puts a few particles (a
    # dozen of 2M at 128^3) on the other side of a mesh-node plane, where the
    # CIC derivative jumps (both one-sided tangents are valid).  Their own
    # tangents are compared only in float64 (the mask comes from the
    # oracle's positions); their tangent-paint deposits still reach their
    # neighbours' force tangents through the Poisson solve, which leaves
    # float32 p1_dot and f1_dot ~1e-4 off at 128^3 (float64 agrees to 1e-9).
    u = x1 * (nm / box)
    clear = np.all(np.abs(u - np.round(u)) > 1e-3, axis=0) if dtype == torch.float32 \
        else np.ones(x1.shape[1], bool)
    e = [rel_rms(f0g, f0d), rel_rms(res[0], x1d), rel_rms(res[1][:, clear], p1d[:, clear]),
         rel_rms(res[2][:, clear], f1d[:, clear])]
    dx = np.abs(np.mod(res[3] - x1 + 0.5 * box, box) - 0.5 * box).max() / (box / nm)
    log(f"tangents {dtype} {shape}: f0_dot {e[0]:.2e} x1_dot {e[1]:.2e} p1_dot {e[2]:.2e} "
        f"f1_dot {e[3]:.2e} ({clear.mean():.4f} of particles compared; state max |dx| "
        f"{dx:.1e} cells)")
    assert dx < (1e-9 if dtype == torch.float64 else 1e-4)
    assert e[0] < tol and e[1] < tol
    assert e[2] < (1e-8 if dtype == torch.float64 else 1e-3)
    assert e[3] < (1e-8 if dtype == torch.float64 else 1e-3)


@pytest.mark.parametrize("seed", [None, 0x5EED1234ABCD], ids=["plain", "rotated"])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_lens_tangent_of_static_field(dtype, seed):
    """One shell's tangent at fixed positions, along a position tangent and
    Omega_m (weights, source distance, a(chi), mean term; shell bounds and
    source membership held)."""
    from oracle import jvp, lens
    wl = W.Workload("lensjvp", 16, 32, 64.0, 0.4, 1.0, 3, 24, 4.0, (1.0, 2.0))
    c = cosmo_of(wl)
    x = W.clustered_positions(16, 32, wl.box, seed=21)
    xd = np.random.default_rng(42).standard_normal(x.shape)
    a_far, a_near = 0.55, 0.7
    om_dot = 0.6
    log(f"lens tangent {dtype} rotation={seed}")
    with new_sim(wl, dtype, modes=PM_MODE_TANGENT) as sim:
        if seed is not None:
            sim.set_replica_rotation(seed)
        sim.set_state(torch.from_numpy(x), torch.zeros((3, 16 ** 3), dtype=torch.float64), a_near)
        xdg = torch.tensor(xd, dtype=dtype, device="cuda")
        zero = torch.zeros_like(xdg)
        kd = sim.new_maps()
        sim.set_tangent(xdg, zero, om_dot)
        sim.lens_jvp(a_far, a_near, kd)
        kdx = sim.new_maps()
        sim.set_tangent(xdg, zero, 0.0)
        sim.lens_jvp(a_far, a_near, kdx)
        kg, kgx = to_np(kd), to_np(kdx)
        sim.sync()
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c, rotation_seed=seed)
    kx = jvp.lens_jvp(x, xd, a_far, a_near, c, wl.box, 16, geom)
    kom = jvp.lens_om_tangent(x, a_far, a_near, c, wl.box, 16, geom)
    e_x = rel_rms(kgx, kx)
    e_om = rel_rms(kg - kgx, om_dot * kom)
    log(f"lens tangent {dtype}: position part {e_x:.2e}, Omega_m part {e_om:.2e}")
    assert np.abs(kx).max() > 0 and np.abs(kom).max() > 0
    assert e_x < (1e-9 if dtype == torch.float64 else 1e-4)
    # the device differentiates the weights analytically with differenced
    # distance tables, the oracle differences the whole projection
    assert e_om < (1e-6 if dtype == torch.float64 else 1e-4)


def _small():
    return W.Workload("jvpsmall", 16, 32, 48.0, 0.4, 1.0, 3, 16, 3.0, (0.5, 1.0), seed=11)


@pytest.mark.parametrize("direction", ["pixel", "mixed"])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_model_tangent_matches_oracle(dtype, direction):
    """The whole model's tangent (initial conditions, three steps, every
    shell): one perturbed noise pixel (the paper's first derivative check),
    and a random noise direction with Omega_m and sigma_8 tangents."""
    from oracle import jvp, lens
    from paper_2012_07266_amd.autograd import jvp as run_jvp
    wl = _small()
    c = cosmo_of(wl)
    a = wl.a_grid()
    rd = _rd(dtype)
    noise = rd(W.white_noise(wl.np_side, wl.seed))
    if direction == "pixel":
        nd = np.zeros_like(noise)
        nd[3, 5, 2] = 1.0
        om_dot, s8_dot = 0.0, 0.0
    else:
        nd = rd(np.random.default_rng(43).standard_normal(noise.shape))
        om_dot, s8_dot = 0.5, -0.8
    log(f"model tangent {dtype} {direction}")
    with new_sim(wl, dtype, modes=PM_MODE_TANGENT) as sim:
        T = lambda v: torch.tensor(v, dtype=dtype, device="cuda")
        kap, kd = run_jvp(sim, T(noise), a, T(nd), om_dot, s8_dot)
        kg, kdg = to_np(kap), to_np(kd)
        sim.sync()
    log("oracle")
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    ko, kdo = jvp.kappa_jvp(noise, nd, om_dot, s8_dot, c, wl.box, wl.nm_side, a, geom)
    e_k, e_d = rel_rms(kg, ko), rel_rms(kdg, kdo)
    log(f"model tangent {dtype} {direction}: kappa {e_k:.2e}, kappa_dot {e_d:.2e}")
    assert e_k < (1e-10 if dtype == torch.float64 else 1e-4)
    assert e_d < (1e-8 if dtype == torch.float64 else 1e-3)


def test_tangent_transposes_the_reverse_pass_at_the_gradient_workload():
    """128^3 particles, 256^3 mesh, 20 steps, one 1024^2 map (the gradient
    workload), float64: <kbar, J v> from the tangent pass against
    <J^T kbar, v> from the reverse pass, for v = (noise direction, Omega_m,
    sigma_8).  Both are linearisations of the same device computation with
    the same differenced factors, so the identity holds to round-off at any
    size."""
    from paper_2012_07266_amd.autograd import LensingModel
    wl = W.CFG3
    dtype = torch.float64
    log("transpose identity, gradient workload, float64")
    model = LensingModel(wl.np_side, wl.nm_side, wl.box, wl.npix, wl.fov_deg, wl.z_src,
                         wl.a_grid(), dtype=dtype, tangent=True, h=wl.h, n_s=wl.n_s,
                         omega_b=wl.omega_b, t_cmb=wl.t_cmb)
    noise = torch.tensor(W.white_noise(wl.np_side, wl.seed), dtype=dtype, device="cuda")
    rng = np.random.default_rng(44)
    nd = torch.tensor(rng.standard_normal(noise.shape), dtype=dtype, device="cuda")
    kbar = torch.tensor(rng.standard_normal((len(wl.z_src), wl.npix, wl.npix)), dtype=dtype,
                        device="cuda")
    om_dot, s8_dot = 0.3, -0.4
    _, kd = model.jvp(noise, wl.omega_m, wl.sigma8, nd, om_dot, s8_dot)
    lhs = float((kbar * kd).sum())
    log("reverse pass")
    w = noise.clone().requires_grad_(True)
    om = torch.tensor(wl.omega_m, dtype=dtype, device="cuda", requires_grad=True)
    s8 = torch.tensor(wl.sigma8, dtype=dtype, device="cuda", requires_grad=True)
    (model(w, om, s8) * kbar).sum().backward()
    torch.cuda.synchronize()
    parts = [float((w.grad * nd).sum()), float(om.grad) * om_dot, float(s8.grad) * s8_dot]
    model.close()
    rhs = sum(parts)
    log(f"<kbar, J v> = {lhs:.12e}, <J^T kbar, v> = {rhs:.12e} (parts {parts})")
    assert abs(lhs) > 0
    assert abs(lhs - rhs) < 1e-9 * sum(abs(v) for v in parts)


def test_tangent_error_paths():
    from paper_2012_07266_amd import MadlensError
    from paper_2012_07266_amd._lib import PM_EINVAL, PM_ESTATE
    wl = _small()
    noise = torch.tensor(W.white_noise(16, 3), dtype=torch.float32, device="cuda")
    n = 16 ** 3
    z = lambda: torch.zeros((3, n), dtype=torch.float32, device="cuda")

    def code(fn, *args):
        with pytest.raises(MadlensError) as e:
            fn(*args)
        return e.value.code
    with new_sim(wl) as sim:                                  # no tangent buffers
        sim.init_ic(noise, 0.4)
        assert code(sim.init_ic_jvp, noise) == PM_EINVAL
        assert code(sim.set_tangent, z(), z()) == PM_EINVAL
        sim.sync()
    with new_sim(wl, modes=PM_MODE_TANGENT | PM_MODE_PGD) as sim:
        assert code(sim.init_ic_jvp, noise) == PM_ESTATE     # no initial conditions yet
        sim.init_ic(noise, 0.4)
        assert code(sim.step_jvp, 0.4, 0.5) == PM_ESTATE     # no tangent yet
        assert code(sim.init_ic_jvp, noise, float("nan")) == PM_EINVAL
        sim.init_ic_jvp(noise, 0.2, 0.1)
        assert code(sim.step_jvp, 0.5, 0.6) == PM_ESTATE     # state is at 0.4
        with pytest.raises(ValueError):                       # wrong dtype
            sim.set_tangent(z().double(), z())
        sim.step_jvp(0.4, 0.5)
        assert code(sim.init_ic_jvp, noise) == PM_ESTATE     # no longer the initial conditions
        kd = sim.new_maps()
        sim.set_pgd(0.5, 0.5, 0.05, 1.5)
        assert code(sim.lens_jvp, 0.4, 0.5, kd) == PM_EINVAL   # no tangent of the PGD shift
        sim.set_pgd(0.5, 0.5, 0.05, 1.5, on=False)
        sim.lens_jvp(0.4, 0.5, kd)
        xd, pd, fd = sim.get_tangent()
        sim.step(0.5, 0.6)                                     # a plain step drops the tangent
        assert code(sim.step_jvp, 0.6, 0.7) == PM_ESTATE
        assert code(sim.get_tangent) == PM_ESTATE
        sim.set_tangent(z(), z())
        f2 = sim.get_tangent()[2]
        sim.sync()
        assert torch.isfinite(kd).all() and torch.isfinite(xd).all() and torch.isfinite(fd).all()
        assert torch.count_nonzero(f2) == 0                    # zero tangent, zero force tangent


@pytest.mark.parametrize("seed", [None, 0x5EED1234ABCD], ids=["plain", "rotated"])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_lens_tangent_with_subevolution(dtype, seed):
    """A sub-evolved shell's tangent at a state with momenta, along a position
    and momentum tangent and Omega_m: the drift momentum's tangent is
    p_dot - K2 f_dot - Om_dot K2' f, with the force tangent of the state."""
    from oracle import jvp, lens, pm
    wl = W.Workload("lensjvpsub", 16, 32, 64.0, 0.4, 1.0, 3, 24, 4.0, (1.0, 2.0))
    c = cosmo_of(wl)
    x = _off_node_planes(W.clustered_positions(16, 32, wl.box, seed=21), wl.box, 32)
    rng = np.random.default_rng(45)
    p = 10.0 * rng.standard_normal(x.shape)
    xd = rng.standard_normal(x.shape)
    pd = rng.standard_normal(x.shape)
    a_far, a_near = 0.55, 0.7
    ah = 0.5 * (a_far + a_near)
    om_dot = 0.6
    rd = _rd(dtype)
    x, p, xd, pd = rd(x), rd(p), rd(xd), rd(pd)
    log(f"sub-evolved lens tangent {dtype} rotation={seed}")
    with new_sim(wl, dtype, modes=PM_MODE_TANGENT) as sim:
        sim.set_interpolation(True)
        if seed is not None:
            sim.set_replica_rotation(seed)
        T = lambda v: torch.tensor(v, dtype=dtype, device="cuda")
        sim.set_state(T(x), T(p), a_near)
        sim.set_tangent(T(xd), T(pd), om_dot)
        kd = sim.new_maps()
        sim.lens_jvp(a_far, a_near, kd)
        kg = to_np(kd)
        sim.sync()
    log("oracle")
    f = pm.particle_force(x, 16, 32, wl.box)
    fd = jvp.force_jvp(x, xd, 16, 32, wl.box)
    k2 = jvp.step_factors(c, a_far, a_near)[2]
    dk2 = (jvp.step_factors(jvp._with_om(c, 0.3 + 1e-5), a_far, a_near)[2]
           - jvp.step_factors(jvp._with_om(c, 0.3 - 1e-5), a_far, a_near)[2]) / 2e-5
    sub = (p - k2 * f, ah)
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c, rotation_seed=seed)
    ko = jvp.lens_jvp(x, xd, a_far, a_near, c, wl.box, 16, geom, sub=sub,
                      ph_dot=pd - k2 * fd - om_dot * dk2 * f)
    # Omega_m moves the images, so its difference takes a small step (the
    # splat's pixel-edge kinks)
    ko += om_dot * jvp.lens_om_tangent(x, a_far, a_near, c, wl.box, 16, geom, dom=1e-7, sub=sub)
    plain = jvp.lens_jvp(x, xd, a_far, a_near, c, wl.box, 16, geom)
    e = rel_rms(kg, ko)
    log(f"sub-evolved lens tangent {dtype}: {e:.2e} (sub-evolution changes it by "
        f"{rel_rms(plain, ko):.2e})")
    assert rel_rms(plain, ko) > 1e-2
    assert e < (1e-6 if dtype == torch.float64 else 1e-4)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_model_tangent_with_subevolution(dtype):
    from oracle import jvp, lens
    from paper_2012_07266_amd.autograd import jvp as run_jvp
    wl = _small()
    c = cosmo_of(wl)
    a = wl.a_grid()
    rd = _rd(dtype)
    noise = rd(W.white_noise(wl.np_side, wl.seed))
    nd = rd(np.random.default_rng(46).standard_normal(noise.shape))
    om_dot, s8_dot = 0.5, -0.8
    log(f"model tangent with sub-evolution {dtype}")
    with new_sim(wl, dtype, modes=PM_MODE_TANGENT) as sim:
        sim.set_interpolation(True)
        T = lambda v: torch.tensor(v, dtype=dtype, device="cuda")
        kap, kd = run_jvp(sim, T(noise), a, T(nd), om_dot, s8_dot)
        kg, kdg = to_np(kap), to_np(kd)
        sim.sync()
    log("oracle")
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    # a step of 1e-7 in the oracle's Omega_m differences (sub-evolved images
    # move with Omega_m); the library's 1e-5 differences of the scalar
    # factors differ from it at O(1e-10)
    ko, kdo = jvp.kappa_jvp(noise, nd, om_dot, s8_dot, c, wl.box, wl.nm_side, a, geom,
                            dom=1e-7, interpolation=True)
    e_k, e_d = rel_rms(kg, ko), rel_rms(kdg, kdo)
    log(f"model tangent with sub-evolution {dtype}: kappa {e_k:.2e}, kappa_dot {e_d:.2e}")
    assert e_k < (1e-10 if dtype == torch.float64 else 1e-4)
    assert e_d < (1e-8 if dtype == torch.float64 else 1e-3)
