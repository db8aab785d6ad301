"""Device noise, arena reuse and the serving loop, through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import cosmo_of, log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_device_noise_matches_oracle_generator(dtype):
    from oracle import rng
    wl = W.Workload("noise", 48, 96, 100.0, 0.1, 1.0, 2, 16, 2.0, (1.0,))
    seed = 2 ** 40 + 17
    with new_sim(wl, dtype) as sim:
        z = to_np(sim.noise(seed)).ravel()
    ref = rng.white_noise(48, seed).ravel()
    log(f"device noise {dtype}: max |diff| {np.max(np.abs(z - ref)):.3e}")
    if dtype == torch.float64:
        # the same words; transcendental functions may differ in the last bits
        assert np.max(np.abs(z - ref) / np.maximum(1.0, np.abs(ref))) < 1e-13
    else:
        ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(z - ref) <= ulp)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_seeded_initial_conditions_equal_array_initial_conditions(dtype):
    wl = W.Workload("seeded", 32, 64, 64.0, 0.1, 1.0, 2, 16, 2.0, (1.0,))
    with new_sim(wl, dtype) as sim:
        noise = sim.noise(99).clone()
        sim.init_ic_seed(99, 0.1)
        x1, p1 = (t.clone() for t in sim.get_state())
        sim.init_ic(noise, 0.1)
        x2, p2 = sim.get_state()
        assert torch.equal(x1, x2) and torch.equal(p1, p2)


def test_reconfigured_arena_equals_fresh_arena():
    wl = W.Workload("reconf", 32, 64, 64.0, 0.1, 1.0, 4, 64, 2.0, (1.0,))
    a = wl.a_grid()
    other = dict(omega_m=0.27, sigma8=0.85)
    with new_sim(wl, torch.float32) as sim:
        sim.init_ic_seed(5, a[0])
        k0 = sim.new_maps()
        for i in range(len(a) - 1):
            sim.step(a[i], a[i + 1])
            sim.lens(a[i], a[i + 1], k0)
        sim.reconfigure(**other, h=wl.h, n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb)
        sim.init_ic_seed(5, a[0])
        k1 = sim.new_maps()
        for i in range(len(a) - 1):
            sim.step(a[i], a[i + 1])
            sim.lens(a[i], a[i + 1], k1)
        k1 = k1.clone()
    with new_sim(wl.with_(**other), torch.float32) as fresh:
        fresh.init_ic_seed(5, a[0])
        k2 = fresh.new_maps()
        for i in range(len(a) - 1):
            fresh.step(a[i], a[i + 1])
            fresh.lens(a[i], a[i + 1], k2)
    assert not torch.equal(k0, k1)
    assert torch.equal(k1, k2)


def _req(i, np_side, nm, nsteps, om, s8, npix=128):
    return W.Workload(f"r{i}", np_side, nm, float(np_side), 0.1, 1.0, nsteps, npix, 2.0, (1.0,),
                      omega_m=om, sigma8=s8, seed=1000 + i)


def test_served_request_matches_oracle():
    """A float64 request through the server against the oracle fed with the
    oracle's own implementation of the same counter-based noise."""
    from oracle import lens, rng
    from paper_2012_07266_amd.serve import Server
    wl = W.Workload("served", 16, 32, 48.0, 0.3, 1.0, 4, 32, 3.0, (1.0,), omega_m=0.28,
                    sigma8=0.83, seed=4242)
    log("served request vs oracle")
    with Server(4 << 30, 2, np.float64) as srv:
        k, t = srv.result(srv.submit(wl), timeout=120)
    c = cosmo_of(wl)
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    ref, _, _ = lens.run_lensing(rng.white_noise(16, wl.seed), c, wl.box, wl.nm_side,
                                 wl.a_grid(), geom)
    e = rel_rms(k, ref)
    log(f"served vs oracle: kappa rel-rms {e:.2e}, latency {1e3 * (t[2] - t[0]):.1f} ms")
    assert t[0] <= t[1] <= t[2]
    assert e < 1e-10


def test_result_alone_equals_result_in_the_mix():
    """Each request's maps are bitwise the same served alone (plain form) and
    interleaved with requests of other sizes and cosmologies."""
    from paper_2012_07266_amd.serve import Server
    reqs = [_req(0, 64, 128, 10, 0.31, 0.78), _req(1, 128, 256, 6, 0.26, 0.88),
            _req(2, 32, 64, 12, 0.34, 0.72), _req(3, 64, 128, 8, 0.29, 0.81)]
    log("serving: alone vs mix")
    alone = []
    with Server(16 << 30, 1) as srv:
        for r in reqs:
            k, _ = srv.result(srv.submit(r), timeout=120)
            alone.append(k)
    with Server(16 << 30, 4) as srv:
        ids = [srv.submit(r) for r in reqs]
        mix = [srv.result(i, timeout=120)[0] for i in ids]
        st = srv.stats()
    log(f"mix: peak running {st['peak_running']}, peak bytes {st['peak_bytes'] / 1e9:.2f} GB")
    assert st["peak_running"] >= 2
    for a, m in zip(alone, mix):
        assert np.isfinite(a).all() and np.abs(a).max() > 0
        assert np.array_equal(a, m)
    # and the same as the plain per-simulation path with the same seed
    r = reqs[2]
    with new_sim(r, torch.float32) as sim:
        a = r.a_grid()
        sim.init_ic_seed(r.seed, a[0])
        k = sim.new_maps()
        for i in range(len(a) - 1):
            sim.step(a[i], a[i + 1])
            sim.lens(a[i], a[i + 1], k)
        assert np.array_equal(to_np(k).astype(np.float32), alone[2])


def test_admission_by_footprint():
    from paper_2012_07266_amd import _lib
    from paper_2012_07266_amd.serve import Server
    from paper_2012_07266_amd.sim import footprint
    r = _req(10, 64, 128, 3, 0.3, 0.8)
    fp = footprint(64, 128, 64.0, r.npix, r.fov_deg, r.z_src)
    budget = int(1.5 * (fp + 2 ** 20))  # room for one arena (+ maps) at a time
    with Server(budget, 8) as srv:
        ids = [srv.submit(_req(10 + i, 64, 128, 3, 0.3, 0.8)) for i in range(4)]
        for i in ids:
            srv.result(i, timeout=120)
        st = srv.stats()
        with pytest.raises(_lib.MadlensError):
            srv.submit(_req(20, 128, 256, 3, 0.3, 0.8))  # above the budget
    log(f"admission: peak running {st['peak_running']}, peak {st['peak_bytes']} of {budget}")
    assert st["peak_running"] == 1 and st["peak_bytes"] <= budget
    assert st["completed"] == 4


def test_result_alone_equals_result_in_the_batched_mix():
    """The batched server (same-shape requests stepped together, replayed
    from a HIP graph): every request's maps are bitwise those of the plain
    form, for a mix of three shapes arriving together."""
    from paper_2012_07266_amd.serve import Server
    reqs = [_req(0, 64, 128, 10, 0.31, 0.78), _req(1, 128, 256, 6, 0.26, 0.88),
            _req(2, 32, 64, 12, 0.34, 0.72), _req(3, 64, 128, 8, 0.29, 0.81),
            _req(4, 64, 128, 5, 0.33, 0.75), _req(5, 32, 64, 7, 0.27, 0.86)]
    log("serving: alone vs batched mix")
    with Server(16 << 30, 1) as srv:
        alone = [srv.result(srv.submit(r), timeout=120)[0] for r in reqs]
    with Server(16 << 30, 6, batched=True) as srv:
        ids = [srv.submit(r) for r in reqs]
        mix = [srv.result(i, timeout=120)[0] for i in ids]
        st = srv.stats()
    log(f"batched mix: peak running {st['peak_running']}")
    assert st["peak_running"] >= 2
    for a, m in zip(alone, mix):
        assert np.isfinite(a).all() and np.abs(a).max() > 0
        assert np.array_equal(a, m)


def test_batched_served_request_matches_oracle():
    from oracle import lens, rng
    from paper_2012_07266_amd.serve import Server
    wl = W.Workload("served_b", 16, 32, 48.0, 0.3, 1.0, 4, 32, 3.0, (1.0,), omega_m=0.28,
                    sigma8=0.83, seed=4242)
    other = wl.with_(name="served_b2", box=40.0, nsteps=6, seed=4243)
    log("batched served request vs oracle")
    with Server(4 << 30, 2, np.float64, batched=True) as srv:
        i0, i1 = srv.submit(wl), srv.submit(other)
        k, t = srv.result(i0, timeout=120)
        srv.result(i1, timeout=120)
    c = cosmo_of(wl)
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    ref, _, _ = lens.run_lensing(rng.white_noise(16, wl.seed), c, wl.box, wl.nm_side,
                                 wl.a_grid(), geom)
    e = rel_rms(k, ref)
    log(f"batched served vs oracle: kappa rel-rms {e:.2e}")
    assert e < 1e-10
