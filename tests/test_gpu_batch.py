"""Batched stepping (pm_batch_*) through the C ABI: every slot's maps and
state are those of pm_run on its handle alone (bit for bit in float32),
whether the passes are replayed from the captured HIP graph or launched
directly, with slots joining and leaving between steps and eager work of
the program's own between replays; one batched simulation against the
float64 oracle; and the error paths."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import cosmo_of, log, new_sim, rel_rms, to_np

pytestmark = pytest.mark.gpu


def _requests(np_side, nm, box, n):
    """n requests of one shape with their own cosmology, seed, time grid and
    map geometry (as a serving stream draws them)."""
    gen = np.random.Generator(np.random.Philox(key=31))
    out = []
    for i in range(n):
        nsteps = int(gen.integers(4, 9))
        a0 = float(gen.uniform(0.1, 0.2))
        out.append(W.Workload(f"b{i}", np_side, nm, box * float(gen.uniform(0.8, 1.2)), a0, 1.0,
                              nsteps, 128, float(gen.uniform(1.5, 3.0)), (1.0, 1.5),
                              omega_m=float(gen.uniform(0.25, 0.35)),
                              sigma8=float(gen.uniform(0.7, 0.9)), seed=500 + i))
    return out


def _alone(wl, dtype):
    with new_sim(wl, dtype) as sim:
        a = wl.a_grid()
        sim.init_ic_seed(wl.seed, a[0])
        k = sim.new_maps()
        sim.steps(a, k)
        x, p = sim.get_state()
        sim.sync()
        return k.clone(), x.clone(), p.clone()


def _batched(reqs, dtype, use_graph, capacity, join_late=()):
    """Requests join as slots free up (those in join_late only from the third
    step on); step until every one has finished, detaching finished ones and
    doing eager work between the replays."""
    from paper_2012_07266_amd.sim import Batch
    sims = [new_sim(r, dtype) for r in reqs]
    maps = [s.new_maps() for s in sims]
    res = [None] * len(reqs)
    with Batch(sims[0], capacity, use_graph=use_graph) as b:
        waiting = [i for i in range(len(reqs)) if i not in join_late]
        late = list(join_late)
        running = {}
        steps = 0
        while waiting or late or running:
            if steps == 2:
                waiting += late
                late = []
            while waiting and len(running) < capacity:
                i = waiting.pop(0)
                a = reqs[i].a_grid()
                sims[i].init_ic_seed(reqs[i].seed, a[0])
                b.attach(sims[i], a, maps[i])
                running[i] = 0
            b.step()
            steps += 1
            for i in list(running):
                running[i] += 1
                if running[i] == reqs[i].nsteps:
                    b.detach(sims[i])
                    x, p = sims[i].get_state()
                    res[i] = (maps[i].clone(), x.clone(), p.clone())
                    del running[i]
            # the program's own eager work between replays
            junk = torch.randn(1 << 16, device="cuda").cumsum(0)
            torch.cuda.synchronize()
            assert torch.isfinite(junk).all()
    for s in sims:
        s.sync()
        s.close()
    return res, steps


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "direct"])
def test_batched_slots_equal_each_run_alone(use_graph):
    reqs = _requests(64, 128, 64.0, 5)
    log(f"batch 5 x 64^3/128^3 float32, graph={use_graph}")
    alone = [_alone(r, torch.float32) for r in reqs]
    res, steps = _batched(reqs, torch.float32, use_graph, capacity=4, join_late=(3,))
    log(f"batch: {steps} batched steps for {sum(r.nsteps for r in reqs)} request steps")
    for i, (a, r) in enumerate(zip(alone, res)):
        assert torch.abs(a[0]).max() > 0
        assert torch.equal(a[0], r[0]), i
        assert torch.equal(a[1], r[1]) and torch.equal(a[2], r[2]), i


def test_batched_float64_slot_matches_oracle():
    """A float64 batch of two requests; the first against the oracle fed with
    the oracle's own implementation of the device noise generator."""
    from oracle import lens, rng
    reqs = [W.Workload("bo0", 16, 32, 48.0, 0.3, 1.0, 4, 32, 3.0, (1.0,), omega_m=0.28,
                       sigma8=0.83, seed=4242),
            W.Workload("bo1", 16, 32, 40.0, 0.25, 1.0, 6, 32, 2.0, (1.0,), omega_m=0.33,
                       sigma8=0.74, seed=4243)]
    log("batch float64 vs oracle")
    res, _ = _batched(reqs, torch.float64, True, capacity=2)
    for wl, r in zip(reqs, res):
        c = cosmo_of(wl)
        geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
        ref, _, _ = lens.run_lensing(rng.white_noise(16, wl.seed), c, wl.box, wl.nm_side,
                                     wl.a_grid(), geom)
        e = rel_rms(to_np(r[0]), ref)
        log(f"batch float64 {wl.name}: kappa rel-rms {e:.2e}")
        assert np.abs(ref).max() > 0 and e < 1e-10


def test_batch_error_paths():
    from paper_2012_07266_amd import MadlensError
    from paper_2012_07266_amd._lib import PM_EFULL, PM_EINVAL, PM_ESTATE
    from paper_2012_07266_amd.sim import Batch
    wl = W.Workload("be", 16, 32, 40.0, 0.2, 1.0, 3, 32, 3.0, (1.0,), seed=7)
    other = wl.with_(np_side=32, nm_side=64)
    a = wl.a_grid()

    def code(fn, *args):
        with pytest.raises(MadlensError) as e:
            fn(*args)
        return e.value.code
    with new_sim(wl) as s1, new_sim(wl) as s2, new_sim(other) as s3, Batch(s1, 1) as b:
        assert code(b.attach, s1, a) == PM_ESTATE            # no initial conditions
        s1.init_ic_seed(1, a[0])
        assert code(b.attach, s1, a[1:]) == PM_ESTATE        # state not at the grid's start
        s3.init_ic_seed(1, a[0])
        assert code(b.attach, s3, a) == PM_EINVAL            # another shape
        b.attach(s1, a)
        assert code(b.attach, s1, a) == PM_EINVAL            # attached already
        s2.init_ic_seed(2, a[0])
        assert code(b.attach, s2, a) == PM_EFULL
        assert code(b.lens, s2, None) == PM_EINVAL           # not attached
        b.step()
        b.detach(s1)                                          # mid-run: between two steps
        assert code(s1.step, a[1], a[2]) == PM_ESTATE
        assert code(b.detach, s1) == PM_EINVAL
        s1.init_ic_seed(1, a[0])                              # new initial conditions continue it
        s1.step(a[0], a[1])
        s1.sync()
