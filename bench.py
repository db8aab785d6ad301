"""Benchmark: particle-steps/s of the PM step + Born lens projection on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--repeats R] [--workload cfg2]

Workload (default): 256^3 particles on a 512^3 force mesh in a 205 Mpc/h
box, 40 PM steps linear in a from 0.01 to 1.0, four 2048^2 convergence maps
over 5 deg x 5 deg at z_s = 0.5, 1, 1.5, 2 (float32), seeded Gaussian white
noise initial conditions.  A "step" is one step of pm_run: a KDK step and
the Born projection of its shell (bit for bit pm_step + lens_project).

Timing: W untimed warm-up steps; then R repeats, each from fresh initial
conditions, of the schedule with its LAST K steps timed (the first N - K
steps run untimed before the timer starts; with K > N the schedule restarts
from fresh initial conditions inside the timed region).  The reported step
time is the median of the R repeats.  With the default K = 40 the whole
schedule is timed; K = 20 times the late, clustered half (a = 0.505 -> 1)
with 20 of its 27 lens shells.  Per-kernel durations come from HIP events
the library records on its own stream: for every kernel over one more,
untimed, pass of the same window; for the roofline's kernel alone inside the
timed repeats (events between kernels cost time of their own).

The line also carries the same run with sub-evolution projection, with the
PGD correction and with replica rotation (mode_bench), the forward + reverse
timing of the gradient workload (gradient_bench), the serving figures named
by the metric: p50/p99 latency (arrival to maps on the host) and throughput
of Poisson streams of mixed-size requests, served (continuous batching) and
plain (one simulation at a time), see serving_bench; and the float64 oracle
on the host (cpu_baseline): timed in full on the 32^3 workload and on a
bounded sample of one step of the benchmark's workload.

Counter-measured HBM traffic (profiles/traffic.json) is taken over one
steady-state step late in the schedule: run `bench.py --traffic-step S`
under rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, and convert with
`bench.py --traffic-from FETCH_CSV WRITE_CSV` (see traffic_from_pmc).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
STEP_GATE = 0.60       # fraction of the HBM peak the PM step is to sustain


def algorithmic_bytes(wl, esize=4):
    """Algorithmic HBM bytes of one launch of every timed kernel class.

    P = particles, M = one real mesh, S = one half spectrum (main + Nyquist
    plane).  Counts each input read once and each output written once, for
    the arrays each kernel of this library actually reads and writes.
    """
    P = wl.np_side ** 3
    nm = wl.nm_side
    M = nm ** 3 * esize
    S = M + nm * nm * 2 * esize
    maps = len(wl.z_src) * wl.npix ** 2 * esize
    return {
        "kick_drift_key": 68 * P,          # R disp,mom,acc,id  W disp,mom,key
        "scatter": 60 * P,                 # R key,disp,mom,id  W disp,mom,id
        "paint": 16 * P + M,               # R disp,id  W rho
        "fft_r2c_axis2": M + S,
        "fft_c2c_axis1_fwd": 2 * S,
        "fft_grad_axis0": 3 * S,           # R 1 spectrum, W 2
        "fft_c2c_axis1_inv": 2 * S,
        "fft_c2c_axis1_dual": 3 * S,       # R 1 spectrum, W 2
        "fft_c2r_axis2": S + M,
        "readout_kick": 3 * M + 52 * P,    # R 3 meshes, disp,id,mom  W mom,acc
        # fused with the next step's kick, drift and keys:
        "readout_kick_drift_key": 3 * M + 56 * P,  # R 3 meshes, disp,id,mom  W disp,mom,key
        "lens_gather": 16 * P + 2 * maps,  # R disp,id  RW maps (incl. mean term)
        "scan": 0,
    }


def model_bytes(wl, esize=4):
    """The byte model of the method's hot path per particle-step unit (one
    step's particles and meshes), for the kernels it names: readout + kick +
    drift reads three force meshes and reads and writes position and
    momentum, 3 M + 48 P (no particle id, no sort key)."""
    P = wl.np_side ** 3
    M = wl.nm_side ** 3 * esize
    return {"readout_kick_drift_key": 3 * M + 48 * P, "readout_kick": 3 * M + 48 * P}


# kernel classes launched on the second stream (beside the force transform)
SIDE_STREAM = {"lens_gather"}
# (method's bytes, kernel's own bytes) of the kernels model_bytes names
BYTES_WHAT = {
    "readout_kick_drift_key": (
        "3 M + 48 P: three force meshes, position and momentum read and written",
        "3 M + 56 P: the kernel's own arrays, with the particle id read and the next step's "
        "sort key written"),
    "readout_kick": (
        "3 M + 48 P: three force meshes, position and momentum read, momentum and force "
        "written",
        "3 M + 52 P: the kernel's own arrays, with the particle id read and the force written"),
}

TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
# kernel class -> (substring of the HIP kernel name in rocprofv3 output, source)
KERNEL_SYMBOL = {
    "kick_drift_key": ("k_kick_drift_key<float", "paper_2012_07266_amd/csrc/particles.hip"),
    "scan": ("k_scan_", "paper_2012_07266_amd/csrc/particles.hip"),
    "scatter": ("k_scatter<float", "paper_2012_07266_amd/csrc/particles.hip"),
    "paint": ("k_paint_group<float", "paper_2012_07266_amd/csrc/particles.hip"),
    "lens_gather": ("k_lens_gather<float", "paper_2012_07266_amd/csrc/lens.hip"),
    "fft_r2c_axis2": ("k_r2c_rows<float", "paper_2012_07266_amd/csrc/fft.hip"),
    "fft_c2c_axis1_fwd": ("k_c2c_view<float, 512, 16, 1>", "paper_2012_07266_amd/csrc/fft.hip"),
    "fft_grad_axis0": ("k_grad_x0<float", "paper_2012_07266_amd/csrc/fft.hip"),
    "fft_c2c_axis1_inv": ("k_c2c_view<float, 512, 16, -1>", "paper_2012_07266_amd/csrc/fft.hip"),
    "fft_c2c_axis1_dual": ("k_c2c_view_dual<float", "paper_2012_07266_amd/csrc/fft.hip"),
    "fft_c2r_axis2": ("k_c2r_rows<float", "paper_2012_07266_amd/csrc/fft.hip"),
    "readout_kick_drift_key": ("k_readout<float>", "paper_2012_07266_amd/csrc/particles.hip"),
    "fill": ("k_fill", "paper_2012_07266_amd/csrc/particles.hip"),
}
COPY_BYTES = 1 << 30  # the calibration copy moves 1 GiB in and 1 GiB out


def _pmc_rows(path, counter):
    """(dispatch order, kernel name, bytes) of every dispatch of one counter."""
    import csv
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = int(r.get("Dispatch_Id") or r.get("Correlation_Id") or len(rows))
        rows.append((key, r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
    rows.sort()
    return rows


def _late_step(rows):
    """The dispatches of the steady-state step that `--traffic-step` runs:
    after the calibration copy (the marker), pm_run steps S and S + 1; step
    S + 1 is every dispatch after the first readout up to and including the
    second.  Returns (calibration bytes, [(name, bytes)])."""
    i_copy = max(range(len(rows)), key=lambda i: rows[i][2] if "copy" in rows[i][1].lower() else -1)
    calib = rows[i_copy][2]
    reads = [i for i in range(i_copy + 1, len(rows)) if "k_readout" in rows[i][1]]
    if len(reads) < 2:
        raise RuntimeError("the counted run holds fewer than two readouts after the marker")
    return calib, [(n, b) for _, n, b in rows[reads[0] + 1:reads[1] + 1]]


def traffic_from_pmc(fetch_csv, write_csv, workload, step):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs of
    `bench.py --traffic-step S` (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch): the HBM bytes of every dispatch of step S + 1 of the
    schedule, a steady-state step of pm_run late in the run.  Each counter
    is scaled by what it reads for the 1 GiB calibration copy that precedes
    the counted steps, whose true traffic is known."""
    import hashlib
    cf, fetch = _late_step(_pmc_rows(fetch_csv, "FETCH_SIZE"))
    cw, write = _late_step(_pmc_rows(write_csv, "WRITE_SIZE"))
    if [n for n, _ in fetch] != [n for n, _ in write]:
        raise RuntimeError("the two counted runs dispatched different kernels")
    sf, sw = COPY_BYTES / cf, COPY_BYTES / cw
    per = {}
    for (name, f), (_, w) in zip(fetch, write):
        cls = next((c for c, (sub, _) in KERNEL_SYMBOL.items() if sub in name), name[:48])
        e = per.setdefault(cls, {"launches": 0, "fetch_bytes": 0.0, "write_bytes": 0.0})
        e["launches"] += 1
        e["fetch_bytes"] += f * sf
        e["write_bytes"] += w * sw
    out = {"_about": ("HBM bytes of one steady-state pm_run step late in the schedule, from "
                      "rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by the counters of a 1 GiB "
                      "device copy; per kernel class: bytes per launch"),
           "_scale": {"fetch": sf, "write": sw}, "_workload": workload, "_step": step + 1,
           "_step_bytes": sum(f * sf + w * sw for (_, f), (_, w) in zip(fetch, write))}
    for cls, e in per.items():
        src = KERNEL_SYMBOL.get(cls, (None, None))[1]
        h = (hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
             if src else None)
        n = e["launches"]
        out[cls] = {"symbol": KERNEL_SYMBOL.get(cls, (cls, None))[0], "source": src,
                    "sha256": h, "launches": n, "fetch_bytes": e["fetch_bytes"] / n,
                    "write_bytes": e["write_bytes"] / n,
                    "bytes_per_launch": (e["fetch_bytes"] + e["write_bytes"]) / n}
    json.dump(out, open(TRAFFIC_JSON, "w"), indent=1)
    print(json.dumps(out))


def _source_current(ent):
    import hashlib
    if not ent.get("source"):
        return True
    h = hashlib.sha256(open(os.path.join(ROOT, ent["source"]), "rb").read()).hexdigest()
    return h == ent["sha256"]


def load_traffic(workload):
    """The counter record of profiles/traffic.json if it was taken on this
    workload, else None; entries whose kernel source has changed since (hash
    recorded with the counters) are marked stale."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    try:
        rec = json.load(open(TRAFFIC_JSON))
    except ValueError:
        return None
    if rec.get("_workload") != workload:
        return None
    for k, v in rec.items():
        if not k.startswith("_"):
            v["current"] = _source_current(v)
    return rec


def cpu_baseline(wl, frac=8):
    """The float64 oracle on the host, as it stands.

    In full: the 32^3 particle / 32^3 mesh workload (5 steps from a = 0.1,
    one 64^2 map), initial conditions excluded, particle-steps/s.
    Sample of the benchmark's workload: the oracle's own Zel'dovich state at
    a = 0.5; CIC paint and CIC readout of 1/frac of the particles and the
    lens projection of the same subsample for one late shell, each scaled by
    frac; the three full-size Fourier force transforms.  Reported as
    particle-steps/s of one step (an estimate from the sample).
    """
    from oracle import lens, pm
    from oracle.cosmology import Cosmology
    import workloads as W
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    def cosmo(w):
        return Cosmology(w.omega_m, w.h, w.n_s, w.sigma8, w.omega_b, w.t_cmb)
    # the 32^3 workload in full
    w1 = W.CFG1
    c1 = cosmo(w1)
    g1 = lens.MapGeometry(w1.npix, w1.fov_deg, w1.z_src, c1)
    a1 = w1.a_grid()
    n1 = W.white_noise(w1.np_side, w1.seed)
    x, p = pm.zeldovich_ic(n1, c1, w1.box, w1.nm_side, a1[0])
    f = pm.particle_force(x, w1.np_side, w1.nm_side, w1.box)
    kap = np.zeros((1, w1.npix, w1.npix))
    t0 = time.perf_counter()
    for i in range(w1.nsteps):
        x, p, f = pm.kdk_step(x, p, f, a1[i], a1[i + 1], c1, w1.np_side, w1.nm_side, w1.box)
        kap += lens.project_shell(x, a1[i], a1[i + 1], c1, w1.box, w1.np_side, g1)
    t_full = time.perf_counter() - t0
    full = {"workload": w1.name, "value": w1.np_side ** 3 * w1.nsteps / t_full,
            "unit": "particle-steps/s", "seconds": t_full, "s_per_step": t_full / w1.nsteps}
    # a bounded sample of one step of the benchmark's workload
    c = cosmo(wl)
    noise = W.white_noise(wl.np_side, wl.seed)
    x, _ = pm.zeldovich_ic(noise, c, wl.box, wl.nm_side, 0.5)
    sub = x[:, ::frac]
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    a = wl.a_grid()
    i = int(0.85 * wl.nsteps)
    t0 = time.perf_counter()
    rho = pm.cic_paint(sub, wl.nm_side, wl.box, mass=(wl.nm_side / wl.np_side) ** 3)
    t1 = time.perf_counter()
    f = pm.force_mesh(rho * frac, wl.box)
    t2 = time.perf_counter()
    for j in range(3):
        pm.cic_readout(sub, f[j], wl.box)
    t3 = time.perf_counter()
    lens.project_shell(sub, a[i], a[i + 1], c, wl.box, wl.np_side, geom)
    t4 = time.perf_counter()
    per_step = (t1 - t0) * frac + (t2 - t1) + (t3 - t2) * frac + (t4 - t3) * frac
    return {"value": wl.np_side ** 3 / per_step, "unit": "particle-steps/s",
            "cores": cores, "kind": "oracle",
            "sample": (f"SAMPLE, an estimate: one PM step + lens shell {i} of {wl.name}: paint, "
                       f"readout and lens of 1/{frac} of the particles (scaled x{frac}) + full "
                       f"{wl.nm_side}^3 float64 FFT force; {t4 - t0:.1f} s of CPU work, est. "
                       f"{per_step:.1f} s/step"),
            "full_run": full}


def gradient_bench(reps=3):
    """Forward + hand-written reverse pass of the gradient workload: 128^3
    particles on a 256^3 mesh, 128 Mpc/h, 20 steps from a = 0.01, one
    1024^2 map over 2 deg at z_s = 1, float32; loss chi^2 = sum (kappa -
    kappa_t)^2 / sigma^2 against a target map from another seed with
    Gaussian pixel noise sigma = 0.01; gradients with respect to the 128^3
    noise values, Omega_m and sigma_8, with per-step checkpoints that carry
    the force at their state (restored by copy; 0.23 GB each at this size).
    The same with state-only checkpoints (whose restores recompute the
    force) is timed beside it."""
    import torch
    import workloads as W
    from paper_2012_07266_amd import Simulation
    from paper_2012_07266_amd.autograd import forward_with_checkpoints, jvp, reverse_pass
    wl = W.CFG3
    a = wl.a_grid()
    dev = torch.device("cuda", 0)
    sim = Simulation(wl.np_side, wl.nm_side, wl.box, wl.npix, wl.fov_deg, wl.z_src,
                     dtype=torch.float32, tangent=True, ckpt_force=True, omega_m=wl.omega_m,
                     sigma8=wl.sigma8, h=wl.h, n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb)
    sigma = 0.01
    target, _ = forward_with_checkpoints(
        sim, torch.from_numpy(W.white_noise(wl.np_side, 4)).to(dev, torch.float32), a)
    gen = np.random.Generator(np.random.Philox(key=5))
    target = target + torch.from_numpy(
        gen.normal(0.0, sigma, size=tuple(target.shape))).to(dev, torch.float32)
    noise = torch.from_numpy(W.white_noise(wl.np_side, wl.seed)).to(dev, torch.float32)
    # a tangent direction: noise, Omega_m and sigma_8 together
    n_dot = torch.from_numpy(W.white_noise(wl.np_side, 6)).to(dev, torch.float32)
    t_f, t_b, t_p, t_j = [], [], [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kappa, states = forward_with_checkpoints(sim, noise, a)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kbar = 2.0 * (kappa - target) / sigma ** 2
        sim.init_ic(noise, a[0])  # the reverse of the IC reads this noise
        nb, g_om, g_s8 = reverse_pass(sim, a, states, kbar)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del states
        # plain forward (no checkpoints), then forward + tangent in one pass
        sim.run_stepwise(noise, a)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        _, kd = jvp(sim, noise, a, n_dot, 0.3, 0.2)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        if r > 0:  # the first pass is a warm-up
            t_f.append(t1 - t0)
            t_b.append(t2 - t1)
            t_p.append(t3 - t2)
            t_j.append(t4 - t3)
    sim.profile(True)
    jvp(sim, noise, a, n_dot, 0.3, 0.2)
    jk = sim.profile_read()
    sim.profile(False)
    jvp_finite = bool(torch.isfinite(kd).all().item())
    sim.close()
    # state-only checkpoints
    sim0 = Simulation(wl.np_side, wl.nm_side, wl.box, wl.npix, wl.fov_deg, wl.z_src,
                      dtype=torch.float32, omega_m=wl.omega_m, sigma8=wl.sigma8, h=wl.h,
                      n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb)
    t_f0, t_b0 = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kappa0, states0 = forward_with_checkpoints(sim0, noise, a)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kbar0 = 2.0 * (kappa0 - target) / sigma ** 2
        sim0.init_ic(noise, a[0])
        reverse_pass(sim0, a, states0, kbar0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del states0
        if r > 0:
            t_f0.append(t1 - t0)
            t_b0.append(t2 - t1)
    sim0.close()
    f0, b0 = float(np.median(t_f0)), float(np.median(t_b0))
    f, b = float(np.median(t_f)), float(np.median(t_b))
    pf, jf = float(np.median(t_p)), float(np.median(t_j))
    ps = wl.np_side ** 3 * wl.nsteps
    return {"workload": (f"{wl.name}: 128^3 particles, 256^3 mesh, 20 steps, 1 x 1024^2 map, "
                         "float32, chi^2 loss, gradients w.r.t. noise, Omega_m, sigma_8"),
            "checkpoints": "state and force (PM_MODE_CKPT_FORCE)",
            "forward_ms": 1e3 * f, "reverse_ms": 1e3 * b, "reverse_over_forward": b / f,
            "gradient_over_plain_forward": (f + b) / pf,
            "state_only_checkpoints": {"forward_ms": 1e3 * f0, "reverse_ms": 1e3 * b0,
                                       "reverse_over_forward": b0 / f0,
                                       "gradient_over_plain_forward": (f0 + b0) / pf},
            "forward_particle_steps_per_s": ps / f,
            "forward_plus_reverse_particle_steps_per_s": ps / (f + b),
            "grad_finite": bool(torch.isfinite(nb).all().item() and np.isfinite(g_om)
                                and np.isfinite(g_s8)),
            "plain_forward_ms": 1e3 * pf,
            "jvp_ms": 1e3 * jf,
            "jvp_over_forward": jf / pf,
            "jvp_what": ("forward pass carrying the tangent along (noise, Omega_m, sigma_8); "
                         "ratio to the plain stepwise forward without checkpoints"),
            "jvp_kernels_ms": {k: round(v[0], 3) for k, v in jk.items()
                               if k.startswith(("jvp", "lens_jvp"))},
            "jvp_finite": jvp_finite}


SERVING_FORMS = (("batched", 8, True), ("streams", 8, False), ("plain", 1, False))


def serving_bench(n_requests, rates=(20.0, 100.0, 200.0)):
    """Poisson streams of serving requests: sizes 64^3/128^3, 128^3/256^3,
    192^3/384^3 (box = Np Mpc/h), 10-30 steps from a = 0.1, Om ~ U[0.25, 0.35],
    s8 ~ U[0.7, 0.9], one 512^2 map over 2 deg at z_s = 1, in three forms:
    batched (up to 8 running, same-shape requests stepped together by
    batched launches replayed from a HIP graph), streams (up to 8 running,
    each on a stream of its own) and plain (one at a time, FIFO); at 20
    requests/s and at the saturating 100 and 200 requests/s."""
    import workloads as W
    from paper_2012_07266_amd.serve import poisson_arrivals, run_stream
    gen = np.random.Generator(np.random.Philox(key=6))
    reqs = [W.serve_request(i, gen) for i in range(n_requests)]
    budget = 64 << 30
    res = {"workload": (f"{n_requests} requests, sizes uniform over 64^3/128^3, 128^3/256^3, "
                        "192^3/384^3, 10-30 steps, 1 x 512^2 map; Poisson arrivals"),
           "hbm_budget_gb": budget / 2 ** 30, "served_max_active": 8}
    for rate in rates:
        arr = poisson_arrivals(n_requests, rate, seed=int(rate))
        row = {}
        for form, act, batched in SERVING_FORMS:
            r, _ = run_stream(reqs, arr, budget, act, batched=batched)
            row[form] = {"p50_ms": r.latency_p50_ms, "p99_ms": r.latency_p99_ms,
                         "mean_ms": r.latency_mean_ms, "particle_steps_per_s": r.throughput,
                         "makespan_s": r.makespan_s, "peak_running": r.peak_running}
        res[f"rate_{int(rate)}_per_s"] = row
    return res


def large_mix_bench(n_background=40, rate=20.0):
    """The 512^3/1024^3 run (10 x 4096^2 maps, 40 steps) submitted at t = 0,
    with a Poisson stream of small requests behind it at `rate` per second:
    64^3 particles, 128^3 mesh, box 64 Mpc/h, 10-30 steps from a = 0.1,
    Om ~ U[0.25, 0.35], s8 ~ U[0.7, 0.9], one 512^2 map over 2 deg at z_s = 1.
    In the three forms of serving_bench."""
    import workloads as W
    from paper_2012_07266_amd.serve import poisson_arrivals, run_stream
    gen = np.random.Generator(np.random.Philox(key=8))
    small = []
    for i in range(n_background):
        nsteps = int(gen.integers(10, 31))
        om, s8 = float(gen.uniform(0.25, 0.35)), float(gen.uniform(0.7, 0.9))
        small.append(W.Workload(f"bg{i}", 64, 128, 64.0, 0.1, 1.0, nsteps, 512, 2.0, (1.0,),
                                omega_m=om, sigma8=s8, seed=2000 + i))
    reqs = [W.CFG5] + small
    arr = np.concatenate([[0.0], poisson_arrivals(n_background, rate, seed=8)])
    budget = 64 << 30
    res = {"workload": (f"{W.CFG5.name} (512^3 particles, 1024^3 mesh, 40 steps, 10 x 4096^2 "
                        f"maps) at t = 0, then {n_background} requests of 64^3/128^3, 10-30 "
                        f"steps, 1 x 512^2 map, Poisson at {rate:g}/s"),
           "hbm_budget_gb": budget / 2 ** 30, "served_max_active": 8}
    for form, act, batched in SERVING_FORMS:
        r, _ = run_stream(reqs, arr, budget, act, batched=batched)
        lat = np.array(r.latencies_ms)
        res[form] = {"large_latency_ms": float(lat[0]),
                     "background_p50_ms": float(np.percentile(lat[1:], 50)),
                     "background_p99_ms": float(np.percentile(lat[1:], 99)),
                     "particle_steps_per_s": r.throughput, "makespan_s": r.makespan_s,
                     "peak_running": r.peak_running}
    return res


# alpha0, mu, k_l, k_s [h/Mpc] for timing only: a correction of about 1% of
# the (filtered) force, shifts of order a cell at the 512^3 mesh.  The cost
# of the lens grows with the largest shift, which widens its frustum margin.
PGD_TIMING = (0.005, 0.5, 0.5, 5.0)
ROTATION_SEED = 12345


def mode_bench(sim, timed_window, wl, steps, mode):
    """The benchmark's timed window with sub-evolution projection (every
    image moved along its step's drift to the scale factor of its own
    distance), with the PGD correction of the projected positions, or with
    rotated replicas."""
    if mode == "interpolation":
        sim.set_interpolation(True)
    elif mode == "rotation":
        sim.set_replica_rotation(ROTATION_SEED)
    else:
        sim.set_pgd(*PGD_TIMING)
    times = [timed_window() for _ in range(3)]
    # kernel averages from another, untimed pass with events around every launch
    prof = timed_window(profile=True)
    sim.set_interpolation(False)
    sim.set_pgd(*PGD_TIMING, on=False)
    sim.set_replica_rotation(None)

    def avg(name):
        ms, cnt = prof.get(name, (0.0, 0))
        return ms / max(cnt, 1)

    t = float(np.median(times))
    out = {"ms_per_step": 1e3 * t / steps,
           "particle_steps_per_s": wl.np_side ** 3 * steps / t,
           "lens_gather_avg_ms": avg("lens_gather")}
    if mode == "interpolation":
        out["what"] = "the same run with sub-evolution projection"
        out["drift_momentum_max_avg_ms"] = avg("drift_momentum_max")
    elif mode == "rotation":
        out["what"] = "the same run with every box replica rotated by a cube symmetry"
    else:
        out["what"] = ("the same run projecting PGD-corrected positions, (alpha0, mu, k_l, k_s) = "
                       + str(PGD_TIMING))
        out["pgd_readout_avg_ms"] = avg("pgd_readout")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats of the window; the median is reported")
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="no per-kernel events in the timed region (roofline omitted)")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the forward + reverse timing of the gradient workload")
    ap.add_argument("--no-interpolation", action="store_true",
                    help="skip the runs with sub-evolution, PGD and replica rotation")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving streams (p50/p99 latency, served vs plain)")
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--no-large-mix", action="store_true",
                    help="skip serving the 512^3/1024^3 run with a stream of small requests")
    ap.add_argument("--traffic-step", type=int, default=None, metavar="S",
                    help="counter run: S untimed steps, a 1 GiB calibration copy, then steps "
                         "S and S + 1 (run under rocprofv3 --pmc), and exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc CSVs of "
                         "--traffic-step runs and exit")
    args = ap.parse_args()
    import workloads as W
    wl = {"cfg1": W.CFG1.with_(name="plain_fp32_32p_32m"), "cfg2": W.CFG2,
          "cfg3": W.CFG3, "cfg5": W.CFG5}[args.workload]
    late = int(0.75 * wl.nsteps)  # step 30 of 40: strong clustering
    if args.traffic_from:
        traffic_from_pmc(*args.traffic_from, wl.name, late if args.traffic_step is None
                         else args.traffic_step)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2012_07266_amd import Simulation
    from paper_2012_07266_amd._lib import PM_MODE_PGD

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    noise = torch.from_numpy(W.white_noise(wl.np_side, wl.seed)).to(dev, torch.float32)
    a = wl.a_grid()
    sim = Simulation(wl.np_side, wl.nm_side, wl.box, wl.npix, wl.fov_deg, wl.z_src,
                     dtype=torch.float32, modes=0 if args.no_interpolation else PM_MODE_PGD,
                     omega_m=wl.omega_m, sigma8=wl.sigma8, h=wl.h,
                     n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb)
    kappa = sim.new_maps()

    def run_steps(k, i0):
        """k steps of the schedule from step i0 (pm_run over each contiguous
        stretch; a new run restarts from fresh initial conditions)."""
        i = i0
        while k > 0:
            if i == wl.nsteps:
                sim.init_ic(noise, a[0])
                kappa.zero_()
                i = 0
            m = min(k, wl.nsteps - i)
            sim.steps(a[i:i + m + 1], kappa)
            i += m
            k -= m
        return i

    if args.traffic_step is not None:
        s0 = args.traffic_step
        sim.init_ic(noise, a[0])
        kappa.zero_()
        run_steps(s0, 0)
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)  # the calibration copy, and the marker before the counted steps
        run_steps(2, s0)
        torch.cuda.synchronize()
        sim.close()
        print(json.dumps({"traffic_step": s0, "workload": wl.name}))
        return

    # the timed window: the last K steps of the schedule (all of it, and
    # restarts, when K exceeds it); the steps before it run untimed
    K = args.steps
    prefix = wl.nsteps - K if K <= wl.nsteps else 0

    def timed_window(profile=False, only=None):
        """Fresh initial conditions, the untimed prefix, then the timed K
        steps; seconds, or with `profile` the per-kernel event table of the
        window (every kernel, or `only` that one, recorded)."""
        sim.init_ic(noise, a[0])
        kappa.zero_()
        run_steps(prefix, 0)
        sim.sync()
        if profile:
            sim.profile_only(only)
            sim.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(K, prefix)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if profile:
            prof = sim.profile_read()
            sim.profile(False)
            sim.profile_only(None)
            return prof if only is None else (t1 - t0, prof)
        return t1 - t0

    sim.init_ic(noise, a[0])
    run_steps(args.warmup, 0)
    prof = {}
    dom = None
    if not args.no_profile:
        # per-kernel table: an untimed pass of the window with events around
        # every launch (they cost time between kernels, so the timed repeats
        # below record only the dominant kernel)
        prof = timed_window(profile=True)
        # the shell projection runs on a second stream beside the force
        # transform, off the step's critical path: the dominant kernel is the
        # main stream's longest in total
        dom = max((k for k in prof if k not in SIDE_STREAM), key=lambda k: prof[k][0])
    times = []
    dom_ms, dom_cnt = 0.0, 0
    for _ in range(max(1, args.repeats)):
        if dom:
            t, pd = timed_window(profile=True, only=dom)
            ms, cnt = pd.get(dom, (0.0, 0))
            dom_ms += ms
            dom_cnt += cnt
        else:
            t = timed_window()
        times.append(t)
    elapsed = float(np.median(times))
    ps = wl.np_side ** 3 * K / elapsed
    ms_step = 1e3 * elapsed / K

    out = {
        "metric": "particle-steps/s at 256^3 (PM+lens) + HBM GB/s; p50/p99 served-sim latency",
        "value": ps, "unit": "particle-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "np": wl.np_side, "nm": wl.nm_side, "box": wl.box,
                   "a_range": [wl.a_start, wl.a_end], "nsteps_schedule": wl.nsteps,
                   "timed_steps": [prefix, prefix + K - 1] if K <= wl.nsteps else "restarts",
                   "maps": f"{len(wl.z_src)}x{wl.npix}^2 over {wl.fov_deg} deg",
                   "z_src": list(wl.z_src)},
        "repeats_ms_per_step": [1e3 * t / K for t in times],
        "timing": (f"median of {len(times)} repeats, each from fresh initial conditions with "
                   f"steps 0..{prefix - 1} untimed and steps {prefix}..{prefix + K - 1} timed"
                   if prefix else f"median of {len(times)} repeats of steps 0..{K - 1}"),
    }
    if prof:
        alg = algorithmic_bytes(wl)
        kern = {}
        total_ms = 0.0
        total_bytes = 0.0
        for name, (ms, cnt) in prof.items():
            b = alg.get(name, 0)
            avg = ms / max(cnt, 1)
            kern[name] = {"launches": cnt, "avg_ms": avg, "total_ms": ms,
                          "alg_bytes_per_launch": b,
                          "alg_gbs": (b / (avg * 1e-3) / 1e9) if avg > 0 and b else None}
            total_ms += ms
            total_bytes += b * cnt
        # the dominant kernel's launches inside the timed repeats
        avg_d = dom_ms / max(dom_cnt, 1)
        b_d = model_bytes(wl).get(dom, alg.get(dom, 0))
        b_own = alg.get(dom, 0)
        gbs_d = (b_d / (avg_d * 1e-3) / 1e9) if avg_d > 0 and b_d else None
        tr = load_traffic(wl.name)
        t_ent = tr.get(dom) if tr else None
        out["roofline"] = {
            "kernel": dom, "bound": "hbm", "achieved": gbs_d, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs_d / HBM_PEAK_GBS if gbs_d else None,
            "traffic": t_ent["bytes_per_launch"] if t_ent and t_ent["current"] else None,
            "avg_ms": avg_d, "launches": dom_cnt,
            "algorithmic_bytes": b_d,
            "algorithmic_bytes_what": BYTES_WHAT.get(dom, ("the kernel's own arrays",))[0],
            "achieved_own_bytes": (b_own / (avg_d * 1e-3) / 1e9) if avg_d > 0 and b_own else None,
            "own_bytes": b_own,
            "own_bytes_what": BYTES_WHAT.get(dom, ("", "the kernel's own arrays"))[-1]}
        out["hbm_effective_gbs_all_kernels"] = total_bytes / (total_ms * 1e-3) / 1e9
        kern_ms_step = total_ms / K
        if tr and "_step_bytes" in tr:
            stale = sorted(k for k, v in tr.items() if not k.startswith("_") and not v["current"])
            sb = tr["_step_bytes"]
            out["step_hbm"] = {
                "counter_bytes_per_step": sb, "counted_step": tr["_step"],
                "achieved_gbs_wall": sb / (ms_step * 1e-3) / 1e9,
                "frac_wall": sb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "achieved_gbs_kernel_time": sb / (kern_ms_step * 1e-3) / 1e9,
                "frac_kernel_time": sb / (kern_ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "gate": STEP_GATE, "stale_kernels": stale,
                "what": ("rocprofv3 FETCH_SIZE + WRITE_SIZE of every dispatch of one steady-state "
                         "step late in the schedule (profiles/traffic.json), divided by the "
                         "median ms per step of the timed window (wall) and by the summed "
                         "kernel time per step of the profiled pass")}
        out["kernels"] = kern
        out["kernels_note"] = ("per-kernel table from an untimed pass over the same window "
                               "with events around every launch; the timed repeats record "
                               "only the roofline's kernel")

    def mode_window(profile=False):
        return timed_window(profile=profile)
    if not args.no_interpolation:
        out["interpolation"] = mode_bench(sim, mode_window, wl, K, "interpolation")
        out["pgd"] = mode_bench(sim, mode_window, wl, K, "pgd")
        out["rotation"] = mode_bench(sim, mode_window, wl, K, "rotation")
    if not args.no_gradient:
        out["gradient"] = gradient_bench()
    if not args.no_serving:
        out["serving"] = serving_bench(args.serve_requests)
    if not args.no_large_mix:
        out["serving_large_mix"] = large_mix_bench()
    out["paper_context"] = ("MADLens on 32 Haswell cores: ~6.2e6 particle-steps/s "
                            "(256^3, 11 steps, 30 s incl. projection; different workload)")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    sim.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
