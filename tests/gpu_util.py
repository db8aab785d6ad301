"""Helpers shared by the GPU tests: build simulations through the C ABI and
compare with the oracle."""
import sys

import numpy as np
import torch

import workloads as W


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def new_sim(wl: W.Workload, dtype=torch.float32, npix=None, fov=None, z_src=None, modes=0):
    from paper_2012_07266_amd import Simulation
    return Simulation(wl.np_side, wl.nm_side, wl.box,
                      npix if npix is not None else wl.npix,
                      fov if fov is not None else wl.fov_deg,
                      z_src if z_src is not None else wl.z_src,
                      dtype=dtype, modes=modes, omega_m=wl.omega_m, sigma8=wl.sigma8,
                      h=wl.h, n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb)


def cosmo_of(wl: W.Workload):
    from oracle.cosmology import Cosmology
    return Cosmology(wl.omega_m, wl.h, wl.n_s, wl.sigma8, wl.omega_b, wl.t_cmb)


def to_np(t):
    return t.detach().double().cpu().numpy()


def periodic_cells(dx, box, nm):
    """Minimum-image difference of positions, in mesh cells."""
    d = np.mod(dx + 0.5 * box, box) - 0.5 * box
    return np.abs(d) / (box / nm)


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))
