"""Differentiable convergence maps: torch.autograd.Function over the C ABI.

Forward: Zel'dovich initial conditions from white noise, the KDK steps and
the lens projection of every shell, keeping the state after each step as a
checkpoint in the library's own particle order (28 bytes per particle per
step in float32).  Backward: for each step in reverse, restore its end state
(which recomputes the force there), reverse its shell and its step, then
reverse the initial conditions.
Forward mode (jvp): the tangent of (x, p, f) is carried with every step and
each shell's tangent is accumulated, in one pass without checkpoints.  All
arithmetic runs in the library; this module only orders the calls.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

from .sim import Simulation


def forward_with_checkpoints(sim: Simulation, noise: torch.Tensor, a_grid: Sequence[float]):
    kappa = sim.new_maps()
    sim.init_ic(noise, a_grid[0])
    states = [sim.checkpoint()]
    for i in range(len(a_grid) - 1):
        sim.step(a_grid[i], a_grid[i + 1])
        sim.lens(a_grid[i], a_grid[i + 1], kappa)
        states.append(sim.checkpoint())
    return kappa, states


def reverse_pass(sim: Simulation, a_grid: Sequence[float], states, kappa_bar: torch.Tensor):
    """(noise_bar, dL/dOmega_m, dL/dsigma_8) for the cotangent kappa_bar."""
    n = len(a_grid) - 1
    kappa_bar = kappa_bar.to(device=sim.device, dtype=sim.dtype).contiguous()
    x_bar = torch.zeros((3, sim.n_particles), dtype=sim.dtype, device=sim.device)
    p_bar = torch.zeros_like(x_bar)
    # the cosmology cotangent accumulates on the device: no wait per call
    sim.vjp_cosmo_read()
    cb = None
    # with sub-evolution each shell also has the cotangent of its step's
    # drift momentum, which joins p_bar at that step's drift
    ph_bar = torch.zeros_like(x_bar) if sim.interpolation else None
    for i in range(n - 1, -1, -1):
        sim.restore(states[i + 1], a_grid[i + 1])
        if ph_bar is not None:
            ph_bar.zero_()
        sim.lens_vjp(a_grid[i], a_grid[i + 1], kappa_bar, x_bar, cb, ph_bar)
        a2 = a_grid[i + 2] if i + 1 < n else -1.0
        sim.step_vjp(a_grid[i], a_grid[i + 1], a2, x_bar, p_bar, cb, ph_bar)
    sim.restore(states[0], a_grid[0])
    noise_bar = sim.init_ic_vjp(a_grid[1], x_bar, p_bar, cb)
    g_om, g_s8 = sim.vjp_cosmo_read()
    return noise_bar, float(g_om), float(g_s8)


def jvp(sim: Simulation, noise: torch.Tensor, a_grid: Sequence[float], noise_dot: torch.Tensor,
        omega_m_dot: float = 0.0, sigma8_dot: float = 0.0):
    """(kappa, kappa_dot): the maps and their directional derivative along
    (noise_dot, Omega_m_dot, sigma8_dot), in one forward pass in which the
    library carries the tangent of (x, p, f) with every step (no
    checkpoints)."""
    kappa = sim.new_maps()
    kappa_dot = sim.new_maps()
    sim.init_ic(noise, a_grid[0])
    sim.init_ic_jvp(noise_dot, omega_m_dot, sigma8_dot)
    for i in range(len(a_grid) - 1):
        sim.step_jvp(a_grid[i], a_grid[i + 1])
        sim.lens(a_grid[i], a_grid[i + 1], kappa)
        sim.lens_jvp(a_grid[i], a_grid[i + 1], kappa_dot)
    return kappa, kappa_dot


class _Maps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, noise, omega_m, sigma8, sim, a_grid):
        # noise's own values feed the simulation; omega_m and sigma8 select
        # the cached handle (their values must match the handle's)
        kappa, states = forward_with_checkpoints(sim, noise, a_grid)
        ctx.sim, ctx.a_grid, ctx.states = sim, a_grid, states
        ctx.noise = noise
        return kappa

    @staticmethod
    def backward(ctx, kappa_bar):
        sim = ctx.sim
        # the reverse of the initial conditions needs this handle's noise copy
        sim.init_ic(ctx.noise, ctx.a_grid[0])
        noise_bar, g_om, g_s8 = reverse_pass(sim, ctx.a_grid, ctx.states, kappa_bar)
        dev = kappa_bar.device
        return (noise_bar.to(kappa_bar.dtype),
                torch.tensor(g_om, dtype=kappa_bar.dtype, device=dev),
                torch.tensor(g_s8, dtype=kappa_bar.dtype, device=dev), None, None)


class LensingModel:
    """kappa(noise, Omega_m, sigma_8) with gradients for all three inputs.

    One library handle is kept per (Omega_m, sigma_8); its device arena is
    allocated once and reused by every forward and backward pass.  `tangent`
    sizes the arenas for forward-mode tangents (`jvp`).
    """

    def __init__(self, np_side, nm_side, box, npix, fov_deg, z_src, a_grid,
                 dtype=torch.float32, interpolation=False, tangent=False, **cosmo):
        self.shape = (np_side, nm_side, box, npix, fov_deg, tuple(z_src))
        self.a_grid = [float(a) for a in a_grid]
        self.dtype = dtype
        self.interpolation = bool(interpolation)
        self.tangent = bool(tangent)
        self.cosmo = dict(cosmo)
        self._sims: Dict[Tuple[float, float], Simulation] = {}

    def sim_for(self, omega_m: float, sigma8: float) -> Simulation:
        key = (round(float(omega_m), 12), round(float(sigma8), 12))
        if key not in self._sims:
            np_side, nm_side, box, npix, fov, zs = self.shape
            self._sims[key] = Simulation(np_side, nm_side, box, npix, fov, zs, dtype=self.dtype,
                                         interpolation=self.interpolation,
                                         tangent=self.tangent, omega_m=key[0], sigma8=key[1],
                                         **self.cosmo)
        return self._sims[key]

    def __call__(self, noise: torch.Tensor, omega_m: torch.Tensor, sigma8: torch.Tensor):
        sim = self.sim_for(float(omega_m), float(sigma8))
        return _Maps.apply(noise, omega_m, sigma8, sim, self.a_grid)

    def jvp(self, noise: torch.Tensor, omega_m: float, sigma8: float, noise_dot: torch.Tensor,
            omega_m_dot: float = 0.0, sigma8_dot: float = 0.0):
        """(kappa, kappa_dot) at (noise, Omega_m, sigma_8) along the tangent
        (noise_dot, Omega_m_dot, sigma8_dot)."""
        return jvp(self.sim_for(float(omega_m), float(sigma8)), noise, self.a_grid, noise_dot,
                   omega_m_dot, sigma8_dot)

    def close(self):
        for s in self._sims.values():
            s.close()
        self._sims.clear()
