"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds only workload descriptions (sizes, cosmology, time grid,
map geometry, seeds) and the white-noise generator that feeds both the
HIP path and the float64 oracle.  It contains none of the method's
arithmetic: no transfer function, no growth factor, no FFT, no painting.

The shapes follow the paper's workloads (particle grids of 32^3..512^3,
force meshes at B = 1 or 2 times the particle grid, boxes of 128..410 Mpc/h,
11..40 steps, source redshifts up to 2; see the parameter table of the
MADLens design section).  No public dataset exists for this method: the
seeded Gaussian white noise below stands in for the paper's initial
conditions.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One simulation request: particle grid, mesh, box, time grid, maps."""
    name: str
    np_side: int            # particles per side (Np)
    nm_side: int            # force mesh cells per side (Nm = B * Np)
    box: float              # periodic box side, Mpc/h
    a_start: float
    a_end: float
    nsteps: int             # PM steps, linear in a
    npix: int               # convergence map pixels per side
    fov_deg: float          # map side, degrees
    z_src: Tuple[float, ...] = (1.0,)
    omega_m: float = 0.3
    sigma8: float = 0.8
    h: float = 0.7
    n_s: float = 0.96
    omega_b: float = 0.05
    t_cmb: float = 2.7255
    seed: int = 1

    @property
    def n_particles(self) -> int:
        return self.np_side ** 3

    def a_grid(self) -> np.ndarray:
        """Step boundaries a_0 < a_1 < ... < a_nsteps, linear in a."""
        return np.linspace(self.a_start, self.a_end, self.nsteps + 1)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads of the benchmark description, plus small parity cases.
CFG1 = Workload("plain_fp64_32p_32m", 32, 32, 128.0, 0.1, 1.0, 5, 64, 2.0,
                (1.0,), seed=1)
CFG2 = Workload("plain_fp32_256p_512m", 256, 512, 205.0, 0.01, 1.0, 40, 2048,
                5.0, (0.5, 1.0, 1.5, 2.0), seed=2)
CFG3 = Workload("grad_128p_256m", 128, 256, 128.0, 0.01, 1.0, 20, 1024, 2.0,
                (1.0,), seed=3)
CFG5 = Workload("large_512p_1024m", 512, 1024, 410.0, 0.01, 1.0, 40, 4096,
                5.0, tuple(np.round(np.linspace(0.2, 2.0, 10), 6)), seed=7)

# Serving request sizes: (Np, Nm, box) with box = Np Mpc/h.
SERVE_SIZES = ((64, 128, 64.0), (128, 256, 128.0), (192, 384, 192.0))


def serve_request(req_id: int, rng: np.random.Generator) -> Workload:
    """One serving request: size, step count and cosmology drawn from rng."""
    np_side, nm_side, box = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
    nsteps = int(rng.integers(10, 31))
    om = float(rng.uniform(0.25, 0.35))
    s8 = float(rng.uniform(0.7, 0.9))
    return Workload(f"req{req_id}", np_side, nm_side, box, 0.1, 1.0, nsteps,
                    512, 2.0, (1.0,), omega_m=om, sigma8=s8, seed=1000 + req_id)


def white_noise(np_side: int, seed: int) -> np.ndarray:
    """N(0,1) white noise on the Np^3 particle lattice, C order, float64.

    Drawn from numpy's Philox counter-based generator keyed by `seed`.
    """
    gen = np.random.Generator(np.random.Philox(key=seed))
    return gen.standard_normal(np_side ** 3).reshape((np_side,) * 3)


def single_mode_noise(np_side: int, n: Tuple[int, int, int],
                      amp: float = 1.0) -> np.ndarray:
    """A real cosine on the lattice: w = amp * cos(2 pi n . i / Np)."""
    i = np.indices((np_side,) * 3).astype(np.float64)
    ph = 2 * np.pi * (n[0] * i[0] + n[1] * i[1] + n[2] * i[2]) / np_side
    return amp * np.cos(ph)


def random_positions(n: int, box: float, seed: int) -> np.ndarray:
    """Uniform random positions in [0, box)^3, shape [3][n], float64."""
    gen = np.random.Generator(np.random.Philox(key=seed))
    return gen.uniform(0.0, box, size=(3, n))


def clustered_positions(np_side: int, nm_side: int, box: float, seed: int,
                        frac_clustered: float = 0.3,
                        n_clumps: int = 8) -> np.ndarray:
    """Particle positions in lattice order with a late-time-like mix.

    Each lattice particle is displaced by a small random offset; a fraction
    is moved into a few compact clumps (Gaussian, 0.5 cell wide) so that
    some cells hold thousands of particles.  Returns [3][Np^3] in [0, box).
    """
    gen = np.random.Generator(np.random.Philox(key=seed))
    n = np_side ** 3
    h = box / nm_side
    lat = box / np_side
    i = np.indices((np_side,) * 3).reshape(3, n).astype(np.float64)
    x = (i + 0.5) * lat + gen.normal(0.0, 2.0 * h, size=(3, n))
    centres = gen.uniform(0.0, box, size=(3, n_clumps))
    pick = gen.random(n) < frac_clustered
    which = gen.integers(0, n_clumps, size=n)
    m = np.nonzero(pick)[0]
    x[:, m] = centres[:, which[m]] + gen.normal(0.0, 0.5 * h, size=(3, m.size))
    return np.mod(x, box)


def random_momenta(n: int, scale: float, seed: int) -> np.ndarray:
    gen = np.random.Generator(np.random.Philox(key=seed))
    return gen.normal(0.0, scale, size=(3, n))
