"""Write the stored expected values of the long GPU parity cases.

    python tests/golden/make_golden.py [schedule40 | grad | served192 | all]

Every value written here comes from the float64 oracle (`oracle/`) fed with
the seeded inputs of `workloads.py`; nothing is read from the HIP library.
The cases are those whose oracle run takes minutes, too long to repeat
inside the GPU test suite:

  schedule40  the headline schedule shape at 128^3 particles on a 256^3
              mesh: box 205 Mpc/h, 40 KDK steps linear in a from 0.01 to
              1.0, Born projection of every shell onto four 256^2 maps over
              5 x 5 deg at z_s = 0.5, 1, 1.5, 2 (design section: FastPM
              steps with the lightcone projected at the end of every step;
              notation section: the Born convergence).  Stores the four
              maps, and the final positions and momenta of every 32nd
              particle in lattice order.
  grad        the gradient workload: 128^3 particles, 256^3 mesh, box 128
              Mpc/h, 20 steps from a = 0.01, one 1024^2 map over 2 deg at
              z_s = 1, loss chi^2 = sum (kappa - kappa_t)^2 / sigma^2 with
              kappa_t the map of another seed plus N(0, sigma^2) pixel noise,
              sigma = 0.01 (appendix on cosmology derivatives: gradients
              with respect to the initial modes, Omega_m and sigma_8).
              Stores dL/dOmega_m, dL/dsigma_8, every 8th element of
              dL/dnoise, and every 16th pixel of the forward map.
  served192   one serving request of the largest serving size: 192^3
              particles, 384^3 mesh, box 192 Mpc/h, 10 steps from a = 0.1,
              one 512^2 map over 2 deg at z_s = 1, a cosmology inside the
              serving ranges (Omega_m in [0.25, 0.35], sigma_8 in [0.7,
              0.9]) and a seeded request noise; the noise is the
              oracle's own implementation of the counter-based generator
              the library draws on the device.  Stores the map and the
              final positions of every 128th particle.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint, lens, rng  # noqa: E402
from oracle.cosmology import Cosmology  # noqa: E402

# The cases, shared with the tests that read the files.
SCHEDULE40 = W.CFG2.with_(name="schedule40_128p_256m", np_side=128, nm_side=256, npix=256)
SCHEDULE40_STRIDE = 32     # particles stored: every 32nd in lattice order
GRAD = W.CFG3
GRAD_TARGET_SEED, GRAD_PIXEL_SEED, GRAD_SIGMA = 4, 5, 0.01
GRAD_NOISE_STRIDE, GRAD_MAP_STRIDE = 8, 16
SERVED192 = W.Workload("served192", 192, 384, 192.0, 0.1, 1.0, 10, 512, 2.0, (1.0,),
                       omega_m=0.3137, sigma8=0.7461, seed=1000 + 192)
SERVED192_STRIDE = 128     # particles stored: every 128th in lattice order


def path(name):
    return os.path.join(HERE, name + ".npz")


def cosmo_of(wl):
    return Cosmology(wl.omega_m, wl.h, wl.n_s, wl.sigma8, wl.omega_b, wl.t_cmb)


def pixel_noise(shape):
    """The target map's N(0, sigma^2) pixel noise (an input, not the method)."""
    gen = np.random.Generator(np.random.Philox(key=GRAD_PIXEL_SEED))
    return gen.normal(0.0, GRAD_SIGMA, size=shape)


def make_schedule40():
    wl = SCHEDULE40
    c = cosmo_of(wl)
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    noise = W.white_noise(wl.np_side, wl.seed)
    kappa, x, p = lens.run_lensing(noise, c, wl.box, wl.nm_side, wl.a_grid(), geom)
    s = SCHEDULE40_STRIDE
    np.savez_compressed(path(wl.name), kappa=kappa.astype(np.float32), x_sample=x[:, ::s],
                        p_sample=p[:, ::s], stride=s)


def make_grad():
    wl = GRAD
    c = cosmo_of(wl)
    a = wl.a_grid()
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    kt, _ = adjoint.forward_with_checkpoints(W.white_noise(wl.np_side, GRAD_TARGET_SEED), c,
                                             wl.box, wl.nm_side, a, geom)
    kt = kt + pixel_noise(kt.shape)
    noise = W.white_noise(wl.np_side, wl.seed)
    kappa, _ = adjoint.forward_with_checkpoints(noise, c, wl.box, wl.nm_side, a, geom)
    kbar = 2.0 * (kappa - kt) / GRAD_SIGMA ** 2
    terms = []
    nbar, g_om, g_s8 = adjoint.kappa_vjp_cosmo(noise, kbar, c, wl.box, wl.nm_side, a, geom,
                                               terms=terms)
    np.savez_compressed(path(wl.name), omega_m_bar=g_om, sigma8_bar=g_s8,
                        omega_m_terms_abs=float(np.sum(np.abs(terms))),
                        noise_bar_sample=nbar.ravel()[::GRAD_NOISE_STRIDE],
                        noise_bar_rms=float(np.sqrt(np.mean(nbar ** 2))),
                        kappa_sample=kappa.ravel()[::GRAD_MAP_STRIDE],
                        loss=float(np.sum((kappa - kt) ** 2) / GRAD_SIGMA ** 2),
                        noise_stride=GRAD_NOISE_STRIDE, map_stride=GRAD_MAP_STRIDE)


def make_served192():
    wl = SERVED192
    c = cosmo_of(wl)
    geom = lens.MapGeometry(wl.npix, wl.fov_deg, wl.z_src, c)
    noise = rng.white_noise(wl.np_side, wl.seed)
    kappa, x, _ = lens.run_lensing(noise, c, wl.box, wl.nm_side, wl.a_grid(), geom)
    s = SERVED192_STRIDE
    np.savez_compressed(path(wl.name), kappa=kappa.astype(np.float32), x_sample=x[:, ::s],
                        stride=s)


CASES = {"schedule40": make_schedule40, "grad": make_grad, "served192": make_served192}


if __name__ == "__main__":
    which = sys.argv[1:] or ["all"]
    for name in (CASES if which == ["all"] else which):
        t0 = time.time()
        CASES[name]()
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)
