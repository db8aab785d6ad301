"""Python front end of the C ABI: one simulation per handle.

Torch provides device memory and the HIP stream; every step of the
computation runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import LensParams, PmParams, check, lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_params(np_side, nm_side, box, omega_m=0.3, sigma8=0.8, h=0.7, n_s=0.96,
                omega_b=0.05, t_cmb=2.7255, dtype=torch.float32, modes=0):
    p = PmParams()
    p.modes = int(modes)
    p.np, p.nm, p.box = int(np_side), int(nm_side), float(box)
    p.omega_m, p.omega_b, p.h, p.n_s = float(omega_m), float(omega_b), float(h), float(n_s)
    p.sigma8, p.t_cmb = float(sigma8), float(t_cmb)
    p.dtype = _lib.PM_F64 if dtype == torch.float64 else _lib.PM_F32
    return p


def make_lens(npix, fov_deg, z_src: Sequence[float]):
    arr = (ctypes.c_double * len(z_src))(*[float(z) for z in z_src])
    l = LensParams()
    l.npix, l.fov_deg, l.nsrc = int(npix), float(fov_deg), len(z_src)
    l.z_src = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    l._keep = arr  # keep the host array alive for the call
    return l


def footprint(np_side, nm_side, box, npix, fov_deg, z_src, dtype=torch.float32, modes=0,
              **cosmo):
    p = make_params(np_side, nm_side, box, dtype=dtype, modes=modes, **cosmo)
    l = make_lens(npix, fov_deg, z_src)
    return int(lib().pm_footprint(ctypes.byref(p), ctypes.byref(l)))


class Simulation:
    """A PM + lightcone simulation resident on one GPU.

    `modes` (PM_MODE_* bits) sizes the arena for the optional passes: the PGD
    correction (implied by `pgd`) and forward-mode tangents (`tangent`);
    `ckpt_force` makes checkpoints carry the force at their state, so that a
    restore copies it back instead of recomputing it (larger checkpoints,
    faster reverse pass, the same values).
    """

    def __init__(self, np_side, nm_side, box, npix, fov_deg, z_src, *,
                 dtype=torch.float32, stream: Optional[torch.cuda.Stream] = None,
                 interpolation: bool = False, pgd=None, tangent: bool = False, modes: int = 0,
                 ckpt_force: bool = False, **cosmo):
        self.np_side, self.nm_side, self.box = int(np_side), int(nm_side), float(box)
        self.npix, self.fov_deg, self.z_src = int(npix), float(fov_deg), tuple(z_src)
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        modes = int(modes) | (_lib.PM_MODE_PGD if pgd is not None else 0) | \
            (_lib.PM_MODE_TANGENT if tangent else 0) | \
            (_lib.PM_MODE_CKPT_FORCE if ckpt_force else 0)
        self.modes = modes
        p = make_params(np_side, nm_side, box, dtype=dtype, modes=modes, **cosmo)
        l = make_lens(npix, fov_deg, z_src)
        h = ctypes.c_void_p()
        check(lib().pm_create(ctypes.byref(p), ctypes.byref(l),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "pm_create")
        self._h = h
        self.a = None
        self.interpolation = False
        if interpolation:
            self.set_interpolation(True)
        if pgd is not None:
            self.set_pgd(*pgd)

    @property
    def n_particles(self):
        return self.np_side ** 3

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the hot path -----------------------------------------------------
    def init_ic(self, noise: torch.Tensor, a0: float):
        noise = noise.to(device=self.device, dtype=self.dtype).contiguous()
        self._noise_keep = noise
        check(lib().pm_init_ic(self._h, _ptr(noise), float(a0)), "pm_init_ic")
        self.a = float(a0)

    def init_ic_seed(self, seed: int, a0: float):
        """Initial conditions from noise drawn on the device from `seed`."""
        check(lib().pm_init_ic_seed(self._h, int(seed), float(a0)), "pm_init_ic_seed")
        self.a = float(a0)

    def noise(self, seed: int) -> torch.Tensor:
        out = torch.empty((self.np_side,) * 3, dtype=self.dtype, device=self.device)
        check(lib().pm_noise(self._h, int(seed), _ptr(out)), "pm_noise")
        return out

    def reconfigure(self, box=None, fov_deg=None, z_src=None, **cosmo):
        """New cosmology / box / map geometry on the same arena."""
        self.box = float(box) if box is not None else self.box
        self.fov_deg = float(fov_deg) if fov_deg is not None else self.fov_deg
        if z_src is not None:
            if len(z_src) != len(self.z_src):
                raise ValueError("the number of source planes is fixed by the arena")
            self.z_src = tuple(z_src)
        p = make_params(self.np_side, self.nm_side, self.box, dtype=self.dtype, modes=self.modes,
                        **cosmo)
        l = make_lens(self.npix, self.fov_deg, self.z_src)
        check(lib().pm_reconfigure(self._h, ctypes.byref(p), ctypes.byref(l)), "pm_reconfigure")
        self.a = None

    def step(self, a0: float, a1: float):
        check(lib().pm_step(self._h, float(a0), float(a1)), "pm_step")
        self.a = float(a1)

    def set_interpolation(self, on: bool):
        """Sub-evolution projection on or off (pm_set_interpolation)."""
        check(lib().pm_set_interpolation(self._h, int(bool(on))), "pm_set_interpolation")
        self.interpolation = bool(on)

    def set_replica_rotation(self, seed):
        """Rotate every box replica by a cube symmetry hashed from its offsets
        and `seed` (an unsigned 64-bit int); None turns rotation off
        (pm_set_replica_rotation)."""
        on = seed is not None
        check(lib().pm_set_replica_rotation(self._h, int(on), int(seed or 0) & (2 ** 64 - 1)),
              "pm_set_replica_rotation")

    def set_pgd(self, alpha0: float, mu: float, k_l: float, k_s: float, on: bool = True):
        """PGD correction of the projected positions on (with its parameters:
        alpha = alpha0 a^mu, k_l and k_s in h/Mpc) or off (pm_set_pgd)."""
        check(lib().pm_set_pgd(self._h, int(bool(on)), float(alpha0), float(mu), float(k_l),
                               float(k_s)), "pm_set_pgd")

    def lens(self, a0: float, a1: float, kappa: torch.Tensor):
        check(lib().lens_project(self._h, float(a0), float(a1), _ptr(kappa)), "lens_project")

    def new_maps(self):
        return torch.zeros((len(self.z_src), self.npix, self.npix), dtype=self.dtype,
                           device=self.device)

    def steps(self, a_grid, kappa):
        """Steps along a_grid (from the current state at a_grid[0]) with the
        projection of every shell into kappa: pm_run, the fused form of
        step + lens per interval."""
        a = np.ascontiguousarray(a_grid, dtype=np.float64)
        check(lib().pm_run(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           len(a) - 1, _ptr(kappa)), "pm_run")
        self.a = float(a[-1])
        return kappa

    def run(self, noise, a_grid, kappa=None):
        """ICs at a_grid[0], then every step and its shell (pm_run)."""
        if kappa is None:
            kappa = self.new_maps()
        self.init_ic(noise, a_grid[0])
        return self.steps(a_grid, kappa)

    def run_stepwise(self, noise, a_grid, kappa=None):
        """The same with one pm_step and one lens_project per interval."""
        if kappa is None:
            kappa = self.new_maps()
        self.init_ic(noise, a_grid[0])
        for i in range(len(a_grid) - 1):
            self.step(a_grid[i], a_grid[i + 1])
            self.lens(a_grid[i], a_grid[i + 1], kappa)
        return kappa

    # -- state and introspection ------------------------------------------
    def get_state(self):
        n = self.n_particles
        x = torch.empty((3, n), dtype=self.dtype, device=self.device)
        p = torch.empty((3, n), dtype=self.dtype, device=self.device)
        a = ctypes.c_double()
        check(lib().pm_get_state(self._h, _ptr(x), _ptr(p), ctypes.byref(a)), "pm_get_state")
        return x, p

    def set_state(self, x: torch.Tensor, p: torch.Tensor, a: float):
        x = x.to(device=self.device, dtype=self.dtype).contiguous()
        p = p.to(device=self.device, dtype=self.dtype).contiguous()
        check(lib().pm_set_state(self._h, _ptr(x), _ptr(p), float(a)), "pm_set_state")
        self._state_keep = (x, p)
        self.a = float(a)

    def checkpoint(self) -> torch.Tensor:
        """The current state in the library's own particle order (a device
        byte tensor for restore)."""
        buf = torch.empty(int(lib().pm_checkpoint_bytes(self._h)), dtype=torch.uint8,
                          device=self.device)
        check(lib().pm_checkpoint_save(self._h, _ptr(buf)), "pm_checkpoint_save")
        return buf

    def restore(self, buf: torch.Tensor, a: float):
        """Restore a checkpoint at scale factor a (the force is recomputed)."""
        if buf.dtype != torch.uint8 or buf.numel() != int(lib().pm_checkpoint_bytes(self._h)):
            raise ValueError("not a checkpoint of this simulation's shape")
        check(lib().pm_checkpoint_load(self._h, _ptr(buf), float(a)), "pm_checkpoint_load")
        self.a = float(a)

    def get_force(self):
        nm, n = self.nm_side, self.n_particles
        rho = torch.empty((nm, nm, nm), dtype=self.dtype, device=self.device)
        fm = torch.empty((3, nm, nm, nm), dtype=self.dtype, device=self.device)
        acc = torch.empty((3, n), dtype=self.dtype, device=self.device)
        check(lib().pm_get_force(self._h, _ptr(rho), _ptr(fm), _ptr(acc)), "pm_get_force")
        return rho, fm, acc

    def sync(self):
        check(lib().pm_sync(self._h), "pm_sync")

    # -- reverse mode -------------------------------------------------------
    # cosmo_bar: a (2,) float64 numpy array, accumulated (the call waits for
    # the stream), or None: accumulated on the device, see vjp_cosmo_read
    @staticmethod
    def _cb(cosmo_bar):
        return None if cosmo_bar is None else (ctypes.c_double * 2)(*cosmo_bar)

    @staticmethod
    def _cb_back(cb, cosmo_bar):
        if cosmo_bar is not None:
            cosmo_bar[:] = list(cb)

    def lens_vjp(self, a0, a1, kappa_bar, x_bar, cosmo_bar, ph_bar=None):
        """x_bar += d kappa/dx^T kappa_bar (state at a1).  With sub-evolution
        on, ph_bar [3][Np^3] receives the drift momentum's cotangent
        (accumulated), for step_vjp."""
        cb = self._cb(cosmo_bar)
        check(lib().lens_project_vjp(self._h, float(a0), float(a1), _ptr(kappa_bar),
                                     _ptr(x_bar), _ptr(ph_bar), cb), "lens_project_vjp")
        self._cb_back(cb, cosmo_bar)

    def step_vjp(self, a0, a1, a2, x_bar, p_bar, cosmo_bar, ph_bar=None):
        cb = self._cb(cosmo_bar)
        check(lib().pm_step_vjp(self._h, float(a0), float(a1), float(a2), _ptr(x_bar),
                                _ptr(p_bar), _ptr(ph_bar), cb), "pm_step_vjp")
        self._cb_back(cb, cosmo_bar)

    def init_ic_vjp(self, a1, x_bar, p_bar, cosmo_bar):
        noise_bar = torch.empty((self.np_side,) * 3, dtype=self.dtype, device=self.device)
        cb = self._cb(cosmo_bar)
        check(lib().pm_init_ic_vjp(self._h, float(a1), _ptr(x_bar), _ptr(p_bar),
                                   _ptr(noise_bar), cb), "pm_init_ic_vjp")
        self._cb_back(cb, cosmo_bar)
        return noise_bar

    def vjp_cosmo_read(self):
        """(dL/dOmega_m, dL/dsigma_8) accumulated on the device by the reverse
        calls made with cosmo_bar=None; waits for the stream, then clears."""
        cb = (ctypes.c_double * 2)(0.0, 0.0)
        check(lib().pm_vjp_cosmo_read(self._h, cb), "pm_vjp_cosmo_read")
        return np.array(list(cb))

    # -- forward mode (tangents) -------------------------------------------
    def _tangent(self, t, shape):
        if t.dtype != self.dtype or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected a {self.dtype} tensor of shape {tuple(shape)}")
        return _ptr(t)

    def init_ic_jvp(self, noise_dot, omega_m_dot=0.0, sigma8_dot=0.0):
        """Start the tangent of the initial conditions that init_ic just made,
        along (noise_dot, Omega_m_dot, sigma8_dot); the library holds it."""
        nd = noise_dot.to(device=self.device, dtype=self.dtype).contiguous()
        check(lib().pm_init_ic_jvp(self._h, _ptr(nd), float(omega_m_dot), float(sigma8_dot)),
              "pm_init_ic_jvp")
        self._tangent_keep = nd

    def set_tangent(self, x_dot, p_dot, omega_m_dot=0.0):
        """Tangent (x_dot, p_dot) [3][Np^3] of the current state, lattice order."""
        sh = (3, self.n_particles)
        check(lib().pm_set_tangent(self._h, self._tangent(x_dot, sh), self._tangent(p_dot, sh),
                                   float(omega_m_dot)), "pm_set_tangent")
        self._tangent_keep = (x_dot, p_dot)

    def get_tangent(self):
        """(x_dot, p_dot, f_dot) [3][Np^3] in lattice order."""
        out = [torch.empty((3, self.n_particles), dtype=self.dtype, device=self.device)
               for _ in range(3)]
        check(lib().pm_get_tangent(self._h, *(_ptr(t) for t in out)), "pm_get_tangent")
        return tuple(out)

    def step_jvp(self, a0, a1):
        """pm_step(a0, a1) with the tangent carried along."""
        check(lib().pm_step_jvp(self._h, float(a0), float(a1)), "pm_step_jvp")
        self.a = float(a1)

    def lens_jvp(self, a0, a1, kappa_dot):
        """kappa_dot += the shell's tangent; state at a1."""
        check(lib().lens_project_jvp(self._h, float(a0), float(a1),
                                     self._tangent(kappa_dot, (len(self.z_src), self.npix,
                                                               self.npix))),
              "lens_project_jvp")

    def profile(self, enable: bool):
        check(lib().pm_profile(self._h, 1 if enable else 0), "pm_profile")

    def profile_only(self, name=None):
        """Record only launches of kernel `name` (None: every launch)."""
        check(lib().pm_profile_only(self._h, name.encode() if name else None),
              "pm_profile_only")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last read."""
        cap = 64
        names = ctypes.create_string_buffer(32 * cap)
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_long * cap)()
        n = ctypes.c_int()
        check(lib().pm_profile_read(self._h, cap, names, ms, cnt, ctypes.byref(n)),
              "pm_profile_read")
        out = {}
        for i in range(min(n.value, cap)):
            nm = names.raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (ms[i], cnt[i])
        return out

    def background(self, a):
        out = (ctypes.c_double * 3)()
        check(lib().pm_background(self._h, float(a), out), "pm_background")
        return tuple(out)


def run_noalloc(noise: torch.Tensor, a_grid, kappa: torch.Tensor, np_side, nm_side, box, npix,
                fov_deg, z_src, *, dtype=torch.float32, stream: Optional[torch.cuda.Stream] = None,
                **cosmo):
    """One whole simulation through pm_run_noalloc: initial conditions from
    `noise`, the steps of `a_grid` and their shells accumulated into `kappa`,
    with the arena in the library's static device scratch (nothing is
    allocated; the tensors are the caller's)."""
    st = stream if stream is not None else torch.cuda.current_stream()
    p = make_params(np_side, nm_side, box, dtype=dtype, **cosmo)
    l = make_lens(npix, fov_deg, z_src)
    a = np.ascontiguousarray(a_grid, dtype=np.float64)
    check(lib().pm_run_noalloc(ctypes.byref(p), ctypes.byref(l), ctypes.c_void_p(st.cuda_stream),
                               _ptr(noise), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               len(a) - 1, _ptr(kappa)), "pm_run_noalloc")
    return kappa


class Batch:
    """Same-shape simulations stepped together (pm_batch_*): one launch per
    pass over every slot, replayed from a HIP graph.  `shape` is any
    Simulation of the shape (its cosmology is not used)."""

    def __init__(self, shape: "Simulation", capacity: int, use_graph: bool = True,
                 stream: Optional[torch.cuda.Stream] = None):
        p = make_params(shape.np_side, shape.nm_side, shape.box, dtype=shape.dtype)
        l = make_lens(shape.npix, shape.fov_deg, shape.z_src)
        self.stream = stream
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        check(lib().pm_batch_create(ctypes.byref(p), ctypes.byref(l), int(capacity),
                                    int(bool(use_graph)), st, ctypes.byref(h)),
              "pm_batch_create")
        self._h = h
        self._sims = {}

    def attach(self, sim: "Simulation", a_grid, kappa: Optional[torch.Tensor] = None) -> int:
        a = np.ascontiguousarray(a_grid, dtype=np.float64)
        slot = ctypes.c_int32()
        check(lib().pm_batch_attach(self._h, sim._h,
                                    a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    len(a) - 1, ctypes.byref(slot)), "pm_batch_attach")
        self._sims[slot.value] = (sim, a)
        if kappa is not None:
            self.lens(sim, kappa)
        return slot.value

    def lens(self, sim: "Simulation", kappa: Optional[torch.Tensor]):
        check(lib().pm_batch_lens(self._h, sim._h, _ptr(kappa)), "pm_batch_lens")

    def step(self) -> int:
        """One fused step of every slot with steps left; returns how many
        still have steps left."""
        r = ctypes.c_int32()
        check(lib().pm_batch_step(self._h, ctypes.byref(r)), "pm_batch_step")
        return r.value

    def detach(self, sim: "Simulation"):
        check(lib().pm_batch_detach(self._h, sim._h), "pm_batch_detach")
        for k, (s, a) in list(self._sims.items()):
            if s is sim:
                del self._sims[k]
                if len(a) > 1:
                    sim.a = float(a[-1])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pm_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
