"""Python side of the serving loop (argument marshalling and the arrival
clock; admission, slots and stepping run in the library's own threads).

    srv = Server(hbm_budget_bytes, max_active)
    rid = srv.submit(workload)          # a workloads.Workload, seed = its seed
    kappa, (t_submit, t_admit, t_done) = srv.result(rid)

`run_stream` replays a stream of requests at their arrival times and
reports latency percentiles and throughput; `max_active = 1` is the plain
form (one simulation at a time, first in first out, the same kernels), and
`batched=True` steps the running requests of each shape together
(pm_srv_create_ex: batched launches replayed from a HIP graph) instead of
on streams of their own.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np
import torch

from . import _lib
from .sim import make_lens, make_params


def _check(rc, what):
    if rc != _lib.PM_OK:
        raise _lib.MadlensError(rc, what)


class Server:
    def __init__(self, hbm_budget: int, max_active: int, dtype=np.float32, batched=False):
        self._L = _lib.lib()
        self.dtype = np.dtype(dtype)
        h = ctypes.c_void_p()
        _check(self._L.pm_srv_create_ex(int(hbm_budget), int(max_active), int(bool(batched)),
                                        ctypes.byref(h)), "pm_srv_create_ex")
        self._h = h
        self._shapes = {}

    def submit(self, wl) -> int:
        tdt = torch.float64 if self.dtype == np.float64 else torch.float32
        p = make_params(wl.np_side, wl.nm_side, wl.box, omega_m=wl.omega_m, sigma8=wl.sigma8,
                        h=wl.h, n_s=wl.n_s, omega_b=wl.omega_b, t_cmb=wl.t_cmb, dtype=tdt)
        l = make_lens(wl.npix, wl.fov_deg, wl.z_src)
        r = _lib.PmRequest(p=p, l=l, a_start=wl.a_start, a_end=wl.a_end,
                           nsteps=wl.nsteps, seed=wl.seed)
        rid = ctypes.c_int64()
        _check(self._L.pm_srv_submit(self._h, ctypes.byref(r), ctypes.byref(rid)),
               "pm_srv_submit")
        self._shapes[rid.value] = (len(wl.z_src), wl.npix, wl.npix)
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0) -> bool:
        rc = self._L.pm_srv_wait(self._h, rid, float(timeout))
        if rc == _lib.PM_EAGAIN:
            return False
        _check(rc, "pm_srv_wait")
        return True

    def result(self, rid: int, timeout: float = -1.0):
        """Maps [nsrc][npix][npix] (host array) and (submit, admit, done) s."""
        if not self.wait(rid, timeout):
            raise TimeoutError(f"request {rid} not finished after {timeout} s")
        out = np.empty(self._shapes.pop(rid), dtype=self.dtype)
        t = (ctypes.c_double * 3)()
        _check(self._L.pm_srv_result(self._h, rid, out.ctypes.data_as(ctypes.c_void_p), t),
               f"request {rid}")
        return out, (t[0], t[1], t[2])

    def stats(self) -> dict:
        s = _lib.PmSrvStats()
        _check(self._L.pm_srv_stats_get(self._h, ctypes.byref(s)), "pm_srv_stats_get")
        return {f: getattr(s, f) for f, _ in _lib.PmSrvStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            self._L.pm_srv_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class StreamResult:
    latency_p50_ms: float
    latency_p99_ms: float
    latency_mean_ms: float
    throughput: float           # particle-steps/s over the makespan
    makespan_s: float
    n: int
    peak_running: int
    peak_bytes: int
    latencies_ms: List[float] = field(default_factory=list)  # per request, in order

    def as_dict(self) -> dict:
        return dict(self.__dict__)


def run_stream(requests: Sequence, arrivals: Sequence[float], hbm_budget: int,
               max_active: int, dtype=np.float32, keep_maps: bool = False, batched=False):
    """Submit requests[i] at time arrivals[i] (seconds from the start) and
    wait for all.  Returns (StreamResult, maps or None)."""
    maps: List = [None] * len(requests)
    with Server(hbm_budget, max_active, dtype, batched=batched) as srv:
        # untimed: one short request per shape, so that both forms start with
        # an arena of every shape in the pool
        shapes = {}
        for wl in requests:
            shapes.setdefault((wl.np_side, wl.nm_side, wl.npix, len(wl.z_src)), wl)
        for rid in [srv.submit(wl.with_(nsteps=1)) for wl in shapes.values()]:
            srv.result(rid)
        t0 = time.perf_counter()
        ids = []
        for wl, ta in zip(requests, arrivals):
            delay = t0 + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(wl))
        lat, first, last = [], None, None
        for i, rid in enumerate(ids):
            k, (ts, _, td) = srv.result(rid)
            if keep_maps:
                maps[i] = k
            lat.append(td - ts)
            first = ts if first is None else min(first, ts)
            last = td if last is None else max(last, td)
        st = srv.stats()
    work = sum(wl.np_side ** 3 * wl.nsteps for wl in requests)
    lat = np.array(lat) * 1e3
    res = StreamResult(float(np.percentile(lat, 50)), float(np.percentile(lat, 99)),
                       float(lat.mean()), work / (last - first), last - first, len(requests),
                       int(st["peak_running"]), int(st["peak_bytes"]), lat.tolist())
    return res, (maps if keep_maps else None)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    gen = np.random.Generator(np.random.Philox(key=seed))
    return np.cumsum(gen.exponential(1.0 / rate, size=n))
