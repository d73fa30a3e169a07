"""Serving loop over the continuous-batching server of the C ABI.

``Server`` marshals the mf_server_* calls.  ``serve`` replays a list of
requests with given arrival times: requests are submitted when they arrive (a
few per iteration), every loop iteration runs one scheduling tick (admission
into free slots within the HBM budget + one batched step of everything
admitted) and collects the requests the server reports finished; latency is
arrival -> result on the host.  ``serve_sequential`` is the baseline: the same
requests served first come, first served, one solve at a time with its own
per-step launches.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import meso

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 64, precision: str = "fp32_fp64acc",
                 limiter: str = "vanleer", max_inflight: int = 4):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the server runs only on the GPU")
        self._lib = meso.load_library()
        self.precision = precision
        self.limiter = limiter
        cfg = meso.ServerConfig(int(hbm_budget), int(max_slots), meso.PRECISION[precision],
                                meso.LIMITER[limiter], int(max_inflight))
        h = C.c_void_p()
        meso._chk("mf_server_create", self._lib.mf_server_create(C.byref(cfg), None, C.byref(h)))
        self._h = h
        self._shape = {}

    @staticmethod
    def request_bytes(nx, ny, precision="fp32_fp64acc", mats=None) -> int:
        g = meso.make_grid(nx, ny, 1.0, 1.0)
        return int(meso.load_library().mf_server_request_bytes(C.byref(g), mats,
                                                              meso.PRECISION[precision]))

    def submit(self, sc, nsteps: int) -> int:
        g = meso.make_grid(sc.nx, sc.ny, sc.dx, sc.dy, sc.bc)
        mats = meso.materials_of(sc)
        opt = meso.Options(sc.cfl, sc.zeps, meso.LIMITER[self.limiter],
                           meso.PRECISION[self.precision], 1, 0)
        nc = 7 if mats[1].reactive else 6
        prim = np.ascontiguousarray(sc.prim, dtype=np.float64)
        assert prim.shape == (nc, sc.ny, sc.nx)
        t = C.c_uint64()
        meso._chk("mf_server_submit",
                  self._lib.mf_server_submit(self._h, C.byref(g), mats, C.byref(opt),
                                             meso._dptr(prim), int(nsteps), C.byref(t)))
        self._shape[t.value] = (nc, sc.ny, sc.nx)
        return t.value

    def tick(self):
        a, q = C.c_int32(), C.c_int32()
        meso._chk("mf_server_tick", self._lib.mf_server_tick(self._h, C.byref(a), C.byref(q)))
        return a.value, q.value

    def poll(self, ticket: int) -> int:
        st = C.c_int32()
        meso._chk("mf_server_poll", self._lib.mf_server_poll(self._h, ticket, C.byref(st)))
        return st.value

    def finished(self, capacity: int = 1024) -> list:
        """Tickets that finished (done or failed) since the last call."""
        buf = (C.c_uint64 * capacity)()
        n = C.c_int32()
        meso._chk("mf_server_finished", self._lib.mf_server_finished(self._h, buf, capacity,
                                                                      C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def result(self, ticket: int, out: np.ndarray | None = None):
        """(conserved planes, final time, steps) of a finished request; `out`
        (C-contiguous float64 of shape (planes, ny, nx)) is filled if given."""
        shape = self._shape.pop(ticket)
        if out is None:
            out = np.empty(shape, dtype=np.float64)
        assert out.shape == shape and out.dtype == np.float64 and out.flags["C_CONTIGUOUS"]
        t = C.c_double()
        n = C.c_int64()
        meso._chk("mf_server_result", self._lib.mf_server_result(self._h, ticket, meso._dptr(out),
                                                                 out.size, C.byref(t), C.byref(n)))
        return out, t.value, n.value

    def drain(self) -> None:
        meso._chk("mf_server_drain", self._lib.mf_server_drain(self._h))

    def stats(self) -> dict:
        st = meso.ServerStats()
        meso._chk("mf_server_get_stats", self._lib.mf_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in meso.ServerStats._fields_ if k != "reserved"}

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.mf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def serve(server: Server, requests, arrivals, nsteps: int, keep_results: bool = False,
          submit_per_tick: int = 8) -> dict:
    """Replay `requests` (scenarios) arriving at `arrivals` (s, sorted) through
    `server`; returns latencies, makespan and aggregate cell-updates/s.  At most
    `submit_per_tick` arrived requests are submitted between two ticks, so a
    burst of arrivals does not hold back the device."""
    n = len(requests)
    lat = np.zeros(n)
    results = [None] * n if keep_results else None
    outstanding = {}
    scratch = {}          # result buffers reused when results are not kept
    i = 0
    t0 = time.perf_counter()
    while i < n or outstanding:
        now = time.perf_counter() - t0
        k = 0
        while i < n and arrivals[i] <= now and k < submit_per_tick:
            outstanding[server.submit(requests[i], nsteps)] = i
            i += 1
            k += 1
        if not outstanding:
            time.sleep(max(0.0, min(arrivals[i] - now, 0.01)))
            continue
        server.tick()
        for tk in server.finished():
            k = outstanding.pop(tk)
            shape = (requests[k].prim.shape[0], requests[k].ny, requests[k].nx)
            buf = None
            if not keep_results:
                buf = scratch.get(shape)
                if buf is None:
                    buf = scratch[shape] = np.empty(shape)
            U, tf, steps = server.result(tk, buf)
            lat[k] = time.perf_counter() - t0 - arrivals[k]
            if keep_results:
                results[k] = (U, tf, steps)
    makespan = time.perf_counter() - t0
    work = float(sum(r.nx * r.ny for r in requests)) * nsteps
    out = {"p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99), "mean_s": float(lat.mean()),
           "makespan_s": makespan, "cell_updates_per_s": work / makespan, "latencies": lat,
           "stats": server.stats()}
    if keep_results:
        out["results"] = results
    return out


def solve_alone(sc, nsteps: int, precision: str = "fp32_fp64acc"):
    """One solve with its own launches (the per-solve baseline)."""
    with meso.Solver.from_scenario(sc, precision=precision) as s:
        s.run_steps(nsteps)
        U = s.read_conserved()
        t, n, _ = s.time()
    return U, t, n


def serve_sequential(requests, arrivals, nsteps: int, precision: str = "fp32_fp64acc") -> dict:
    """First come, first served, one solve at a time (per-solve launches)."""
    n = len(requests)
    lat = np.zeros(n)
    t0 = time.perf_counter()
    for k, sc in enumerate(requests):
        now = time.perf_counter() - t0
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        solve_alone(sc, nsteps, precision)
        lat[k] = time.perf_counter() - t0 - arrivals[k]
    makespan = time.perf_counter() - t0
    work = float(sum(r.nx * r.ny for r in requests)) * nsteps
    return {"p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99), "mean_s": float(lat.mean()),
            "makespan_s": makespan, "cell_updates_per_s": work / makespan, "latencies": lat}
