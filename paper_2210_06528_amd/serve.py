"""Continuous-batching serving loop for MFA encode requests on one GPU.

Requests (2-D or 3-D blocks of uneven size and degree) arrive over time.  The
scheduler admits them in arrival order whenever a slot is free and the device
memory they need (workspace, input, output) fits the HBM budget next to the
requests already resident.  Every slot is a worker thread that drives its
request through the C ABI on its own HIP stream (default priority): setup,
encode to the jump tolerance, decode.  The ctypes calls release the Python
GIL, so requests admitted while others are on the GPU overlap on the device;
a slot and its memory are released as soon as its request completes, and the
next waiting request is admitted at once.

Each request's control points stay on the device until the request
completes (its Schwarz state lives in the handle's workspace); results can be
kept for inspection.  Per-request kernels depend only on the request's own
shape, so a result is the same whether the request runs alone or in a mix.
"""
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import _lib
from . import workloads as W


def spectral_field_torch(shape, kmax, seed, device, nmodes=512):
    """The seeded spectral field of `workloads.field_spectral` evaluated as a
    separable sum: with G[k] = sum of a_m e^{i phi_m} over the modes m with
    wave vector k (|k_a| <= kmax), f = Re sum_k G[k] prod_a e^{i k_a x_a}, i.e.
    one small mode product per axis (real matrix products on the device, no
    FFT plan per shape).  Normalised to unit RMS, returned as float32."""
    import torch
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    K, amp, phase = W.spectral_modes(dim, nmodes, kmax, seed)
    r = 2 * kmax + 1
    G = np.zeros((r,) * dim, dtype=np.complex128)
    for k, a, ph in zip(K, amp, phase):
        G[tuple(int(v) + kmax for v in k)] += a * np.exp(1j * ph)
    T = torch.from_numpy(G).to(device)
    ks = torch.arange(-kmax, kmax + 1, dtype=torch.float64, device=device)
    # contract the last axes first; keep (Re, Im) while complex
    for a in range(dim - 1, 0, -1):
        x = 2.0 * np.pi * torch.arange(shape[a], dtype=torch.float64, device=device) / shape[a]
        E = torch.exp(1j * ks[:, None] * x[None, :])            # (r, m_a)
        T = torch.tensordot(T, E, dims=([a], [0]))               # axis a -> m_a, moved last
        T = torch.movedim(T, -1, a)
    x = 2.0 * np.pi * torch.arange(shape[0], dtype=torch.float64, device=device) / shape[0]
    ang = ks[:, None] * x[None, :]                              # (r, m_0)
    Tr = T.real.reshape(r, -1)
    Ti = T.imag.reshape(r, -1)
    f = torch.cos(ang).T @ Tr - torch.sin(ang).T @ Ti          # Re(E^T T)
    f = f.reshape(shape)
    f = f / torch.sqrt(torch.mean(f * f))
    return f.to(torch.float32).contiguous()


def spectral_field_gpu(shape, kmax, seed, device, nmodes=512):
    """Device copy of the seeded spectral field (see spectral_field_torch)."""
    return spectral_field_torch(shape, kmax, seed, device, nmodes)


def request_bytes(w: W.Workload):
    """Device bytes a request holds while resident: workspace, input, output."""
    ws = _lib.workspace_size(w.npts, w.degree, w.sizes, w.overlap, w.precision)
    return ws + 256 + 2 * 4 * w.npoints


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    sweeps: int = 0
    converged: bool = False
    jump: List[float] = field(default_factory=list)
    npoints: int = 0
    ctrl: Optional[np.ndarray] = None

    @property
    def latency(self):
        return self.done - self.arrival


class Server:
    def __init__(self, slots=8, hbm_budget=200e9, device="cuda:0", max_sweeps=300,
                 check_every=0, keep_results=False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.slots = slots
        self.budget = float(hbm_budget)
        self.max_sweeps = max_sweeps
        self.check_every = check_every
        self.keep = keep_results
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        _lib.load()

    def _work(self, slot, req, res, inputs):
        torch = self.torch
        w = req.workload
        s = self.streams[slot]
        with torch.cuda.stream(s):
            q = inputs(req) if callable(inputs) else inputs[req.rid]
            if q.device != self.device:
                q = q.to(self.device, non_blocking=False)
            enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, w.precision, w.combine,
                               device=self.device, stream=s)
            st = enc.encode(q, self.max_sweeps, w.jump_tol or 0.0, self.check_every,
                            raise_on_notconv=False)
            out = torch.empty(w.npts, dtype=torch.float32, device=self.device)
            enc.decode(out)
            if self.keep:
                res.ctrl = enc.get_ctrl().cpu().numpy()
            s.synchronize()
            enc.close()
            del enc, out, q
        res.sweeps = st["sweep"]
        res.converged = st["converged"]
        res.jump = st["jump"]
        res.npoints = w.npoints

    def run(self, requests: List[W.Request], inputs, time_scale=1.0,
            progress=None) -> Dict:
        """Serve `requests` (arrival times in seconds, scaled by time_scale).

        `inputs` maps a request to its device tensor (callable, or dict by rid).
        `progress(done, total)` is called about every 10 s while requests run.
        Returns the per-request results and the aggregate metrics.
        """
        pending = queue.Queue()
        results = {r.rid: Result(r.rid, 0.0) for r in requests}
        need = {r.rid: request_bytes(r.workload) for r in requests}
        for r in requests:
            if need[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs more than the HBM budget")
        lock = threading.Condition()
        state = {"resident": 0.0, "free": list(range(self.slots)), "done": 0, "err": None}
        t0 = time.perf_counter()

        def arrivals():
            for r in requests:
                delay = r.arrival * time_scale - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                results[r.rid].arrival = time.perf_counter() - t0
                pending.put(r)
            pending.put(None)

        def worker(slot, req):
            res = results[req.rid]
            try:
                self._work(slot, req, res, inputs)
            except Exception as e:  # surfaced after the run
                state["err"] = e
            res.done = time.perf_counter() - t0
            with lock:
                state["resident"] -= need[req.rid]
                state["free"].append(slot)
                state["done"] += 1
                lock.notify_all()

        th = threading.Thread(target=arrivals, daemon=True)
        th.start()
        threads = []
        waiting = []
        finished_arrivals = False
        last_report = time.perf_counter()
        while True:
            if progress is not None and time.perf_counter() - last_report > 10.0:
                last_report = time.perf_counter()
                progress(state["done"], len(requests))
            # collect arrivals without blocking while work is waiting
            try:
                item = pending.get(timeout=0.0005 if waiting else 0.05)
                if item is None:
                    finished_arrivals = True
                else:
                    waiting.append(item)
            except queue.Empty:
                pass
            with lock:
                while waiting and state["free"] and \
                        state["resident"] + need[waiting[0].rid] <= self.budget:
                    req = waiting.pop(0)
                    slot = state["free"].pop()
                    state["resident"] += need[req.rid]
                    results[req.rid].admitted = time.perf_counter() - t0
                    t = threading.Thread(target=worker, args=(slot, req), daemon=True)
                    threads.append(t)
                    t.start()
                if finished_arrivals and not waiting and state["done"] == len(requests):
                    break
                if waiting and (not state["free"] or
                                state["resident"] + need[waiting[0].rid] > self.budget):
                    lock.wait(timeout=0.05)
        for t in threads:
            t.join()
        if state["err"] is not None:
            raise state["err"]
        res = [results[r.rid] for r in requests]
        lat = np.array([r.latency for r in res]) * 1e3
        span = max(r.done for r in res) - min(r.arrival for r in res)
        pts = sum(r.npoints for r in res)
        return {"results": res, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "points_per_s": pts / span,
                "requests": len(res), "wall_s": span,
                "converged": int(sum(r.converged for r in res))}
