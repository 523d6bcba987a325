"""Continuous-batching serving loop for MFA encode and refit requests on one GPU.

Requests (2-D or 3-D blocks of uneven size and degree) arrive over time.  An
encode request creates a model: a handle whose workspace holds the plan, the
factored local normal matrices, the control points and the Schwarz state.  A
refit request brings new data for a model that is still resident: its handle
skips the setup and its encode starts from the control points it holds
(Algorithm 1's branch for P != 0).  A model stays resident, its bytes counted
against the budget, until the last refit the stream holds for it is done.

The scheduler admits waiting requests in arrival order whenever a slot is
free and the device memory they need fits the HBM budget next to the
resident models and requests: an encode needs its workspace, input and
output, a refit only its input and output.  A refit whose model is still
busy (its previous request not done) waits without blocking the requests
behind it.  Every slot is one long-lived worker thread with its own HIP
stream (default priority) that drives its requests through the C ABI: setup
(encodes only), encode to the jump tolerance, decode.  The ctypes calls
release the Python GIL, so requests on different slots overlap on the
device; a slot and its request's bytes are released as soon as it completes,
and the next admissible request is admitted at once.

Per-request kernels and schedules depend only on the request's own shape, so
a result is the same whether the request runs alone or in a mix.
"""
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import _lib
from . import workloads as W


def spectral_field_torch(shape, kmax, seed, device, nmodes=512, t=0.0):
    """The seeded spectral field of `workloads.field_spectral` evaluated as a
    separable sum: with G[k] = sum of a_m e^{i (phi_m + |k_m| t)} over the
    modes m with wave vector k (|k_a| <= kmax), f = Re sum_k G[k] prod_a
    e^{i k_a x_a}, i.e. one small mode product per axis (real matrix products
    on the device, no FFT plan per shape).  t advances every mode's phase by
    |k| t (t = 0: the field itself).  Normalised to unit RMS, float32."""
    import torch
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    K, amp, phase = W.spectral_modes(dim, nmodes, kmax, seed)
    r = 2 * kmax + 1
    G = np.zeros((r,) * dim, dtype=np.complex128)
    for k, a, ph in zip(K, amp, phase):
        G[tuple(int(v) + kmax for v in k)] += a * np.exp(1j * (ph + np.linalg.norm(k) * t))
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


def spectral_field_gpu(shape, kmax, seed, device, nmodes=512, t=0.0):
    """Device copy of the seeded spectral field (see spectral_field_torch)."""
    return spectral_field_torch(shape, kmax, seed, device, nmodes, t)


def request_input(req, device):
    """The input of a request on the device: its model's field at time req.t."""
    w = req.workload
    return spectral_field_gpu(w.npts, w.extra["kmax"], w.seed, device, t=req.t)


def model_bytes(w: W.Workload):
    """Device bytes a resident model holds: its workspace."""
    return _lib.workspace_size(w.npts, w.degree, w.sizes, w.overlap, w.precision) + 256


def io_bytes(w: W.Workload):
    """Device bytes of one request's input and output (float32 each)."""
    return 2 * 4 * w.npoints


def request_bytes(w: W.Workload):
    """Device bytes an encode request holds while it runs: workspace, input, output."""
    return model_bytes(w) + io_bytes(w)


@dataclass
class Result:
    rid: int
    arrival: float
    kind: str = "encode"
    model: int = -1
    admitted: float = 0.0
    done: float = 0.0
    sweeps: int = 0
    converged: bool = False
    jump: List[float] = field(default_factory=list)
    npoints: int = 0
    ctrl: Optional[np.ndarray] = None
    slot: int = -1

    @property
    def latency(self):
        return self.done - self.arrival


class Server:
    """Slots are long-lived worker threads, each with its own HIP stream; the
    library keeps its auxiliary streams per host thread, so their number is
    bounded by the slot count however many requests are served."""

    def __init__(self, slots=8, hbm_budget=200e9, device="cuda:0", max_sweeps=300,
                 check_every=0, keep_results=False):
        """keep_results: True, False, or a predicate on the request: whose
        control points are copied to the host into the result."""
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
        self._jobs = [queue.Queue() for _ in range(slots)]
        self._workers = [threading.Thread(target=self._slot_loop, args=(s,), daemon=True)
                         for s in range(slots)]
        for t in self._workers:
            t.start()

    def close(self):
        """Stop the slot workers (idempotent)."""
        for q in self._jobs:
            q.put(None)
        for t in self._workers:
            t.join()
        self._workers = []

    def __del__(self):
        try:
            if self._workers:
                self.close()
        except Exception:
            pass

    def _slot_loop(self, slot):
        torch = self.torch
        torch.cuda.set_device(self.device)
        while True:
            job = self._jobs[slot].get()
            if job is None:
                return
            fn, done = job
            try:
                fn(slot)
                done(None)
            except Exception as e:  # surfaced by run()
                done(e)

    def _serve_one(self, slot, req, res, inputs, models, keep_model):
        torch = self.torch
        w = req.workload
        s = self.streams[slot]
        with torch.cuda.stream(s):
            q = inputs(req) if callable(inputs) else inputs[req.rid]
            if q.device != self.device:
                q = q.to(self.device, non_blocking=False)
            if req.kind == "refit":
                enc = models[req.model]
                enc.set_stream(s)
                enc.warm_start()
            else:
                enc = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, w.precision, w.combine,
                                   device=self.device, stream=s)
            st = enc.encode(q, self.max_sweeps, w.jump_tol or 0.0, self.check_every,
                            raise_on_notconv=False)
            out = torch.empty(w.npts, dtype=torch.float32, device=self.device)
            enc.decode(out)
            if self.keep(req) if callable(self.keep) else self.keep:
                res.ctrl = enc.get_ctrl().cpu().numpy()
            s.synchronize()
            if keep_model:
                models[req.model] = enc
            else:
                enc.close()
                models.pop(req.model, None)
            del out, q
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
        results = {r.rid: Result(r.rid, 0.0, r.kind, r.model) for r in requests}
        # refits of each model still to come: the model stays resident until
        # the last one is done
        refits_left = {}
        for r in requests:
            if r.kind == "refit":
                refits_left[r.model] = refits_left.get(r.model, 0) + 1
        known = {r.rid for r in requests if r.kind == "encode"}
        for r in requests:
            if r.kind == "refit" and r.model not in known:
                raise ValueError(f"refit {r.rid} names model {r.model}, not encoded in this run")
        need = {}
        for r in requests:
            w = r.workload
            need[r.rid] = io_bytes(w) + (model_bytes(w) if r.kind == "encode" else 0)
            if need[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs more than the HBM budget")
        lock = threading.Condition()
        models = {}                    # resident handles by model id
        busy = set()                   # models with a request in flight
        state = {"resident": 0.0, "free": list(range(self.slots)), "done": 0, "err": None,
                 "inflight": 0}
        t0 = time.perf_counter()

        def arrivals():
            for r in requests:
                delay = r.arrival * time_scale - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                results[r.rid].arrival = time.perf_counter() - t0
                pending.put(r)
            pending.put(None)

        def launch(slot, req):
            w = req.workload
            if req.kind == "refit":
                refits_left[req.model] -= 1
            keep_model = refits_left.get(req.model, 0) > 0
            res = results[req.rid]
            res.slot = slot

            def fn(s):
                self._serve_one(s, req, res, inputs, models, keep_model)

            def done(err):
                res.done = time.perf_counter() - t0
                with lock:
                    if err is not None:
                        state["err"] = err
                    # the request's input and output are freed; the model's
                    # workspace too once no refit is left for it
                    state["resident"] -= io_bytes(w)
                    if not keep_model:
                        state["resident"] -= model_bytes(w)
                    busy.discard(req.model)
                    state["free"].append(slot)
                    state["done"] += 1
                    state["inflight"] -= 1
                    lock.notify_all()

            self._jobs[slot].put((fn, done))

        th = threading.Thread(target=arrivals, daemon=True)
        th.start()
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
                if state["err"] is not None:
                    # a request failed: admit nothing more, let the others finish
                    if state["inflight"] == 0:
                        break
                    lock.wait(timeout=0.05)
                    continue
                i = 0
                while i < len(waiting) and state["free"]:
                    req = waiting[i]
                    if req.kind == "refit" and (req.model in busy or req.model not in models):
                        i += 1          # its model is busy or not created yet
                        continue
                    if state["resident"] + need[req.rid] > self.budget:
                        break           # admission in arrival order
                    waiting.pop(i)
                    slot = state["free"].pop()
                    state["resident"] += need[req.rid]
                    state["inflight"] += 1
                    busy.add(req.model)
                    results[req.rid].admitted = time.perf_counter() - t0
                    launch(slot, req)
                if finished_arrivals and not waiting and state["done"] == len(requests):
                    break
                if waiting:
                    lock.wait(timeout=0.05)
        for enc in list(models.values()):
            enc.close()
        models.clear()
        if state["err"] is not None:
            raise state["err"]
        res = [results[r.rid] for r in requests]
        lat = np.array([r.latency for r in res]) * 1e3
        span = max(r.done for r in res) - min(r.arrival for r in res)
        pts = sum(r.npoints for r in res)
        out = {"results": res, "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "points_per_s": pts / span,
               "requests": len(res), "wall_s": span,
               "converged": int(sum(r.converged for r in res))}
        ref = [r for r in res if r.kind == "refit"]
        if ref:
            enc_ = [r for r in res if r.kind == "encode"]
            out["refits"] = len(ref)
            out["mean_sweeps_encode"] = float(np.mean([r.sweeps for r in enc_])) if enc_ else 0.0
            out["mean_sweeps_refit"] = float(np.mean([r.sweeps for r in ref]))
        return out
