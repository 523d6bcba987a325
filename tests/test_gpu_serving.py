"""GPU checks of the continuous-batching serving loop.

A mix of 2-D/3-D encode and refit requests of uneven size and degree is
served with several slots active at once.  Every result must equal the same
requests served one after another on a single slot (bitwise: per-request
kernels depend only on the request's own shape, and a refit starts from its
model's previous result), must match the oracle's single-domain fit of its
own data (the fixed point), and a refit on a resident model must give the
fit of a fresh encode of the same data.  Admission keeps the resident bytes
within the budget, and slots are long-lived worker threads.
"""
import threading

import numpy as np
import pytest

from oracle import schwarz
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _stream(n=10, seed=5, refit_frac=0.0):
    return W.serving_stream(n, rate=500.0, seed=seed, side_lo=40, side_hi=96, block=8,
                            refit_frac=refit_frac, refit_window=4, refit_dt=0.05)


def _inputs(dev):
    from paper_2210_06528_amd.serve import request_input

    cache = {}

    def make(req):
        if req.rid not in cache:
            cache[req.rid] = request_input(req, dev)
        return cache[req.rid]
    return make, cache


def _oracle_fit(w, Q):
    S = schwarz.setup(schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap))
    return schwarz.global_direct(S, Q.astype(np.float64))


def test_mix_equals_alone_and_oracle():
    from paper_2210_06528_amd.serve import Server
    dev = torch.device("cuda:0")
    reqs = _stream()
    make, cache = _inputs(dev)
    for r in reqs:
        make(r)
    torch.cuda.synchronize()
    srv = Server(slots=4, keep_results=True)
    mixed = srv.run(reqs, make, time_scale=0.0)
    srv.close()
    assert mixed["converged"] == len(reqs)
    alone_srv = Server(slots=1, keep_results=True)
    for r, rm in zip(reqs, mixed["results"]):
        ra = alone_srv.run([W.Request(r.rid, 0.0, r.workload)], make)["results"][0]
        assert np.array_equal(ra.ctrl, rm.ctrl), r.rid
        Pstar = _oracle_fit(r.workload, cache[r.rid].cpu().numpy())
        err = np.max(np.abs(rm.ctrl - Pstar)) / np.max(np.abs(Pstar))
        assert err < 1e-6, (r.rid, r.workload.npts, r.workload.degree, err)
    alone_srv.close()


def test_refits_on_resident_models():
    """Refits warm-start resident handles (no setup, no decoupled first
    sweep): each equals the same stream served in order on one slot, equals a
    fresh encode of its data within 1e-6, matches the oracle's fit of its
    data within 1e-6, and needs fewer sweeps than the encodes on average."""
    from paper_2210_06528_amd import _lib
    from paper_2210_06528_amd.serve import Server
    dev = torch.device("cuda:0")
    reqs = _stream(14, seed=8, refit_frac=0.45)
    kinds = [r.kind for r in reqs]
    assert kinds.count("refit") >= 3, kinds
    make, cache = _inputs(dev)
    for r in reqs:
        make(r)
    torch.cuda.synchronize()
    srv = Server(slots=4, keep_results=True)
    mixed = srv.run(reqs, make, time_scale=0.0)
    srv.close()
    assert mixed["converged"] == len(reqs)
    assert mixed["mean_sweeps_refit"] < mixed["mean_sweeps_encode"], mixed
    one = Server(slots=1, keep_results=True)
    seq = one.run(reqs, make, time_scale=0.0)
    one.close()
    for r, rm, rs in zip(reqs, mixed["results"], seq["results"]):
        assert rm.kind == r.kind and np.array_equal(rm.ctrl, rs.ctrl), r.rid
        if r.kind != "refit":
            continue
        w = r.workload
        fresh = _lib.Encoder(w.npts, w.degree, w.sizes, w.overlap, w.precision, device=dev)
        fresh.encode(cache[r.rid], 300, w.jump_tol, 0)
        Pf = fresh.get_ctrl().cpu().numpy()
        fresh.close()
        scale = np.max(np.abs(Pf))
        assert np.max(np.abs(rm.ctrl - Pf)) / scale < 1e-6, r.rid
        Pstar = _oracle_fit(w, cache[r.rid].cpu().numpy())
        assert np.max(np.abs(rm.ctrl - Pstar)) / np.max(np.abs(Pstar)) < 1e-6, r.rid


def test_admission_respects_budget():
    from paper_2210_06528_amd.serve import Server, request_bytes
    dev = torch.device("cuda:0")
    reqs = _stream(8, seed=9)
    make, _ = _inputs(dev)
    biggest = max(request_bytes(r.workload) for r in reqs)
    # a budget that holds only the largest request at a time serialises the mix
    srv = Server(slots=4, hbm_budget=biggest * 1.01)
    out = srv.run(reqs, make, time_scale=0.0)
    assert out["converged"] == len(reqs)
    res = sorted(out["results"], key=lambda r: r.admitted)
    for a, b in zip(res, res[1:]):
        # with room for one request only, the next is admitted after the last finished
        assert b.admitted >= a.done - 1e-3 or \
            request_bytes(reqs[a.rid].workload) + request_bytes(reqs[b.rid].workload) <= biggest * 1.01
    srv.close()
    small = Server(slots=2, hbm_budget=biggest * 0.5)
    with pytest.raises(ValueError):
        small.run(reqs, make, time_scale=0.0)
    small.close()


def test_slot_workers_are_long_lived():
    """Many more requests than slots run on the same slot threads (the
    library's auxiliary streams are kept per thread)."""
    from paper_2210_06528_amd.serve import Server
    dev = torch.device("cuda:0")
    reqs = _stream(24, seed=11)
    make, _ = _inputs(dev)
    before = {t.ident for t in threading.enumerate()}
    srv = Server(slots=3)
    workers = {t.ident for t in srv._workers}
    out = srv.run(reqs, make, time_scale=0.0)
    assert out["converged"] == len(reqs)
    assert {r.slot for r in out["results"]} <= {0, 1, 2}
    during = {t.ident for t in threading.enumerate()} - before
    assert workers <= during
    srv.close()
    assert not any(t.is_alive() for t in threading.enumerate() if t.ident in workers)
