"""GPU checks of the continuous-batching serving loop.

A mix of 2-D/3-D requests of uneven size and degree is served with several
slots active at once; every result must equal the same request served alone
(bitwise: per-request kernels depend only on the request's own shape) and must
match the oracle's single-domain fit (the fixed point), and the loop must keep
its resident bytes within the budget.
"""
import numpy as np
import pytest

from oracle import schwarz
from paper_2210_06528_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _stream(n=10, seed=5):
    reqs = W.serving_stream(n, rate=500.0, seed=seed, side_lo=40, side_hi=96, block=8)
    return reqs


def _inputs(dev):
    from paper_2210_06528_amd.serve import spectral_field_gpu

    cache = {}

    def make(req):
        if req.rid not in cache:
            w = req.workload
            cache[req.rid] = spectral_field_gpu(w.npts, w.extra["kmax"], w.seed, dev)
        return cache[req.rid]
    return make, cache


def test_mix_equals_alone_and_oracle():
    from paper_2210_06528_amd.serve import Server
    dev = torch.device("cuda:0")
    reqs = _stream()
    make, cache = _inputs(dev)
    for r in reqs:
        make(r)
    torch.cuda.synchronize()
    mixed = Server(slots=4, keep_results=True).run(reqs, make, time_scale=0.0)
    assert mixed["converged"] == len(reqs)
    alone_srv = Server(slots=1, keep_results=True)
    for r, rm in zip(reqs, mixed["results"]):
        ra = alone_srv.run([W.Request(r.rid, 0.0, r.workload)], make)["results"][0]
        assert np.array_equal(ra.ctrl, rm.ctrl), r.rid
        w = r.workload
        S = schwarz.setup(schwarz.make_plan(w.npts, w.degree, w.sizes, w.overlap))
        Q = cache[r.rid].cpu().numpy().astype(np.float64)
        Pstar = schwarz.global_direct(S, Q)
        err = np.max(np.abs(rm.ctrl - Pstar)) / np.max(np.abs(Pstar))
        assert err < 1e-6, (r.rid, w.npts, w.degree, err)


def test_admission_respects_budget():
    from paper_2210_06528_amd.serve import Server, request_bytes
    dev = torch.device("cuda:0")
    reqs = _stream(8, seed=9)
    make, _ = _inputs(dev)
    biggest = max(request_bytes(r.workload) for r in reqs)
    # a budget that holds only the largest request at a time serialises the mix
    out = Server(slots=4, hbm_budget=biggest * 1.01).run(reqs, make, time_scale=0.0)
    assert out["converged"] == len(reqs)
    res = sorted(out["results"], key=lambda r: r.admitted)
    for a, b in zip(res, res[1:]):
        # with room for one request only, the next is admitted after the last finished
        assert b.admitted >= a.done - 1e-3 or \
            request_bytes(reqs[a.rid].workload) + request_bytes(reqs[b.rid].workload) <= biggest * 1.01
    with pytest.raises(ValueError):
        Server(slots=2, hbm_budget=biggest * 0.5).run(reqs, make, time_scale=0.0)
