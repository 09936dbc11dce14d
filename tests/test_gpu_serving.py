"""The request loop (rbf_server_*) on the GPU, through the C ABI (-m gpu).

Isolation: every request's weights from a mix of concurrent requests equal,
bit for bit, the weights of the same request solved alone on a fresh handle,
whether the server advances the solves together in packed launches (with or
without the step captured as a graph) or runs each on its own stream.
Admission: with a budget that fits about two requests the server still
finishes every request, never charges more than the budget plus one request,
and releases everything at the end.  A failing request does not disturb the
others.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_0909_5413_amd as R
from paper_0909_5413_amd import workloads as W
from tests.gates import residual_gate

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return torch


def mix(k, seed_base):
    reqs = W.serving_requests(k, seed_base=seed_base, n_lo=2e3, n_hi=6e4, hs_lo=0.75)
    out = []
    for i, w in enumerate(reqs):
        pts = w.points()
        out.append((w, pts, w.values(pts), (R.RBF_FP64, R.RBF_MIXED, R.RBF_FP64_PC32)[i % 3]))
    return out


def alone(w, pts, f, prec):
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff, w.overlap)
    try:
        lam, info, st = R.rbf_solve(h, w.n, R.default_opts(rtol=w.rtol, precision=prec),
                                    ok=(R.RBF_OK, R.RBF_ENOCONV))
    finally:
        R.rbf_destroy(h)
    return lam, st


def oracle_judges(w, pts, f, lam, st):
    """A served request that reports convergence meets its tolerance by the
    oracle's own FP64 residual (Section 2.1's system, truncated matrix)."""
    if st != R.RBF_OK:
        return
    P = oracle.Problem(pts, w.sigma, w.cutoff, w.overlap)
    try:
        res = P.rel_residual(f, lam)
        gate = residual_gate(P, f, lam, w.rtol)
    finally:
        P.close()
    say("oracle residual", w.name, res, "gate", gate)
    assert res <= gate, (w.name, res, gate)


@pytest.mark.parametrize("packed,graphs,pmax", [(1, True, 0), (2, True, 0), (2, False, 0),
                                                (2, True, 12000), (0, False, 0)])
def test_mix_equals_alone(torch_dev, packed, graphs, pmax):
    """Every request of a mix served concurrently equals, bit for bit, the
    same request solved alone: with packed engines (every solve advanced in
    shared launches, with and without the step captured as a graph, and with
    the larger requests routed past the engines) and with one stream per
    request."""
    reqs = mix(8, 777000)
    ref = []
    for w, pts, f, prec in reqs:
        say("alone", w.name, w.n, w.h_over_sigma, prec)
        ref.append(alone(w, pts, f, prec))
    if pmax:
        n = [w.n for w, _, _, _ in reqs]
        assert min(n) <= pmax < max(n)
    say("serving packed", packed, "graphs", graphs, "pack_max_points", pmax)
    srv = R.rbf_server_create(max_active=4, packed=packed, graphs=graphs, pack_max_points=pmax)
    try:
        ids = [R.rbf_server_submit(srv, pts, f, w.sigma, w.cutoff, w.overlap,
                                   R.default_opts(rtol=w.rtol, precision=prec))
               for w, pts, f, prec in reqs]
        for (w, pts, f, prec), rid, (lam0, st0) in zip(reqs, ids, ref):
            lam, res, st = R.rbf_server_wait(srv, rid, w.n)
            say("mixed-in", w.name, R.status_name(st), res.latency, res.info.iterations)
            assert st == st0
            assert np.array_equal(lam, lam0)
            oracle_judges(w, pts, f, lam, st)
        stats = R.rbf_server_stats(srv)
        assert stats["finished"] == len(reqs) and stats["active"] == 0
        assert stats["bytes_charged"] == 0
    finally:
        R.rbf_server_destroy(srv)


def test_admission_budget_and_failures(torch_dev):
    reqs = mix(6, 888000)
    # one request with two identical points: fails alone, the others are unaffected
    w, pts, f, prec = reqs[2]
    bad = pts.copy()
    bad[5] = bad[9]
    reqs[2] = (w, bad, f, prec)
    srv0 = R.rbf_server_create(max_active=1)
    try:
        sizes = []
        for w, pts, f, prec in reqs:
            rid = R.rbf_server_submit(srv0, pts, f, w.sigma, w.cutoff, w.overlap,
                                      R.default_opts(rtol=w.rtol, precision=prec))
            _, res, _ = R.rbf_server_wait(srv0, rid, w.n, ok=tuple(range(11)))
            sizes.append(res.predicted_bytes)
    finally:
        R.rbf_server_destroy(srv0)
    budget = int(2.2 * max(sizes))
    srv = R.rbf_server_create(max_active=8, max_device_bytes=budget)
    try:
        ids = [R.rbf_server_submit(srv, pts, f, w.sigma, w.cutoff, w.overlap,
                                   R.default_opts(rtol=w.rtol, precision=prec))
               for w, pts, f, prec in reqs]
        peak = 0
        while True:
            s = R.rbf_server_stats(srv)
            peak = max(peak, s["bytes_charged"])
            if s["finished"] == len(reqs):
                break
            time.sleep(0.002)
        assert peak <= budget + max(sizes)
        for i, ((w, pts, f, prec), rid) in enumerate(zip(reqs, ids)):
            lam, res, st = R.rbf_server_wait(srv, rid, w.n, ok=tuple(range(11)))
            say("budgeted", w.name, R.status_name(st))
            if i == 2:
                assert st == R.RBF_EDUPLICATE
            else:
                assert st == R.RBF_OK
                lam0, st0 = alone(w, pts, f, prec)
                assert np.array_equal(lam, lam0)
                oracle_judges(w, pts, f, lam, st)
        assert R.rbf_server_stats(srv)["bytes_charged"] == 0
    finally:
        R.rbf_server_destroy(srv)


def test_packed_stream_of_uneven_requests(torch_dev):
    """A longer stream through the packed engine: 24 requests of uneven size
    and spacing (h/sigma down to 0.6, so some stop at the iteration cap),
    FP64, mixed and FP64 with FP32 local inverses, at most 6 on the device,
    arriving while others run: every
    status, iteration count and weight vector equals the lone solve's."""
    reqs = W.serving_requests(24, seed_base=555000, n_lo=1.5e3, n_hi=4e4)
    data = []
    for i, w in enumerate(reqs):
        pts = w.points()
        data.append((w, pts, w.values(pts), (R.RBF_MIXED, R.RBF_FP64, R.RBF_FP64_PC32)[i % 3]))
    srv = R.rbf_server_create(max_active=6)
    try:
        ids = []
        for k, (w, pts, f, prec) in enumerate(data):
            ids.append(R.rbf_server_submit(srv, pts, f, w.sigma, w.cutoff, w.overlap,
                                           R.default_opts(rtol=w.rtol, precision=prec,
                                                          max_iters=200)))
            if k % 4 == 3:
                time.sleep(0.01)
        got = [R.rbf_server_wait(srv, rid, w.n, ok=(R.RBF_OK, R.RBF_ENOCONV))
               for (w, _, _, _), rid in zip(data, ids)]
    finally:
        R.rbf_server_destroy(srv)
    for (w, pts, f, prec), (lam, res, st) in zip(data, got):
        h = R.rbf_setup(pts, f, w.sigma, w.cutoff, w.overlap)
        try:
            lam0, info0, st0 = R.rbf_solve(h, w.n, R.default_opts(rtol=w.rtol, precision=prec,
                                                                   max_iters=200),
                                           ok=(R.RBF_OK, R.RBF_ENOCONV))
        finally:
            R.rbf_destroy(h)
        say("packed stream", w.name, w.n, round(w.h_over_sigma, 3), prec, R.status_name(st),
            res.info.iterations, info0.iterations)
        assert st == st0 and res.info.iterations == info0.iterations
        assert res.info.outer_iterations == info0.outer_iterations
        assert np.array_equal(lam, lam0)
        oracle_judges(w, pts, f, lam, st)


def test_block_cache_reuse_is_clean(torch_dev):
    """Blocks handed back by one problem and reused by the next (dirty, of a
    nearby size) leave every result unchanged, and trimming empties the cache."""
    reqs = mix(3, 999000)
    R.rbf_block_cache(-1, trim=True)
    assert R.rbf_block_cache(-1) == 0
    w, pts, f, prec = reqs[0]
    say("cache fresh", w.name, w.n)
    lam0, st0 = alone(w, pts, f, R.RBF_FP64)
    idle = R.rbf_block_cache(-1)
    say("cache idle bytes", idle)
    assert idle > 0
    for w1, p1, f1, _ in reqs[1:]:
        say("cache other", w1.name, w1.n)
        alone(w1, p1, f1, R.RBF_MIXED)
    say("cache reuse", w.name, w.n)
    lam1, st1 = alone(w, pts, f, R.RBF_FP64)
    assert st1 == st0
    assert np.array_equal(lam1, lam0)
    R.rbf_block_cache(-1, trim=True)
    assert R.rbf_block_cache(-1) == 0


def test_stalled_mixed_requests_equal_alone(torch_dev):
    """Mixed requests at h/sigma = 0.6, whose outer refinement stalls and is
    undone: served by the packed engines (and by one stream per request) each
    ends as it does alone, with the same status, residual and weights."""
    reqs = W.serving_requests(3, seed_base=999000, n_lo=2e3, n_hi=8e3, hs_lo=0.6, hs_hi=0.62)
    data = [(w, w.points()) for w in reqs]
    opts = dict(rtol=1e-12, precision=R.RBF_MIXED, max_iters=600)
    ref = []
    for w, pts in data:
        f = w.values(pts)
        h = R.rbf_setup(pts, f, w.sigma, w.cutoff, w.overlap)
        try:
            lam, info, st = R.rbf_solve(h, w.n, R.default_opts(**opts),
                                        ok=(R.RBF_OK, R.RBF_ENOCONV))
            ref.append((lam, st, info.rel_residual))
        finally:
            R.rbf_destroy(h)
        say("alone", w.name, w.n, R.status_name(st), ref[-1][2])
    for packed in (2, 0):
        srv = R.rbf_server_create(max_active=3, packed=packed)
        try:
            ids = [R.rbf_server_submit(srv, pts, w.values(pts), w.sigma, w.cutoff, w.overlap,
                                       R.default_opts(**opts)) for w, pts in data]
            for (w, _), rid, (lam0, st0, rel0) in zip(data, ids, ref):
                lam, res, st = R.rbf_server_wait(srv, rid, w.n)
                say("served", packed, w.name, R.status_name(st), res.info.rel_residual)
                assert st == st0
                assert res.info.rel_residual == rel0
                assert np.array_equal(lam, lam0)
        finally:
            R.rbf_server_destroy(srv)


def test_stall_stop_equal_alone(torch_dev):
    """FP64 and FP64-with-FP32-inverse requests at h/sigma = 0.6, where
    restarted GMRES stagnates, with the stall stop on (stall_cycles = 2): alone
    each ends with RBF_ENOCONV after a few cycles, far below its iteration
    budget, its residual above half of its value two cycles earlier; served by
    the packed engines or one stream per request, each ends the same, bit for
    bit.  With the stop off the same solve runs to its budget."""
    reqs = W.serving_requests(3, seed_base=998000, n_lo=2e3, n_hi=8e3, hs_lo=0.6, hs_hi=0.62)
    data = [(w, w.points()) for w in reqs]
    ref = []
    for i, (w, pts) in enumerate(data):
        prec = (R.RBF_FP64, R.RBF_FP64_PC32)[i % 2]
        opts = dict(rtol=1e-12, precision=prec, max_iters=3000, stall_cycles=2)
        f = w.values(pts)
        h = R.rbf_setup(pts, f, w.sigma, w.cutoff, w.overlap)
        try:
            lam, info, st = R.rbf_solve(h, w.n, R.default_opts(**opts),
                                        ok=(R.RBF_OK, R.RBF_ENOCONV))
            d = info.as_dict()
            say("alone", w.name, w.n, R.status_name(st), d["iterations"], d["history"][-3:])
            assert st == R.RBF_ENOCONV and d["iterations"] < 3000
            hist = d["history"]
            assert len(hist) >= 3 and hist[-1] > 0.5 * hist[-3]
            assert "stalled" in R.last_error()
            ref.append((lam, st, info.rel_residual, opts))
            if i == 0:   # the stop off: the budget is spent
                _, info2, st2 = R.rbf_solve(h, w.n, R.default_opts(
                    rtol=1e-12, precision=prec, max_iters=150), ok=(R.RBF_OK, R.RBF_ENOCONV))
                assert st2 == R.RBF_ENOCONV and info2.iterations == 150
        finally:
            R.rbf_destroy(h)
    for packed in (2, 0):
        srv = R.rbf_server_create(max_active=3, packed=packed)
        try:
            ids = [R.rbf_server_submit(srv, pts, w.values(pts), w.sigma, w.cutoff, w.overlap,
                                       R.default_opts(**o)) for (w, pts), (_, _, _, o)
                   in zip(data, ref)]
            for (w, _), rid, (lam0, st0, rel0, _) in zip(data, ids, ref):
                lam, res, st = R.rbf_server_wait(srv, rid, w.n)
                say("served", packed, w.name, R.status_name(st), res.info.rel_residual)
                assert st == st0
                assert res.info.rel_residual == rel0
                assert np.array_equal(lam, lam0)
        finally:
            R.rbf_server_destroy(srv)


def test_stall_stop_leaves_converging_solves_alone(torch_dev):
    """A system that converges (c0, h/sigma = 0.8, to 1e-12 over two cycles)
    is not stopped by stall_cycles = 1, and its weights are bit-identical to
    the solve with the stop off."""
    w = W.C0
    pts = w.points()
    f = w.values(pts)
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff, w.overlap)
    try:
        lam0, i0, st0 = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-12))
        lam1, i1, st1 = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-12, stall_cycles=1))
        assert st0 == st1 == R.RBF_OK
        assert i0.iterations == i1.iterations and np.array_equal(lam0, lam1)
        with pytest.raises(R.RbfError) as e:
            R.rbf_solve(h, w.n, R.default_opts(rtol=1e-12, stall_cycles=-1))
        assert e.value.status == R.RBF_EINVAL
    finally:
        R.rbf_destroy(h)
