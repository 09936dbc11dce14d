#!/usr/bin/env python3
"""Whole-job throughput of the Gaussian-RBF interpolation hot path on one MI355X.

One step = the whole hot path on the resident N = 1,000,000 workload (jittered
1000 x 1000 lattice on [-1, 1]^2, h/sigma = 0.8, cutoff 6 sigma, 3x3-cell RASM
subdomains, GMRES(30) to a relative residual of 1e-12): cell binning, local
Cholesky factorisations and inverse rows, and the preconditioned GMRES solve,
all through the C ABI on device buffers.

value = in-cutoff Gaussian interactions evaluated by the FP64 matvecs of the
timed steps / timed seconds (the metric's unit, whole job).  The JSON line also
carries the seconds to 1e-12 in FP64 and mixed precision, per-kernel rooflines
(HIP events on the library's stream), the request loop's solves/s and p50/p99
latency on the serving stream (FP64 and mixed), and the CPU oracle timed on a
bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gaussian matvec interactions/s; s to 1e-12 residual, FP64 vs mixed; p99 lat"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector (= FP64 matrix)
VALU_OPS_PER_S = 256 * 64 * 2.4e9   # one FP64 VALU lane-op per lane per clock
OPS_PER_INTERACTION = 20       # FP64 VALU ops charged per in-cutoff interaction


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def block_sizes(cell_start, ncx, ncy, overlap=1):
    """n_omega and n_c per cell from the binning (host arithmetic on counts)."""
    import numpy as np
    cnt = np.diff(cell_start.astype(np.int64)).reshape(ncy, ncx)
    pad = np.pad(cnt, overlap)
    k = 2 * overlap + 1
    tot = np.zeros_like(cnt)
    for dy in range(k):
        for dx in range(k):
            tot += pad[dy:dy + ncy, dx:dx + ncx]
    return tot.ravel(), cnt.ravel()


def step_kernel_flops(n_omega):
    """Algorithmic FP64 flops of the factorisation-step launches for blocks of
    n points: per 64-column block column J, the update of the rows below the
    diagonal block (2 * 64 * J flops per row) and their solve against the
    64x64 diagonal factor (64^2 flops per row)."""
    import numpy as np
    total = 0.0
    for n in np.asarray(n_omega, dtype=np.int64):
        J = np.arange(0, max(int(n) - 64, 0), 64, dtype=np.float64)
        rows = n - J - 64
        total += float(np.sum(rows * (128.0 * J + 4096.0)))
    return total


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current source of that kernel and of the
    headers it includes (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c1.md")
    if not os.path.exists(path):
        return None
    for m in re.finditer(r"^traffic (\S+) bytes_per_launch=(\S+) source=(\S+) sha256=(\S+)$",
                         open(path).read(), flags=re.M):
        name, val, src, sha = m.groups()
        if name != kernel:
            continue
        # the kernel's source file and the headers it includes, hashed in order
        h = hashlib.sha256()
        for f in src.split(","):
            h.update(open(os.path.join(ROOT, f), "rb").read())
        return float(val) if h.hexdigest() == sha else None
    return None


def serving_run(R, W, k, precision, max_active, max_iters, packed=2, n_hi=1e6, stall_cycles=0):
    """The request stream of the serving configuration through rbf_server_*:
    a closed-loop run (all k requests submitted at once) measures the capacity
    in solves/s, then an open-loop run submits the same requests at Poisson
    arrival times with 0.7x that rate and records each request's latency
    (submission to completion, the server's steady clock).  stall_cycles > 0
    lets the FP64 solves give up on a stagnating system (the library's
    stall stop); the mixed form has its own stop."""
    import numpy as np
    reqs = W.serving_requests(k, n_hi=n_hi)
    data = []
    for w in reqs:
        p = w.points()
        data.append((w, p, w.values(p)))

    def submit(srv, w, p, f):
        return R.rbf_server_submit(srv, p, f, w.sigma, w.cutoff, w.overlap,
                                   R.default_opts(rtol=w.rtol, precision=precision,
                                                  max_iters=max_iters,
                                                  stall_cycles=stall_cycles))

    everything = tuple(range(11))
    srv = R.rbf_server_create(max_active=max_active, packed=packed)
    try:
        t0 = time.perf_counter()
        ids = [submit(srv, w, p, f) for w, p, f in data]
        closed = [R.rbf_server_wait(srv, i, w.n, ok=everything) for (w, _, _), i in zip(data, ids)]
        makespan = time.perf_counter() - t0
    finally:
        R.rbf_server_destroy(srv)
    cap = k / makespan
    rate = 0.7 * cap
    arrivals = np.cumsum(np.random.default_rng(W.SEED_BASE * 1000 + 999).exponential(1.0 / rate, k))
    srv = R.rbf_server_create(max_active=max_active, packed=packed)
    try:
        t0 = time.perf_counter()
        ids = []
        for (w, p, f), ta in zip(data, arrivals):
            delay = t0 + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(submit(srv, w, p, f))
        opened = [R.rbf_server_wait(srv, i, w.n, ok=everything) for (w, _, _), i in zip(data, ids)]
        span = time.perf_counter() - t0
    finally:
        R.rbf_server_destroy(srv)
    lat = np.array([r.latency for _, r, _ in opened])
    status = [st for _, _, st in opened]
    conv = np.array([r.latency for _, r, st in opened if st == R.RBF_OK])
    return {
        "requests": k,
        "precision": {R.RBF_FP64: "fp64", R.RBF_MIXED: "mixed"}.get(precision, "fp64_pc32"),
        "mode": f"{packed} packed engines" if packed else "one stream per request",
        "max_active": max_active, "max_iters": max_iters, "n_hi": n_hi,
        "stall_cycles": stall_cycles if precision != R.RBF_MIXED else None,
        "converged_latency_p50_s": float(np.percentile(conv, 50)) if conv.size else None,
        "converged_latency_p99_s": float(np.percentile(conv, 99)) if conv.size else None,
        "capacity_solves_per_s": cap, "offered_rate_per_s": rate,
        "completed_solves_per_s": k / span,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "ok": status.count(R.RBF_OK), "enoconv": status.count(R.RBF_ENOCONV),
        "other": len(status) - status.count(R.RBF_OK) - status.count(R.RBF_ENOCONV),
        "closed_loop_ok": sum(1 for _, _, st in closed if st == R.RBF_OK),
    }


def event_time(torch, stream, fn, reps):
    """Average milliseconds of fn() over reps launches, HIP events on stream."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def event_median(torch, stream, fn, warmup, reps):
    """Median milliseconds of fn() over reps launches, each bracketed by its
    own HIP event pair on stream, after warmup untimed launches."""
    import numpy as np
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    ev[-1][1].synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def eval_run(R, torch, w, d_pts, d_f, d_lam, stream, opts):
    """rbf_evaluate_device at two target sets of about N points each, after an
    FP64 solve: its median time over 20 event-timed calls after 3, the
    in-cutoff interactions it sums (rbf_target_counts_device) and their rate
    against R64."""
    import numpy as np
    from paper_0909_5413_amd import workloads as W
    lo = d_pts.min(dim=0).values.cpu().numpy()
    hi = d_pts.max(dim=0).values.cpu().numpy()
    sets = {"staggered_lattice": W.staggered_lattice(w.n_side),
            "uniform": np.random.default_rng(W.SEED_BASE + 21).uniform(lo, hi, (w.n, 2))}
    out = {}
    h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
    try:
        R.rbf_precond_setup(h, R.RBF_FP64, stream)
        R.rbf_solve_device(h, d_lam, opts)
        # candidates: the sources of the 3x3 cell block around each target's
        # (clamped) cell, every one of which the kernel evaluates
        (x0, y0, _, inv), (ncx, ncy) = R.rbf_grid(h)
        _, _, cs = R.rbf_binning(h, w.n)
        cnt = np.diff(cs.astype(np.int64)).reshape(ncy, ncx)
        pad = np.zeros((ncy + 2, ncx + 2), np.int64)
        pad[1:-1, 1:-1] = cnt
        block = sum(pad[1 + dy:ncy + 1 + dy, 1 + dx:ncx + 1 + dx]
                    for dy in (-1, 0, 1) for dx in (-1, 0, 1))
        for name, tg in sets.items():
            d_t = torch.tensor(tg, device=d_pts.device)
            m = tg.shape[0]
            d_s = torch.empty(m, device=d_pts.device, dtype=torch.float64)
            d_c = torch.empty(m, device=d_pts.device, dtype=torch.int32)
            R.rbf_target_counts_device(h, d_t, m, d_c, stream)
            inter = int(d_c.to(torch.int64).sum().item())
            ms = event_median(torch, stream, lambda: R.rbf_evaluate_device(h, d_t, m, d_s, stream),
                              3, 20)
            rate = inter / (ms * 1e-3)
            cx = np.clip(np.floor((tg[:, 0] - x0) * inv).astype(np.int64), 0, ncx - 1)
            cy = np.clip(np.floor((tg[:, 1] - y0) * inv).astype(np.int64), 0, ncy - 1)
            cand = int(block[cy, cx].sum())
            out[name] = {"targets": m, "ms": ms, "evaluations_per_s": m / (ms * 1e-3),
                         "interactions": inter, "interactions_per_s": rate,
                         "frac_r64": rate * OPS_PER_INTERACTION / VALU_OPS_PER_S,
                         "candidate_pairs": cand, "in_cutoff_share": inter / cand,
                         "candidate_pairs_per_s": cand / (ms * 1e-3)}
        # the same staggered lattice through the lattice entry point (targets
        # x0 + a h, the cells' shared 3x3 blocks and separable factors)
        n1, hh = w.n_side - 1, w.h
        x0l = -1.0 + hh
        ax = x0l + np.arange(n1, dtype=np.float64) * hh
        gx, gy = np.meshgrid(ax, ax, indexing="xy")
        tg = np.ascontiguousarray(np.stack([gx.ravel(), gy.ravel()], axis=1))
        m = tg.shape[0]
        d_t = torch.tensor(tg, device=d_pts.device)
        d_c = torch.empty(m, device=d_pts.device, dtype=torch.int32)
        R.rbf_target_counts_device(h, d_t, m, d_c, stream)
        inter = int(d_c.to(torch.int64).sum().item())
        d_s = torch.empty(m, device=d_pts.device, dtype=torch.float64)
        ms = event_median(torch, stream, lambda: R.rbf_evaluate_lattice_device(
            h, x0l, x0l, hh, hh, n1, n1, d_s, stream), 3, 20)
        rate = inter / (ms * 1e-3)
        out["staggered_lattice_separable"] = {
            "targets": m, "ms": ms, "evaluations_per_s": m / (ms * 1e-3), "interactions": inter,
            "interactions_per_s": rate, "frac_r64": rate * OPS_PER_INTERACTION / VALU_OPS_PER_S,
            "speedup_vs_targets": out["staggered_lattice"]["ms"] / ms}
    finally:
        R.rbf_destroy(h)
    return out


def geometry_solve(R, torch, w, d_pts, d_f, d_lam, stream, B, D, precision, reps=3, T=0.0):
    """Seconds from the resident points to weights at the workload's tolerance
    with box subdomains (setup, geometry, local factorisations, solve): the
    median of reps - 1 runs after one warm-up.  T > 0 truncates the product
    by the square of side T around each box instead of the radial cutoff."""
    import ctypes as C
    import numpy as np
    times, info, zbytes = [], None, 0.0
    opts = R.default_opts(rtol=w.rtol, precision=precision, stream=stream, max_iters=2000)
    for rep in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
        try:
            R.rbf_set_geometry(h, B, D, T, stream=stream)
            R.rbf_precond_setup(h, precision, stream)
            inf, st = R.rbf_solve_device(h, d_lam, opts, ok=(R.RBF_OK, R.RBF_ENOCONV))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            info = inf.as_dict()
            info["status"] = R.status_name(st)
            if rep == 0:
                nx = int(np.floor((float(d_pts[:, 0].max()) - float(d_pts[:, 0].min())) * (1.0 / B))) + 1
                ny = int(np.floor((float(d_pts[:, 1].max()) - float(d_pts[:, 1].min())) * (1.0 / B))) + 1
                no, nc = C.c_int(), C.c_int()
                for b in range(nx * ny):
                    R.lib().rbf_precond_block(h, b, precision, None, None, C.byref(no), C.byref(nc))
                    zbytes += float(no.value) * nc.value
        finally:
            R.rbf_destroy(h)
    s = 8.0 if precision == R.RBF_FP64 else 4.0
    rec = {"s_to_tol": float(np.median(times[1:])), "status": info["status"],
           "iterations": info["iterations"], "outer": info["outer_iterations"],
           "rel_residual": info["rel_residual"], "t_pcsetup": info["t_pcsetup"],
           "z_bytes": zbytes * s}
    if T > 0 and info["matvecs64"] > 0:   # the box-truncated product as launched in the solve
        ms = 1e3 * info["t_matmult"] / info["matvecs64"]
        pairs = info["interactions_per_matvec"]
        rec.update({"T_over_sigma": T / w.sigma, "pairs_per_matvec": pairs,
                    "matvec_ms": ms, "pairs_per_s": pairs / (ms * 1e-3),
                    "frac_r64": pairs / (ms * 1e-3) * OPS_PER_INTERACTION / VALU_OPS_PER_S})
    return rec


def paper_truncation(w, B):
    """The paper's box truncation side (Section 3.2): the box widened by 6 sigma
    on every side at h/sigma = 0.8, by 4 sigma from 0.9 up."""
    return B + 2 * (6.0 if w.h_over_sigma < 0.85 else 4.0) * w.sigma


def geometry_sweep(R, torch, w, d_pts, d_f, d_lam, stream, ratios, box_t):
    """Iterations and seconds to the workload's tolerance (FP64) over B in
    {3, 4, 5, 6, 7} sigma and D in {1.5, 1.7, 1.9, 2.1, 2.3} B (the study of
    Figs. 6 and 7), at each h/sigma in ratios on the same points (sigma and the
    cutoff follow the ratio), with the radial cutoff or the paper's box
    truncation."""
    import dataclasses
    rows = []
    for r in ratios:
        wr = dataclasses.replace(w, name=f"{w.name}_hs{r}", h_over_sigma=r)
        for Bs in (3.0, 4.0, 5.0, 6.0, 7.0):
            for Dr in (1.5, 1.7, 1.9, 2.1, 2.3):
                B = Bs * wr.sigma
                T = paper_truncation(wr, B) if box_t else 0.0
                res = geometry_solve(R, torch, wr, d_pts, d_f, d_lam, stream, B, Dr * B,
                                     R.RBF_FP64, reps=2, T=T)
                rows.append({"h_over_sigma": r, "B_over_sigma": Bs, "D_over_B": Dr,
                             "T_over_sigma": T / wr.sigma, **res})
                log("sweep", rows[-1])
    return rows


def geometry_run(R, torch, w, d_pts, d_f, d_lam, stream, sweep, ratios=(), box_t=False):
    """The paper's optimum B = 5 sigma, D = 1.9 B (Section 3.2) on the
    workload, FP64 and mixed; with sweep, iterations and seconds over
    B in {3, 4, 5, 6, 7} sigma and D in {1.5, 1.7, 1.9, 2.1, 2.3} B."""
    out = {"B_over_sigma": 5.0, "D_over_B": 1.9}
    B = 5.0 * w.sigma
    for tag, prec in (("fp64", R.RBF_FP64), ("mixed", R.RBF_MIXED)):
        out[tag] = geometry_solve(R, torch, w, d_pts, d_f, d_lam, stream, B, 1.9 * B, prec)
        log("geometry", tag, out[tag])
    T = paper_truncation(w, B)
    for tag, prec in (("fp64_boxT", R.RBF_FP64), ("fp64_pc32_boxT", R.RBF_FP64_PC32)):
        out[tag] = geometry_solve(R, torch, w, d_pts, d_f, d_lam, stream, B, 1.9 * B, prec, T=T)
        log("geometry", tag, out[tag])
    if sweep:
        out["sweep_fp64" + ("_boxT" if box_t else "")] = geometry_sweep(
            R, torch, w, d_pts, d_f, d_lam, stream, ratios or (w.h_over_sigma,), box_t)
    return out


def host_memory_gib():
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    return int(line.split()[1]) / 2 ** 20
    except OSError:
        pass
    return None


def cpu_baseline(workload, n_side, targets=None):
    """The oracle (setup with every local factor kept, FP64 GMRES(30) to the
    workload's tolerance) on the workload itself, or on an n_side lattice of
    the same spacing when n_side is smaller.  Returns the record, and on the
    full workload also the oracle's weights and its interpolant at targets."""
    import numpy as np
    import oracle
    from paper_0909_5413_amd import workloads as W
    w = workload if (not n_side or n_side >= workload.n_side) else W.sub_lattice(workload, n_side)
    pts = w.points()
    f = w.values(pts)
    P = oracle.Problem(pts, w.sigma, w.cutoff, w.overlap)
    _, nnb = P.matvec(np.ones(w.n), with_counts=True)
    inter = int(nnb.sum())
    P.close()
    t0 = time.perf_counter()
    P = oracle.Problem(pts, w.sigma, w.cutoff, w.overlap)
    P.rasm_setup()
    x, info = P.gmres(f, 30, workload.rtol)
    dt = time.perf_counter() - t0
    matvecs = info.iterations + len(info.history)
    s = P.evaluate(x, targets) if (targets is not None and w is workload) else None
    P.close()
    rec = {
        "value": inter * matvecs / dt, "unit": "interactions/s",
        "cores": oracle.num_threads(), "kind": "oracle",
        "sample": (f"oracle setup (every local Cholesky factor kept) + FP64 GMRES(30) solve to "
                   f"{workload.rtol:g} on {'the workload itself' if w is workload else 'a sample'}:"
                   f" {w.n_side}x{w.n_side} jittered lattice (N={w.n}), {matvecs} matvecs x "
                   f"{inter} interactions in {dt:.2f} s"),
        "seconds": dt, "iterations": info.iterations, "rel_residual": info.rel_residual,
        "host_memory_gib": host_memory_gib(),
    }
    return rec, (x if w is workload else None), s


def oracle_matvec_1thread(names):
    """One oracle matvec per workload on one thread (w ~ U(-1, 1))."""
    import numpy as np
    import oracle
    from paper_0909_5413_amd import workloads as W
    threads = oracle.num_threads()
    out = {}
    oracle.set_num_threads(1)
    try:
        for name in names:
            w = W.WORKLOADS[name]
            pts = w.points()
            P = oracle.Problem(pts, w.sigma, w.cutoff, w.overlap)
            wv = W.random_weights(w.n, W.SEED_BASE + 11)
            t0 = time.perf_counter()
            _, nnb = P.matvec(wv, with_counts=True)
            dt = time.perf_counter() - t0
            P.close()
            out[name] = {"seconds": dt, "interactions_per_s": float(nnb.sum()) / dt, "threads": 1}
    finally:
        oracle.set_num_threads(threads)
    return out


def large_run(R, torch, W):
    """Wall time of setup + local factorisations + solve on the large
    configurations: the 4.2M-point lattices at h/sigma 0.6, 0.8 and 1.0 (FP64
    and mixed to 1e-12) and the 50M-point lattice (mixed to 1e-12, then FP64 to
    1e-14), each through the device entry points on one stream."""
    stream = torch.cuda.current_stream()
    out = {}

    def run(w, prec, rtol):
        pts = w.points()
        d_pts = torch.tensor(pts, device="cuda")
        d_f = torch.tensor(w.values(pts), device="cuda")
        del pts
        d_lam = torch.empty(w.n, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
        try:
            R.rbf_precond_setup(h, prec, stream)
            info, st = R.rbf_solve_device(h, d_lam, R.default_opts(rtol=rtol, precision=prec,
                                                                  stream=stream, max_iters=300),
                                          ok=(R.RBF_OK, R.RBF_ENOCONV))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            R.rbf_destroy(h)
        d = info.as_dict()
        del d_pts, d_f, d_lam
        return {"n": w.n, "s_to_tol": dt, "rtol": rtol, "status": R.status_name(st),
                "iterations": d["iterations"], "outer": d["outer_iterations"],
                "rel_residual": d["rel_residual"], "t_pcsetup": d["t_pcsetup"]}

    for name in ("c2_0.6", "c2_0.8", "c2_1.0"):
        w = W.WORKLOADS[name]
        tags = [("fp64", R.RBF_FP64), ("mixed", R.RBF_MIXED)]
        if name == "c2_0.8":
            tags.append(("fp64_pc32", R.RBF_FP64_PC32))
        for tag, prec in tags:
            out[f"{name}_{tag}"] = run(w, prec, 1e-12)
            log("large", name, tag, out[f"{name}_{tag}"])
    w = W.WORKLOADS["c4"]
    for tag, prec, rtol in (("mixed", R.RBF_MIXED, 1e-12), ("fp64_pc32", R.RBF_FP64_PC32, 1e-14),
                            ("fp64", R.RBF_FP64, 1e-14)):
        out[f"c4_{tag}"] = run(w, prec, rtol)
        log("large", "c4", tag, out[f"c4_{tag}"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-side", type=int, default=0,
                    help="oracle lattice side (0: the workload itself)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 4.2M-point and 50M-point legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-geometry", action="store_true")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--sweep-geometry", action="store_true",
                    help="also time B in {3..7} sigma x D/B in {1.5..2.3} (Figs. 6 and 7)")
    ap.add_argument("--sweep-ratios", type=str, default="",
                    help="h/sigma values of the sweep, comma-separated (default: the workload's)")
    ap.add_argument("--sweep-box-truncation", action="store_true",
                    help="run the sweep with the paper's box truncation instead of the radial cutoff")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream to run (the configuration's 512)")
    ap.add_argument("--serve-active", type=int, default=8)
    ap.add_argument("--serve-max-iters", type=int, default=300)
    ap.add_argument("--serve-stall-cycles", type=int, default=0,
                    help="FP64 requests end once the residual has not halved in this many "
                         "GMRES cycles (0: off; otherwise the FP64 stream also runs without it)")
    ap.add_argument("--serve-engines", type=int, default=2,
                    help="packed engines of the server (0: one stream per request)")
    ap.add_argument("--serve-n-hi", type=float, default=1e6,
                    help="largest request size of the stream (the configuration's 1e6)")
    ap.add_argument("--serve-compare", type=str, default="",
                    help="comma-separated further engine counts to serve the stream with")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a run", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0909_5413_amd as R
    from paper_0909_5413_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    w = W.WORKLOADS[args.workload]
    log("workload", w.name, "N", w.n)
    pts = w.points()
    f = w.values(pts)
    dev = torch.device("cuda:0")
    d_pts = torch.tensor(pts, device=dev)
    d_f = torch.tensor(f, device=dev)
    d_lam = torch.empty(w.n, device=dev, dtype=torch.float64)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    # interactions per matvec: a property of the point set (counted once)
    h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
    _, inter = R.rbf_neighbor_counts(h, w.n)
    _, (ncx, ncy) = R.rbf_grid(h)
    _, _, cs = R.rbf_binning(h, w.n)
    R.rbf_destroy(h)
    n_omega, n_c = block_sizes(cs, ncx, ncy, w.overlap)
    log("interactions/matvec", inter, "cells", ncx * ncy)

    opts = R.default_opts(rtol=w.rtol, stream=stream)

    def step():
        h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
        try:
            R.rbf_precond_setup(h, R.RBF_FP64, stream)
            info, _ = R.rbf_solve_device(h, d_lam, opts)
        finally:
            R.rbf_destroy(h)
        return info.as_dict()

    for i in range(args.warmup):
        info = step()
        log("warmup", i, "iterations", info["iterations"], "rel", info["rel_residual"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(step())
        log("step", i, "done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mv = sum(i["matvecs64"] for i in infos)
    value = inter * mv / dt
    ms_step = 1e3 * dt / args.steps
    last = infos[-1]
    log("ms/step", ms_step, "value", value)

    # ---- per-kernel rooflines: HIP events on the stream the library uses -------
    h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
    kernels = {}
    try:
        t_pc = event_time(torch, stream, lambda: R.rbf_precond_setup(h, R.RBF_FP64, stream), 1)
        own = n_c > 0
        no, nc = n_omega[own].astype(np.float64), n_c[own].astype(np.float64)
        flops = float(np.sum(no ** 3 / 3.0 + nc * no ** 2))
        kernels["precond_setup64"] = {
            "bound": "alu", "achieved": flops / (t_pc * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "ms": t_pc, "flops_per_launch": flops}
        # the matvec microbenchmark: w ~ U(-1, 1) from seed 5413 + 11, five
        # warm-up launches, the median of 50 launches each timed by its own
        # event pair
        wv = torch.tensor(W.random_weights(w.n, W.SEED_BASE + 11), device=dev)
        yv = torch.empty_like(wv)
        t_mv = event_median(torch, stream, lambda: R.rbf_matvec_device(
            h, wv, yv, R.RBF_FP64, R.RBF_ORDER_SORTED, stream), 5, 50)
        t_mv_b2b = event_time(torch, stream, lambda: R.rbf_matvec_device(
            h, wv, yv, R.RBF_FP64, R.RBF_ORDER_SORTED, stream), args.kernel_reps)
        rate = inter / (t_mv * 1e-3)
        # in the solve the matvec launches sit between the RASM applies and the
        # Krylov kernels; back to back (above) the sustained FP64 load lowers the
        # clock, so both rates are reported
        ms_in_solve = 1e3 * last["t_matmult"] / max(1, last["matvecs64"])
        kernels["matvec64"] = {
            "bound": "alu", "achieved": rate * OPS_PER_INTERACTION / 1e12,
            "peak": VALU_OPS_PER_S / 1e12, "unit": "TFLOP/s", "ms": t_mv,
            "interactions_per_s": rate, "timing": "median of 50 event-timed launches after 5",
            "back_to_back_ms": t_mv_b2b,
            "back_to_back_interactions_per_s": inter / (t_mv_b2b * 1e-3),
            "r64_interactions_per_s": VALU_OPS_PER_S / OPS_PER_INTERACTION,
            "in_solve_ms": ms_in_solve,
            "in_solve_interactions_per_s": inter / (ms_in_solve * 1e-3),
            "in_solve_frac_r64": inter / (ms_in_solve * 1e-3) * OPS_PER_INTERACTION / VALU_OPS_PER_S}
        t_mv32 = event_median(torch, stream, lambda: R.rbf_matvec_device(
            h, wv, yv, R.RBF_MIXED, R.RBF_ORDER_SORTED, stream), 5, 50)
        kernels["matvec32"] = {"ms": t_mv32, "interactions_per_s": inter / (t_mv32 * 1e-3)}
        R.rbf_precond_apply_device(h, wv, yv, R.RBF_FP64, R.RBF_ORDER_SORTED, stream)
        t_ra = event_time(torch, stream, lambda: R.rbf_precond_apply_device(
            h, wv, yv, R.RBF_FP64, R.RBF_ORDER_SORTED, stream), args.kernel_reps)
        zbytes = float(np.sum(no * nc)) * 8.0
        bytes_ = zbytes + 16.0 * w.n
        kernels["rasm_apply64"] = {
            "bound": "hbm", "achieved": bytes_ / (t_ra * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "ms": t_ra, "bytes_per_launch": bytes_}
        # the same apply with the FP32 centre rows and FP64 sums (RBF_FP64_PC32)
        R.rbf_precond_apply_device(h, wv, yv, R.RBF_FP64_PC32, R.RBF_ORDER_SORTED, stream)
        t_rp = event_time(torch, stream, lambda: R.rbf_precond_apply_device(
            h, wv, yv, R.RBF_FP64_PC32, R.RBF_ORDER_SORTED, stream), args.kernel_reps)
        bytes32 = zbytes / 2 + 16.0 * w.n
        kernels["rasm_apply32x64"] = {
            "bound": "hbm", "achieved": bytes32 / (t_rp * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "ms": t_rp, "bytes_per_launch": bytes32}
    finally:
        R.rbf_destroy(h)
    # the setup's kernels one by one: HIP events the library records around
    # each of its launches (profiling on), one FP64 setup
    h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
    try:
        R.rbf_set_profiling(h, True)
        R.rbf_precond_setup(h, R.RBF_FP64, stream)
        setup_k = R.rbf_setup_kernel_times(h, R.RBF_FP64)
    finally:
        R.rbf_destroy(h)
    ms_cs, n_cs = setup_k["chol_step"]
    sflops = step_kernel_flops(no)
    kernels["chol_step64"] = {
        "bound": "mfma", "achieved": sflops / (ms_cs * 1e-3) / 1e12,
        "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "ms": ms_cs / n_cs,
        "launches": n_cs, "flops_per_launch": sflops / n_cs}
    for k in kernels.values():
        if "peak" in k:
            k["frac"] = k["achieved"] / k["peak"]
    # the dominant kernel: the single kernel with the largest share of the FP64
    # step (all launches of it in one step)
    share = {
        "chol_step64": ms_cs,
        "matvec64": kernels["matvec64"]["ms"] * last["matvecs64"],
        "rasm_apply64": kernels["rasm_apply64"]["ms"] * last["precond_applies"],
    }
    share.update({f"setup_{k}": v[0] for k, v in setup_k.items() if k != "chol_step"})
    dom = max((k for k in share if k in kernels and "peak" in kernels[k]), key=share.get)
    k = kernels[dom]
    traffic = profiled_traffic(dom)
    roofline = {"kernel": dom, "bound": k["bound"], "achieved": k["achieved"], "peak": k["peak"],
                "unit": k["unit"], "frac": k["frac"], "traffic": traffic,
                "step_share_ms": share}

    # ---- mixed precision: time to the same tolerance ---------------------------
    mixed = None
    if not args.no_mixed:
        mopts = R.default_opts(rtol=w.rtol, precision=R.RBF_MIXED, stream=stream)
        lam64 = d_lam.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
        try:
            R.rbf_precond_setup(h, R.RBF_MIXED, stream)
            minfo, mst = R.rbf_solve_device(h, d_lam, mopts, ok=(R.RBF_OK, R.RBF_ENOCONV))
            torch.cuda.synchronize()
            tm = time.perf_counter() - t1
            # the interpolant at the staggered lattice between the nodes, against
            # the closed-form data and the FP64 interpolant (evaluated below)
            tg = W.staggered_lattice(w.n_side)
            d_tg = torch.tensor(tg, device=dev)
            s_mx = torch.empty(tg.shape[0], device=dev, dtype=torch.float64)
            R.rbf_evaluate_device(h, d_tg, tg.shape[0], s_mx, stream)
        finally:
            R.rbf_destroy(h)
        werr = float(torch.linalg.norm(d_lam - lam64) / torch.linalg.norm(lam64))
        lam_mx_host = d_lam.cpu().numpy()
        lam_64_host = lam64.cpu().numpy()
        h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
        try:
            R.rbf_precond_setup(h, R.RBF_FP64, stream)
            R.rbf_solve_device(h, d_lam, opts)
            s_64 = torch.empty_like(s_mx)
            R.rbf_evaluate_device(h, d_tg, tg.shape[0], s_64, stream)
            t_ev = event_time(torch, stream, lambda: R.rbf_evaluate_device(
                h, d_tg, tg.shape[0], s_64, stream), 5)
        finally:
            R.rbf_destroy(h)
        fex = torch.tensor(W.gaussian_vortex(tg, w.r0), device=dev)
        fmax = float(fex.abs().max())
        mixed = {"s_to_tol": tm, "status": R.status_name(mst),
                 "iterations_inner": minfo.iterations, "outer": minfo.outer_iterations,
                 "shifted_blocks": minfo.shifted_blocks,
                 "rel_residual": minfo.rel_residual, "weight_rel_diff_vs_fp64": werr,
                 "interpolant_points": int(tg.shape[0]),
                 "interp_err_fp64": float((s_64 - fex).abs().max()) / fmax,
                 "interp_err_mixed": float((s_mx - fex).abs().max()) / fmax,
                 "interp_rel_diff_mixed_vs_fp64": float((s_mx - s_64).abs().max() / s_64.abs().max()),
                 "evaluate_ms": t_ev, "evaluations_per_s": tg.shape[0] / (t_ev * 1e-3)}
        log("mixed", mixed)
        s_mx_host, s_64_host = s_mx.cpu().numpy(), s_64.cpu().numpy()
        # the FP64 method with the FP32 local inverses as its preconditioner
        popts = R.default_opts(rtol=w.rtol, precision=R.RBF_FP64_PC32, stream=stream)
        pc32_t = []
        for rep in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap, stream)
            try:
                R.rbf_precond_setup(h, R.RBF_FP64_PC32, stream)
                pinfo, pst = R.rbf_solve_device(h, d_lam, popts, ok=(R.RBF_OK, R.RBF_ENOCONV))
                torch.cuda.synchronize()
                pc32_t.append(time.perf_counter() - t1)
                pinfo = pinfo.as_dict()
            finally:
                R.rbf_destroy(h)
        lam_pc_host = d_lam.cpu().numpy()
        mixed["fp64_pc32"] = {
            "s_to_tol": float(np.median(pc32_t)), "status": R.status_name(pst),
            "iterations": pinfo["iterations"], "rel_residual": pinfo["rel_residual"],
            "t_pcsetup": pinfo["t_pcsetup"], "t_matsolve": pinfo["t_matsolve"],
            "shifted_blocks": pinfo["shifted_blocks"],
            "weight_rel_diff_vs_fp64": float(np.linalg.norm(lam_pc_host - lam_64_host)
                                             / np.linalg.norm(lam_64_host))}
        log("fp64 with fp32 local inverses", mixed["fp64_pc32"])

    # ---- evaluation of the interpolant at separate targets (eq. rbf1; the
    # remeshing use): the staggered lattice between the nodes and seeded
    # uniform points over the nodes' box, in-cutoff interactions per second
    evaluation = None
    if not args.no_eval:
        evaluation = eval_run(R, torch, w, d_pts, d_f, d_lam, stream, opts)
        log("evaluation", evaluation)

    # ---- the paper's subdomain geometry: boxes of side B, overlapping squares of
    # side D (its measured optimum B = 5 sigma, D = 1.9 B) against the 3x3 cells
    geometry = None
    if not args.no_geometry:
        ratios = tuple(float(v) for v in args.sweep_ratios.split(",") if v)
        geometry = geometry_run(R, torch, w, d_pts, d_f, d_lam, stream, args.sweep_geometry,
                                ratios, args.sweep_box_truncation)
        geometry["cells_3x3_fp64"] = {
            "s_to_tol": ms_step / 1e3, "iterations": last["iterations"],
            "z_bytes": float(np.sum(n_omega[n_c > 0].astype(np.float64) * n_c[n_c > 0])) * 8.0}
        log("geometry", geometry)

    serving = None
    if not args.no_serve:
        serving = {}
        for tag, prec in (("fp64", R.RBF_FP64), ("mixed", R.RBF_MIXED),
                          ("fp64_pc32", R.RBF_FP64_PC32)):
            log("serving", tag, args.serve_requests, "requests")
            serving[tag] = serving_run(R, W, args.serve_requests, prec, args.serve_active,
                                       args.serve_max_iters, packed=args.serve_engines,
                                       n_hi=args.serve_n_hi,
                                       stall_cycles=args.serve_stall_cycles)
            log("serving", tag, serving[tag])
            if prec == R.RBF_FP64 and args.serve_stall_cycles:   # the same stream without it
                serving["fp64_no_stall_stop"] = serving_run(
                    R, W, args.serve_requests, prec, args.serve_active, args.serve_max_iters,
                    packed=args.serve_engines, n_hi=args.serve_n_hi)
                log("serving", "fp64_no_stall_stop", serving["fp64_no_stall_stop"])
            for e in (int(v) for v in args.serve_compare.split(",") if v.strip()):
                serving[f"{tag}_engines{e}"] = serving_run(R, W, args.serve_requests, prec,
                                                           args.serve_active, args.serve_max_iters,
                                                           packed=e, n_hi=args.serve_n_hi)
                log("serving", tag, e, "engines", serving[f"{tag}_engines{e}"])

    large = None
    if not args.no_large:
        large = large_run(R, torch, W)

    cpu = None
    oracle_cmp = None
    if not args.no_cpu:
        side = args.cpu_side or w.n_side
        log("cpu baseline: oracle on a", side, "lattice")
        tg_host = W.staggered_lattice(w.n_side) if mixed is not None else None
        cpu, lam_or, s_or = cpu_baseline(w, side, tg_host)
        log("cpu", cpu)
        cpu["matvec_1thread"] = oracle_matvec_1thread(["c0", w.name])
        log("cpu 1-thread matvec", cpu["matvec_1thread"])
        if lam_or is not None and mixed is not None:
            # the GPU's weights and interpolants against the oracle's: two
            # solutions that both meet the tolerance differ by up to
            # kappa(A) (res1 + res2) in the weights; the interpolants agree far
            # more closely
            nl = np.linalg.norm(lam_or)
            smax = np.abs(s_or).max()
            oracle_cmp = {
                "weights_rel_diff_fp64": float(np.linalg.norm(lam_64_host - lam_or) / nl),
                "weights_rel_diff_mixed": float(np.linalg.norm(lam_mx_host - lam_or) / nl),
                "weights_rel_diff_fp64_pc32": float(np.linalg.norm(lam_pc_host - lam_or) / nl),
                "interp_rel_diff_fp64": float(np.abs(s_64_host - s_or).max() / smax),
                "interp_rel_diff_mixed": float(np.abs(s_mx_host - s_or).max() / smax),
                "oracle_rel_residual": cpu["rel_residual"], "points": int(s_or.shape[0])}
            log("vs oracle", oracle_cmp)

    line = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{w.name}: N={w.n} jittered {w.n_side}x{w.n_side} lattice on "
                                f"[-1,1]^2, h/sigma={w.h_over_sigma}, cutoff 6 sigma, RASM 3x3 "
                                f"cells, GMRES(30) to {w.rtol:g}; step = binning + local "
                                "factorisations + solve"),
                   "n": w.n, "rtol": w.rtol, "interactions_per_matvec": inter},
        "s_to_tol_fp64": ms_step / 1e3,
        "fp64_solve": {k: last[k] for k in ("iterations", "restarts", "rel_residual",
                                            "t_init", "t_pcsetup", "t_matmult", "t_matsolve",
                                            "t_vecmdot", "t_other", "matvecs64",
                                            "precond_applies")},
        "mixed": mixed,
        "vs_oracle": oracle_cmp,
        "large": large,
        "p99_latency_s": serving["fp64"]["latency_p99_s"] if serving else None,
        "serving": serving,
        "geometry": geometry,
        "evaluation": evaluation,
        "roofline": roofline,
        "kernels": kernels,
        "setup_kernels_ms": {k: {"ms": v[0], "launches": v[1]} for k, v in setup_k.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
