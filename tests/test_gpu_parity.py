"""GPU library vs CPU oracle, through the C ABI (run with -m gpu on an MI355X).

Bars: bit-exact for binning and neighbour counts; componentwise
|y_gpu - y_oracle| <= 1e-13 (|A| |w|)_i for the FP64 matvec; solved weights
judged by the oracle's own FP64 residual; FP32 forms against bounds derived
from FP32 rounding.
"""
import sys

import numpy as np
import pytest

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
    R.lib()   # fails loudly if the HIP library is not built
    return torch


def ragged():
    # 45 x 31 points over a non-square box, h/sigma = 1.0, cutoff 9 sigma: about
    # 81 points per cell (two 64-column passes of the inverse rows), local blocks
    # of up to 729 points (three 256-row passes of the factorisation update),
    # partial border cells; local condition numbers ~3e3
    rng = np.random.default_rng(77)
    nx, ny = 45, 31
    h = 2 / nx
    xs = -1 + (np.arange(nx) + 0.5) * h
    ys = -0.6 + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(xs, ys)
    pts = np.stack([X.ravel(), Y.ravel()], 1) + rng.uniform(-0.1 * h, 0.1 * h, (nx * ny, 2))
    sigma = h / 1.0
    return "ragged", pts, sigma, 9 * sigma


def ill():
    # h/sigma = 0.6: local blocks with condition numbers ~1e15
    w = W.Workload("ill", 24, 0.6, seed=99)
    return "ill", w.points(), w.sigma, w.cutoff


def case(name):
    if name == "ragged":
        return ragged()
    if name == "ill":
        return ill()
    w = W.WORKLOADS[name]
    return name, w.points(), w.sigma, w.cutoff


CASES = ["mini", "c0", "ragged"]
ALL = CASES + ["ill"]


@pytest.fixture(scope="module")
def problems(torch_dev, oracle_mod):
    out = {}
    for name in ALL:
        nm, pts, sigma, cutoff = case(name)
        f = W.gaussian_vortex(pts)
        say("setup", nm, pts.shape[0])
        h = R.rbf_setup(pts, f, sigma, cutoff, 1)
        P = oracle_mod.Problem(pts, sigma, cutoff, 1)
        out[name] = (h, P, pts, f, sigma, cutoff)
    yield out
    for v in out.values():
        R.rbf_destroy(v[0])


@pytest.mark.parametrize("name", CASES)
def test_binning_bit_exact(problems, name):
    say("binning", name)
    h, P, pts, *_ = problems[name]
    g, (ncx, ncy) = R.rbf_grid(h)
    assert g[0] == P.x0 and g[1] == P.y0 and g[2] == P.L and g[3] == P.invL
    assert (ncx, ncy) == (P.ncx, P.ncy)
    cell_of, perm, cs = R.rbf_binning(h, pts.shape[0])
    o_cell, o_perm, o_cs = P.binning()
    assert np.array_equal(cell_of, o_cell)
    assert np.array_equal(perm, o_perm)
    assert np.array_equal(cs.astype(np.int64), o_cs)


@pytest.mark.parametrize("name", CASES)
def test_neighbour_counts_bit_exact(problems, name):
    say("nnb", name)
    h, P, pts, *_ = problems[name]
    nnb, tot = R.rbf_neighbor_counts(h, pts.shape[0])
    _, o_nnb = P.matvec(np.ones(pts.shape[0]), with_counts=True)
    assert np.array_equal(nnb, o_nnb)
    assert tot == int(o_nnb.sum())


def gpu_matvec(torch, h, w, precision=R.RBF_FP64):
    dw = torch.tensor(w, device="cuda", dtype=torch.float64)
    dy = torch.empty_like(dw)
    R.rbf_matvec_device(h, dw, dy, precision, R.RBF_ORDER_ORIGINAL,
                        torch.cuda.current_stream())
    torch.cuda.synchronize()
    return dy.cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_matvec64_parity(torch_dev, problems, name):
    say("matvec64", name)
    h, P, pts, *_ = problems[name]
    w = W.random_weights(pts.shape[0], 11)
    y = gpu_matvec(torch_dev, h, w)
    yo = P.matvec(w)
    scale = P.matvec(np.abs(w))          # (|A| |w|)_i, A is elementwise >= 0
    err = np.abs(y - yo) / scale
    assert err.max() <= 1e-13, err.max()


@pytest.mark.parametrize("name", CASES)
def test_matvec32_accuracy(torch_dev, problems, name):
    say("matvec32", name)
    h, P, pts, *_ = problems[name]
    w = W.random_weights(pts.shape[0], 12)
    y = gpu_matvec(torch_dev, h, w, R.RBF_MIXED)
    yo = P.matvec(w)
    scale = P.matvec(np.abs(w))
    # FP32 coordinates (cell-relative), FP32 exp2, compensated sum: a few 1e-6
    # of the absolute sum; pairs within FP32 rounding of the cutoff may flip,
    # each worth e^-18 of the peak
    err = np.abs(y - yo) / scale
    assert err.max() <= 2e-5, err.max()


@pytest.mark.parametrize("name", CASES)
def test_rasm_apply_parity(torch_dev, problems, name):
    say("rasm64", name)
    h, P, pts, *_ = problems[name]
    P.rasm_setup()
    v = W.random_weights(pts.shape[0], 13)
    dv = torch_dev.tensor(v, device="cuda", dtype=torch_dev.float64)
    dz = torch_dev.empty_like(dv)
    R.rbf_precond_apply_device(h, dv, dz, R.RBF_FP64, R.RBF_ORDER_ORIGINAL,
                               torch_dev.cuda.current_stream())
    torch_dev.cuda.synchronize()
    z = dz.cpu().numpy()
    zo = P.rasm_apply(v)
    # both sides solve the same ill-conditioned local systems: agreement is
    # limited by cond(A_c) * u, cond(A_c) ~ 1e6..1e8 at these h/sigma
    rel = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    assert rel <= 1e-7, rel


@pytest.mark.parametrize("name", ["ragged", "mini"])
def test_rasm_apply_elementwise(torch_dev, problems, name):
    """Element by element against the oracle's RASM (eq. rasm: forward and back
    substitution with the local Cholesky factor, centre rows kept).  Both sides
    solve the same local systems backward-stably, so each centre value z_i of
    cell c differs by at most about n_c kappa_c u (|A_c^-1| |v_c|)_i, with
    kappa_c the local condition number (about 3e3 on the ragged h/sigma = 1.0
    case, 1e6 at h/sigma = 0.8) and n_c the block size; the bar takes
    10 n_c kappa_c u with |A_c^-1| from numpy's inverse of each block."""
    say("rasm64 elementwise", name)
    h, P, pts, f, sigma, cutoff = problems[name]
    from tests import bruteforce as bf
    P.rasm_setup()
    v = W.random_weights(pts.shape[0], 17)
    dv = torch_dev.tensor(v, device="cuda", dtype=torch_dev.float64)
    dz = torch_dev.empty_like(dv)
    R.rbf_precond_apply_device(h, dv, dz, R.RBF_FP64, R.RBF_ORDER_ORIGINAL,
                               torch_dev.cuda.current_stream())
    torch_dev.cuda.synchronize()
    z = dz.cpu().numpy()
    zo = P.rasm_apply(v)
    u = np.finfo(float).eps / 2
    worst = 0.0
    for cell in range(P.ncells):
        mem, kc, _ = P.rasm_block(cell, with_factor=False)
        if kc == 0:
            continue
        A = bf.dense_matrix(pts[mem], sigma, None)
        inv = np.linalg.inv(A)
        ev = np.linalg.eigvalsh(A)
        kappa = ev[-1] / ev[0]
        own = mem[len(mem) - kc:]
        scale = (np.abs(inv) @ np.abs(v[mem]))[len(mem) - kc:]
        bar = 10 * len(mem) * kappa * u * scale
        err = np.abs(z[own] - zo[own])
        worst = max(worst, float((err / bar).max()))
        assert np.all(err <= bar), (cell, float((err / bar).max()), kappa)
    say("rasm64 elementwise worst error / bar", name, worst)


@pytest.mark.parametrize("name", ["mini", "ragged"])
def test_evaluate_off_nodes(problems, name):
    """The interpolant (eq. rbf1) at targets off the nodes: between nodes,
    scattered in the box, outside the nodes' bounding box (the target's cell
    is clamped to the border cells) and farther than the cutoff from every
    node (exactly zero), against the oracle's evaluation of the same weights,
    element by element within 1e-13 of sum_j |lam_j| phi(|t - x_j|)."""
    say("evaluate off nodes", name)
    h, P, pts, f, sigma, cutoff = problems[name]
    lam, info, st = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-10))
    tg, nfar = W.evaluation_targets(pts, cutoff)
    s = R.rbf_evaluate(h, tg)
    so = P.evaluate(lam, tg)
    scale = P.evaluate(np.abs(lam), tg)
    err = np.abs(s - so)
    assert np.all(err <= 1e-13 * scale), float(np.max(err / np.where(scale > 0, scale, 1)))
    assert np.all(s[-nfar:] == 0.0) and np.all(so[-nfar:] == 0.0)
    # the sources summed at each target, bit-exact (the staggered lattice too)
    import torch
    for t in (tg, W.staggered_lattice(int(round(np.sqrt(pts.shape[0]))))):
        d_t = torch.tensor(t, device="cuda", dtype=torch.float64)
        d_c = torch.empty(t.shape[0], device="cuda", dtype=torch.int32)
        R.rbf_target_counts_device(h, d_t, t.shape[0], d_c, torch.cuda.current_stream())
        torch.cuda.synchronize()
        _, oc = P.evaluate(lam, t, with_counts=True)
        assert np.array_equal(d_c.cpu().numpy(), oc)


@pytest.mark.parametrize("name", ["mini", "ragged", "ill"])
def test_centre_rows_are_inverse_rows(problems, name):
    """Z_c is a backward-stable set of rows of A_c^{-1}: with A_c rebuilt in numpy,
    ||Z_c A_c - E_C|| <= c n u ||Z_c|| ||A_c|| whatever cond(A_c) is (the
    ill-conditioned case has cond ~1e15, where no two factorisations agree
    elementwise)."""
    say("zrows", name)
    h, P, pts, f, sigma, cutoff = problems[name]
    _, (ncx, ncy) = R.rbf_grid(h)
    from tests import bruteforce as bf
    u = np.finfo(float).eps / 2
    for cell in (0, ncx + 1, (ncx * ncy) // 2, ncx * ncy - 1):
        mem, Z = R.rbf_precond_block(h, cell, R.RBF_FP64)
        o_mem, kc, _ = P.rasm_block(cell, with_factor=False)
        assert np.array_equal(mem, o_mem)
        if Z.shape[0] == 0:
            continue
        A = bf.dense_matrix(pts[mem], sigma, None)
        n = len(mem)
        E = np.eye(n)[n - kc:]
        res = np.linalg.norm(Z @ A - E, 2)
        bound = 10 * n * u * np.linalg.norm(Z, 2) * np.linalg.norm(A, 2)
        assert res <= bound, (cell, res, bound)


@pytest.mark.parametrize("name", ["mini", "ragged"])
def test_centre_rows_fp32_backward_error(problems, name):
    """FP32 Z_c (mixed form): backward error at FP32 level.  A block may carry
    a diagonal shift mu <= 1000 n u32 phi(0) (shifted Cholesky), so
    ||Z_c A_c - E_C|| <= (10 n u32 ||A_c|| + mu_max) ||Z_c||."""
    say("zrows32", name)
    h, P, pts, f, sigma, cutoff = problems[name]
    _, (ncx, ncy) = R.rbf_grid(h)
    from tests import bruteforce as bf
    u32 = 2.0 ** -24
    phi0 = 1.0 / (2 * np.pi * sigma * sigma)
    for cell in (0, ncx + 1, (ncx * ncy) // 2, ncx * ncy - 1):
        mem, Z = R.rbf_precond_block(h, cell, R.RBF_MIXED)
        o_mem, kc, _ = P.rasm_block(cell, with_factor=False)
        assert np.array_equal(mem, o_mem)
        if Z.shape[0] == 0:
            continue
        Z = Z.astype(np.float64)
        A = bf.dense_matrix(pts[mem], sigma, None)
        n = len(mem)
        E = np.eye(n)[n - kc:]
        res = np.linalg.norm(Z @ A - E, 2)
        bound = (10 * n * u32 * np.linalg.norm(A, 2) + 1000 * n * u32 * phi0) * np.linalg.norm(Z, 2)
        assert res <= bound, (cell, res, bound)


@pytest.mark.parametrize("name,rtol", [("mini", 1e-12), ("c0", 1e-10), ("ragged", 1e-12)])
def test_solve_fp64(problems, name, rtol):
    say("solve64", name)
    h, P, pts, f, *_ = problems[name]
    o = R.default_opts(rtol=rtol)
    lam, info, st = R.rbf_solve(h, pts.shape[0], o)
    res = P.rel_residual(f, lam)
    assert info.rel_residual <= rtol
    assert res <= residual_gate(P, f, lam, rtol), (res, info.as_dict())
    _, oinfo = P.gmres(f, 30, rtol)
    assert abs(info.iterations - oinfo.iterations) <= 2, (info.iterations, oinfo.iterations)
    # evaluate at the nodes reproduces the data, and matches the oracle
    s = R.rbf_evaluate(h, pts)
    assert np.linalg.norm(s - f) <= 1.1 * rtol * np.linalg.norm(f)
    stag = pts[:50] + 0.3 * (pts[1] - pts[0])
    so = P.evaluate(lam, stag)
    assert np.all(np.abs(R.rbf_evaluate(h, stag) - so) <= 1e-13 * (np.abs(so).max() + 1))


@pytest.mark.parametrize("name", ["ragged", "mini"])
def test_rasm_apply_fp32_rows_fp64_sums(torch_dev, problems, name):
    """RBF_FP64_PC32's apply: the FP32 centre rows (as rbf_precond_block
    returns them, widened exactly to FP64) times the FP64 member values, summed
    in FP64: element by element against the same product formed on the host,
    within the rounding of two n_omega-term FP64 sums."""
    say("rasm fp32 rows, fp64 sums", name)
    h, P, pts, *_ = problems[name]
    v = W.random_weights(pts.shape[0], 23)
    dv = torch_dev.tensor(v, device="cuda", dtype=torch_dev.float64)
    dz = torch_dev.empty_like(dv)
    R.rbf_precond_apply_device(h, dv, dz, R.RBF_FP64_PC32, R.RBF_ORDER_ORIGINAL,
                               torch_dev.cuda.current_stream())
    torch_dev.cuda.synchronize()
    z = dz.cpu().numpy()
    u = np.finfo(float).eps / 2
    ncells = R.rbf_grid(h)[1][0] * R.rbf_grid(h)[1][1]
    worst = 0.0
    for cell in range(ncells):
        mem, Z = R.rbf_precond_block(h, cell, R.RBF_FP64_PC32)
        if Z.shape[0] == 0:
            continue
        own = mem[len(mem) - Z.shape[0]:]
        assert np.array_equal(Z, Z.astype(np.float32).astype(np.float64))
        ref = Z @ v[mem]
        bar = 2 * len(mem) * u * (np.abs(Z) @ np.abs(v[mem])) + 1e-300
        err = np.abs(z[own] - ref)
        worst = max(worst, float((err / bar).max()))
        assert np.all(err <= bar), (cell, float((err / bar).max()))
    say("worst error / bar", worst)


@pytest.mark.parametrize("name,rtol", [("mini", 1e-12), ("c0", 1e-10), ("ragged", 1e-12)])
def test_solve_fp64_with_fp32_local_inverses(problems, name, rtol):
    """RBF_FP64_PC32: the FP64 method with the FP32 local inverses as its
    (fixed, linear) preconditioner reaches the same FP64 residual bar as the
    FP64 method, judged by the oracle, in about as many iterations."""
    say("solve fp64 pc32", name)
    h, P, pts, f, *_ = problems[name]
    lam, info, st = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=rtol, precision=R.RBF_FP64_PC32))
    d = info.as_dict()
    assert d["rel_residual"] <= rtol and d["outer_iterations"] == 0
    assert d["matvecs32"] == 0 and d["matvecs64"] > 0
    res = P.rel_residual(f, lam)
    assert res <= residual_gate(P, f, lam, rtol), (res, d)
    _, i64, _ = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=rtol))
    say("iterations pc32", d["iterations"], "fp64", i64.iterations)
    assert abs(d["iterations"] - i64.iterations) <= max(2, i64.iterations // 5)


@pytest.mark.parametrize("name", ["mini", "c0"])
def test_solve_mixed(problems, name):
    say("solve_mixed", name)
    h, P, pts, f, sigma, cutoff = problems[name]
    o = R.default_opts(rtol=1e-12, precision=R.RBF_MIXED)
    lam, info, st = R.rbf_solve(h, pts.shape[0], o)
    res = P.rel_residual(f, lam)
    assert info.rel_residual <= 1e-12
    assert res <= residual_gate(P, f, lam, 1e-12), (res, info.as_dict())
    xo, oinfo = P.gmres(f, 30, 1e-12)
    werr = np.linalg.norm(lam - xo) / np.linalg.norm(xo)
    # two weight vectors that both meet the residual test agree only to the
    # conditioning of A: ||lam - xo|| <= ||A^-1|| ||A (lam - xo)|| and
    # ||A (lam - xo)|| <= (res + res_oracle) ||f||, with ||xo|| >= ||f|| / ||A||
    stag = W.staggered_lattice(int(round(np.sqrt(pts.shape[0]))))
    s_mixed = R.rbf_evaluate(h, stag)
    s_or = P.evaluate(xo, stag)
    ierr = np.abs(s_mixed - s_or).max() / np.abs(f).max()
    say("mixed vs oracle", name, "weights", werr, "interpolant", ierr,
        "outer", info.outer_iterations)
    if name == "mini":
        from tests import bruteforce as bf
        ev = np.linalg.eigvalsh(bf.dense_matrix(pts, sigma, cutoff))
        kappa = ev[-1] / ev[0]
        bound = kappa * (res + oinfo.rel_residual)
        say("mixed weight error bound kappa (res + res_oracle)", kappa, bound)
        assert werr <= bound, (werr, bound)
    # the interpolants differ by A(lam - xo) at the nodes and its smooth
    # continuation between them: far below the interpolation error itself
    assert ierr <= 1e-8, ierr


def test_mixed_shifted_blocks(problems):
    """The FP32 factorisation of the h/sigma = 0.6 blocks (condition numbers
    ~1e15, far beyond FP32) needs diagonal shifts on some blocks; the FP64 one
    never shifts; the mixed solve still meets its FP64 residual."""
    say("shifted blocks")
    h, P, pts, f, *_ = problems["ill"]
    _, i64, _ = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-10),
                            ok=(R.RBF_OK, R.RBF_ENOCONV))
    lam, i32, st = R.rbf_solve(h, pts.shape[0],
                               R.default_opts(rtol=1e-10, precision=R.RBF_MIXED, max_iters=600),
                               ok=(R.RBF_OK, R.RBF_ENOCONV))
    say("shifted blocks", i32.shifted_blocks, "of", P.ncells, R.status_name(st))
    assert i64.shifted_blocks == 0
    assert i32.shifted_blocks > 0


def test_determinism(torch_dev, problems):
    say("determinism")
    h, P, pts, f, *_ = problems["c0"]
    w = W.random_weights(pts.shape[0], 21)
    assert np.array_equal(gpu_matvec(torch_dev, h, w), gpu_matvec(torch_dev, h, w))
    o = R.default_opts(rtol=1e-10)
    a, _, _ = R.rbf_solve(h, pts.shape[0], o)
    b, _, _ = R.rbf_solve(h, pts.shape[0], o)
    assert np.array_equal(a, b)


def test_order_invariance(problems):
    say("order invariance")
    _, P, pts, f, sigma, cutoff = problems["mini"]
    rng = np.random.default_rng(5)
    p = rng.permutation(pts.shape[0])
    h2 = R.rbf_setup(pts[p], f[p], sigma, cutoff, 1)
    try:
        lam2, _, _ = R.rbf_solve(h2, pts.shape[0], R.default_opts(rtol=1e-12))
    finally:
        R.rbf_destroy(h2)
    lam = np.empty_like(lam2)
    lam[p] = lam2
    assert P.rel_residual(f, lam) <= residual_gate(P, f, lam, 1e-12)


def test_error_codes(torch_dev):
    say("errors")
    w = W.Workload("t", 20, 0.8)
    pts = w.points()
    f = w.values(pts)
    bad = pts.copy()
    bad[4] = bad[11]
    with pytest.raises(R.RbfError) as e:
        R.rbf_setup(bad, f, w.sigma, w.cutoff)
    assert e.value.status == R.RBF_EDUPLICATE
    bad = pts.copy()
    bad[2, 0] = np.inf
    with pytest.raises(R.RbfError) as e:
        R.rbf_setup(bad, f, w.sigma, w.cutoff)
    assert e.value.status == R.RBF_EINVAL
    with pytest.raises(R.RbfError) as e:
        R.rbf_setup(pts, f, -1.0, w.cutoff)
    assert e.value.status == R.RBF_EINVAL
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff)
    try:
        with pytest.raises(R.RbfError) as e:
            R.rbf_evaluate(h, pts[:3])
        assert e.value.status == R.RBF_ESTATE
        lam, info, st = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-30, max_iters=5),
                                    ok=(R.RBF_ENOCONV,))
        assert st == R.RBF_ENOCONV and info.iterations == 5
        with pytest.raises(R.RbfError) as e:
            R.rbf_solve(h, w.n, R.default_opts(max_device_bytes=1024))
        assert e.value.status == R.RBF_ENOMEM
    finally:
        R.rbf_destroy(h)


def test_setup_kernel_times(problems):
    """Event timing of the setup kernels: one assembly per batch, one step and
    one diagonal launch per 64-column block column below the first, one
    forward and one back solve per batch; all times positive."""
    say("setup kernel times")
    _, P, pts, f, sigma, cutoff = problems["c0"]
    h = R.rbf_setup(pts, f, sigma, cutoff, 1)
    try:
        with pytest.raises(R.RbfError) as e:
            R.rbf_setup_kernel_times(h, R.RBF_FP64)
        assert e.value.status == R.RBF_ESTATE
        R.rbf_set_profiling(h, True)
        R.rbf_precond_setup(h, R.RBF_FP64)
        kt = R.rbf_setup_kernel_times(h, R.RBF_FP64)
    finally:
        R.rbf_destroy(h)
    ms = {k: v[0] for k, v in kt.items()}
    n = {k: v[1] for k, v in kt.items()}
    assert n["assemble"] >= 1 and n["forward"] == n["assemble"]
    assert n["chol_step"] == n["chol_diag"] and n["chol_step"] % n["assemble"] == 0
    assert n["back"] == n["assemble"]
    assert all(v > 0 for v in ms.values()), ms
