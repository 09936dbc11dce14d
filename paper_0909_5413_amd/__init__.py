"""Python binding of librbf_hip.so (include/rbf.h): argument marshalling only.

Every step of the method runs in the library's gfx950 kernels; this module
only converts arguments.  Importing it does not load the library; the first
call does, and fails loudly (RbfLibraryMissing) if it has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import importlib.util
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbf_hip.so")

RBF_OK, RBF_EINVAL, RBF_EDUPLICATE, RBF_ENOMEM, RBF_EDEVICE = 0, 1, 2, 3, 4
RBF_ENOTPD, RBF_ENOCONV, RBF_EBREAKDOWN, RBF_ENAN, RBF_ESTATE, RBF_ELIMIT = 5, 6, 7, 8, 9, 10
RBF_FP64, RBF_MIXED, RBF_FP64_PC32 = 0, 1, 2
RBF_ORDER_ORIGINAL, RBF_ORDER_SORTED = 0, 1
RBF_MAX_BLOCK = 1536
RBF_MAX_CELL_POINTS = 1536
RBF_NOALLOC_MAX_POINTS = 4194304

EXPORTED = [
    "rbf_default_opts", "rbf_setup", "rbf_setup_device", "rbf_set_values",
    "rbf_precond_setup", "rbf_solve", "rbf_solve_device", "rbf_evaluate",
    "rbf_evaluate_device", "rbf_evaluate_lattice", "rbf_evaluate_lattice_device",
    "rbf_target_counts_device", "rbf_destroy", "rbf_block_cache", "rbf_grid", "rbf_binning",
    "rbf_neighbor_counts", "rbf_matvec_device", "rbf_matvec_device_noalloc",
    "rbf_precond_apply_device",
    "rbf_precond_block", "rbf_set_geometry", "rbf_set_profiling", "rbf_set_graphs", "rbf_setup_kernel_times",
    "rbf_server_default_opts", "rbf_server_create", "rbf_server_submit", "rbf_server_wait",
    "rbf_server_stats", "rbf_server_destroy", "rbf_status_string", "rbf_last_error",
]
RBF_K_ASSEMBLE, RBF_K_CHOL_STEP, RBF_K_CHOL_DIAG, RBF_K_FORWARD, RBF_K_BACK = range(5)
RBF_K_SETUP_KINDS = 5
SETUP_KERNELS = ["assemble", "chol_step", "chol_diag", "forward", "back"]


class RbfLibraryMissing(RuntimeError):
    pass


class RbfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status_name(status)}: {detail}")
        self.status = status


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iters", C.c_int), ("rtol", C.c_double),
                ("precision", C.c_int), ("inner_rtol", C.c_double), ("max_outer", C.c_int),
                ("max_device_bytes", C.c_size_t), ("stream", C.c_void_p),
                ("stall_cycles", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer_iterations", C.c_int), ("restarts", C.c_int),
                ("rel_residual", C.c_double), ("t_init", C.c_double),
                ("t_pcsetup", C.c_double), ("t_matmult", C.c_double),
                ("t_matsolve", C.c_double), ("t_vecmdot", C.c_double), ("t_other", C.c_double),
                ("interactions_per_matvec", C.c_longlong), ("matvecs64", C.c_int),
                ("matvecs32", C.c_int), ("precond_applies", C.c_int),
                ("device_bytes", C.c_size_t),
                ("history_len", C.c_int), ("history", C.POINTER(C.c_double)),
                ("shifted_blocks", C.c_int)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history"}
        d["history"] = [self.history[i] for i in range(self.history_len)] if self.history else []
        return d


_lib = None


class Geometry(C.Structure):
    _fields_ = [("box", C.c_double), ("overlap", C.c_double), ("truncation", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("max_active", C.c_int), ("max_device_bytes", C.c_size_t), ("packed", C.c_int),
                ("graphs", C.c_int), ("pack_max_points", C.c_longlong)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int), ("info", SolveInfo), ("t_queue", C.c_double),
                ("t_run", C.c_double), ("latency", C.c_double),
                ("predicted_bytes", C.c_size_t), ("message", C.c_char * 256)]


def lib():
    """The loaded C library (raises RbfLibraryMissing if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RbfLibraryMissing(
            f"{LIB_PATH} not found: build it with `python -m paper_0909_5413_amd.build` "
            "(there is no CPU fallback)")
    # PyTorch ships its own HIP runtime under the same soname as the system's,
    # and whichever loads first serves the whole process.  If this library
    # brought in the system runtime and PyTorch then initialised its device,
    # the library's later HIP calls would find no device; loading PyTorch
    # first (when it is installed) gives one runtime in either import order.
    if importlib.util.find_spec("torch") is not None:
        import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, dp, ip, lp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_longlong)
    pp = C.POINTER(C.c_void_p)
    sig = {
        "rbf_default_opts": (None, [C.POINTER(SolveOpts)]),
        "rbf_setup": (C.c_int, [vp, vp, C.c_longlong, C.c_double, C.c_double, C.c_int, pp]),
        "rbf_setup_device": (C.c_int, [vp, vp, C.c_longlong, C.c_double, C.c_double, C.c_int,
                                       vp, pp]),
        "rbf_set_values": (C.c_int, [vp, vp, C.c_int, vp]),
        "rbf_precond_setup": (C.c_int, [vp, C.c_int, vp]),
        "rbf_solve": (C.c_int, [vp, C.POINTER(SolveOpts), vp, vp, C.POINTER(SolveInfo)]),
        "rbf_solve_device": (C.c_int, [vp, C.POINTER(SolveOpts), vp, vp, C.POINTER(SolveInfo)]),
        "rbf_evaluate": (C.c_int, [vp, vp, C.c_longlong, vp]),
        "rbf_evaluate_device": (C.c_int, [vp, vp, C.c_longlong, vp, vp]),
        "rbf_evaluate_lattice": (C.c_int, [vp, C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_longlong, C.c_longlong, vp]),
        "rbf_evaluate_lattice_device": (C.c_int, [vp, C.c_double, C.c_double, C.c_double,
                                                  C.c_double, C.c_longlong, C.c_longlong, vp,
                                                  vp]),
        "rbf_target_counts_device": (C.c_int, [vp, vp, C.c_longlong, vp, vp]),
        "rbf_destroy": (None, [vp]),
        "rbf_block_cache": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
        "rbf_grid": (C.c_int, [vp, dp, lp]),
        "rbf_binning": (C.c_int, [vp, vp, vp, vp]),
        "rbf_neighbor_counts": (C.c_int, [vp, vp, lp]),
        "rbf_matvec_device": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, vp]),
        "rbf_matvec_device_noalloc": (C.c_int, [vp, vp, vp, C.c_int, vp]),
        "rbf_precond_apply_device": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, vp]),
        "rbf_precond_block": (C.c_int, [vp, C.c_longlong, C.c_int, vp, vp, ip, ip]),
        "rbf_set_geometry": (C.c_int, [vp, C.POINTER(Geometry), vp]),
        "rbf_set_profiling": (C.c_int, [vp, C.c_int]),
        "rbf_set_graphs": (C.c_int, [vp, C.c_int]),
        "rbf_server_default_opts": (None, [C.POINTER(ServerOpts)]),
        "rbf_server_create": (C.c_int, [C.POINTER(ServerOpts), pp]),
        "rbf_server_submit": (C.c_int, [vp, vp, vp, C.c_longlong, C.c_double, C.c_double, C.c_int,
                                        C.POINTER(SolveOpts), lp]),
        "rbf_server_wait": (C.c_int, [vp, C.c_longlong, vp, C.POINTER(RequestResult)]),
        "rbf_server_stats": (C.c_int, [vp, lp, lp, ip, ip, C.POINTER(C.c_size_t)]),
        "rbf_server_destroy": (None, [vp]),
        "rbf_setup_kernel_times": (C.c_int, [vp, C.c_int, dp, ip]),
        "rbf_status_string": (C.c_char_p, [C.c_int]),
        "rbf_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_name(s: int) -> str:
    try:
        return lib().rbf_status_string(s).decode()
    except RbfLibraryMissing:
        return str(s)


def last_error() -> str:
    return lib().rbf_last_error().decode()


def _check(status: int, where: str, ok=(RBF_OK,)):
    if status not in ok:
        raise RbfError(status, where, last_error())
    return status


def _host(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a) -> int | None:
    """Data pointer of a numpy array or a torch tensor (device or host)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().rbf_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "stream":
            v = _stream(v)
        setattr(o, k, v)
    return o


# ---- the C ABI, one Python function per entry point --------------------------

def rbf_setup(points, values, sigma: float, cutoff: float, overlap: int = 1) -> int:
    pts = _host(points).reshape(-1, 2)
    vals = _host(values) if values is not None else None
    h = C.c_void_p()
    _check(lib().rbf_setup(_ptr(pts), _ptr(vals), pts.shape[0], sigma, cutoff, overlap,
                           C.byref(h)), "rbf_setup")
    return h.value


def rbf_setup_device(d_points, d_values, n: int, sigma: float, cutoff: float, overlap: int = 1,
                     stream=None) -> int:
    h = C.c_void_p()
    _check(lib().rbf_setup_device(_ptr(d_points), _ptr(d_values), n, sigma, cutoff, overlap,
                                  _stream(stream), C.byref(h)), "rbf_setup_device")
    return h.value


def rbf_set_values(h: int, values, on_device: bool = False, stream=None):
    v = values if on_device else _host(values)
    _check(lib().rbf_set_values(h, _ptr(v), int(on_device), _stream(stream)), "rbf_set_values")


def rbf_precond_setup(h: int, precision: int = RBF_FP64, stream=None):
    _check(lib().rbf_precond_setup(h, precision, _stream(stream)), "rbf_precond_setup")


def rbf_solve(h: int, n: int, opts: SolveOpts | None = None, lambda0=None,
              ok=(RBF_OK,)):
    out = np.empty(n)
    info = SolveInfo()
    l0 = _host(lambda0) if lambda0 is not None else None
    st = lib().rbf_solve(h, C.byref(opts) if opts is not None else None, _ptr(l0), _ptr(out),
                         C.byref(info))
    _check(st, "rbf_solve", ok)
    return out, info, st


def rbf_solve_device(h: int, d_lambda_out, opts: SolveOpts | None = None, d_lambda0=None,
                     ok=(RBF_OK,)):
    info = SolveInfo()
    st = lib().rbf_solve_device(h, C.byref(opts) if opts is not None else None,
                                _ptr(d_lambda0), _ptr(d_lambda_out), C.byref(info))
    _check(st, "rbf_solve_device", ok)
    return info, st


def rbf_evaluate(h: int, targets) -> np.ndarray:
    t = _host(targets).reshape(-1, 2)
    out = np.empty(t.shape[0])
    _check(lib().rbf_evaluate(h, _ptr(t), t.shape[0], _ptr(out)), "rbf_evaluate")
    return out


def rbf_evaluate_device(h: int, d_targets, m: int, d_out, stream=None):
    _check(lib().rbf_evaluate_device(h, _ptr(d_targets), m, _ptr(d_out), _stream(stream)),
           "rbf_evaluate_device")


def rbf_evaluate_lattice(h: int, x0: float, y0: float, hx: float, hy: float, nx: int,
                         ny: int) -> np.ndarray:
    """The interpolant at (x0 + a hx, y0 + b hy), a < nx, b < ny, as an
    (ny, nx) array (row b, column a)."""
    out = np.empty((max(ny, 0), max(nx, 0)))
    _check(lib().rbf_evaluate_lattice(h, x0, y0, hx, hy, nx, ny, _ptr(out)),
           "rbf_evaluate_lattice")
    return out


def rbf_evaluate_lattice_device(h: int, x0: float, y0: float, hx: float, hy: float, nx: int,
                                ny: int, d_out, stream=None):
    _check(lib().rbf_evaluate_lattice_device(h, x0, y0, hx, hy, nx, ny, _ptr(d_out),
                                             _stream(stream)), "rbf_evaluate_lattice_device")


def rbf_target_counts_device(h: int, d_targets, m: int, d_counts, stream=None):
    _check(lib().rbf_target_counts_device(h, _ptr(d_targets), m, _ptr(d_counts), _stream(stream)),
           "rbf_target_counts_device")


def rbf_destroy(h: int):
    if h:
        lib().rbf_destroy(h)


def rbf_block_cache(device: int = -1, trim: bool = False) -> int:
    """Idle bytes held by the library's device block cache (before trimming);
    trim=True returns them to the runtime."""
    b = C.c_size_t()
    _check(lib().rbf_block_cache(device, 1 if trim else 0, C.byref(b)), "rbf_block_cache")
    return b.value


def rbf_grid(h: int):
    g = (C.c_double * 4)()
    nc = (C.c_longlong * 2)()
    _check(lib().rbf_grid(h, g, nc), "rbf_grid")
    return tuple(g), (int(nc[0]), int(nc[1]))


def rbf_binning(h: int, n: int):
    _, (ncx, ncy) = rbf_grid(h)
    cell_of = np.empty(n, np.int32)
    perm = np.empty(n, np.int32)
    cs = np.empty(ncx * ncy + 1, np.int32)
    _check(lib().rbf_binning(h, _ptr(cell_of), _ptr(perm), _ptr(cs)), "rbf_binning")
    return cell_of, perm, cs


def rbf_neighbor_counts(h: int, n: int):
    nnb = np.empty(n, np.int32)
    tot = C.c_longlong()
    _check(lib().rbf_neighbor_counts(h, _ptr(nnb), C.byref(tot)), "rbf_neighbor_counts")
    return nnb, tot.value


def rbf_matvec_device(h: int, d_w, d_y, precision: int = RBF_FP64,
                      order: int = RBF_ORDER_ORIGINAL, stream=None):
    _check(lib().rbf_matvec_device(h, _ptr(d_w), _ptr(d_y), precision, order, _stream(stream)),
           "rbf_matvec_device")


def rbf_matvec_device_noalloc(h: int, d_w, d_y, precision: int = RBF_FP64, stream=None):
    _check(lib().rbf_matvec_device_noalloc(h, _ptr(d_w), _ptr(d_y), precision, _stream(stream)),
           "rbf_matvec_device_noalloc")


def rbf_precond_apply_device(h: int, d_v, d_z, precision: int = RBF_FP64,
                             order: int = RBF_ORDER_ORIGINAL, stream=None):
    _check(lib().rbf_precond_apply_device(h, _ptr(d_v), _ptr(d_z), precision, order,
                                          _stream(stream)), "rbf_precond_apply_device")


def rbf_set_geometry(h: int, box: float, overlap: float, truncation: float = 0.0, stream=None):
    """Subdomain boxes of side `box` with overlapping squares of side `overlap`;
    a `truncation` side T > 0 truncates the product by the square of side T
    around each point's box instead of the radial cutoff."""
    g = Geometry(float(box), float(overlap), float(truncation))
    _check(lib().rbf_set_geometry(h, C.byref(g), _stream(stream)), "rbf_set_geometry")


def rbf_set_profiling(h: int, enable: bool = True):
    _check(lib().rbf_set_profiling(h, 1 if enable else 0), "rbf_set_profiling")


def rbf_set_graphs(h: int, enable: bool = True):
    _check(lib().rbf_set_graphs(h, 1 if enable else 0), "rbf_set_graphs")


def rbf_setup_kernel_times(h: int, precision: int = RBF_FP64) -> dict:
    """{kind: (total ms, launches)} of the last profiled rbf_precond_setup."""
    ms = (C.c_double * RBF_K_SETUP_KINDS)()
    n = (C.c_int * RBF_K_SETUP_KINDS)()
    _check(lib().rbf_setup_kernel_times(h, precision, ms, n), "rbf_setup_kernel_times")
    return {SETUP_KERNELS[k]: (ms[k], n[k]) for k in range(RBF_K_SETUP_KINDS)}


def rbf_server_create(max_active: int = 8, max_device_bytes: int = 0, packed: int = 2,
                      graphs: bool = True, pack_max_points: int = 65536) -> int:
    """packed: number of packed engines (0: one stream per request); requests
    above pack_max_points points (0: no limit) solve alone."""
    o = ServerOpts()
    lib().rbf_server_default_opts(C.byref(o))
    o.max_active = max_active
    o.max_device_bytes = max_device_bytes
    o.packed = int(packed)
    o.graphs = 1 if graphs else 0
    o.pack_max_points = int(pack_max_points)
    h = C.c_void_p()
    _check(lib().rbf_server_create(C.byref(o), C.byref(h)), "rbf_server_create")
    return h.value


def rbf_server_submit(srv: int, points, values, sigma: float, cutoff: float, overlap: int = 1,
                      opts: SolveOpts | None = None) -> int:
    pts = _host(points).reshape(-1, 2)
    vals = _host(values)
    rid = C.c_longlong()
    _check(lib().rbf_server_submit(srv, _ptr(pts), _ptr(vals), pts.shape[0], sigma, cutoff,
                                   overlap, C.byref(opts) if opts is not None else None,
                                   C.byref(rid)), "rbf_server_submit")
    return rid.value


def rbf_server_wait(srv: int, rid: int, n: int, ok=(RBF_OK, RBF_ENOCONV)):
    """(lambda (original order) or None, RequestResult, status)."""
    lam = np.empty(n)
    res = RequestResult()
    st = lib().rbf_server_wait(srv, rid, _ptr(lam), C.byref(res))
    if st not in ok:
        raise RbfError(st, "rbf_server_wait", res.message.decode() or last_error())
    return (lam if st in (RBF_OK, RBF_ENOCONV) else None), res, st


def rbf_server_stats(srv: int) -> dict:
    sub, fin = C.c_longlong(), C.c_longlong()
    act, que = C.c_int(), C.c_int()
    b = C.c_size_t()
    _check(lib().rbf_server_stats(srv, C.byref(sub), C.byref(fin), C.byref(act), C.byref(que),
                                  C.byref(b)), "rbf_server_stats")
    return {"submitted": sub.value, "finished": fin.value, "active": act.value,
            "queued": que.value, "bytes_charged": b.value}


def rbf_server_destroy(srv: int):
    if srv:
        lib().rbf_server_destroy(srv)


def rbf_precond_block(h: int, cell: int, precision: int = RBF_FP64):
    no, nc = C.c_int(), C.c_int()
    _check(lib().rbf_precond_block(h, cell, precision, None, None, C.byref(no), C.byref(nc)),
           "rbf_precond_block")
    mem = np.empty(max(no.value, 1), np.int64)
    z = np.empty((max(nc.value, 1), max(no.value, 1)))
    _check(lib().rbf_precond_block(h, cell, precision, _ptr(mem), _ptr(z), C.byref(no),
                                   C.byref(nc)), "rbf_precond_block")
    return mem[: no.value], z[: nc.value, : no.value]


# ---- convenience wrapper (same calls, owns the handle) -----------------------

@dataclass
class Result:
    weights: np.ndarray
    info: dict
    status: int


class Problem:
    """An interpolation problem on the GPU: rbf_setup + rbf_solve + rbf_evaluate."""

    def __init__(self, points, values, sigma: float, cutoff: float, overlap: int = 1):
        pts = _host(points).reshape(-1, 2)
        self.n = pts.shape[0]
        self.sigma, self.cutoff, self.overlap = sigma, cutoff, overlap
        self.h = rbf_setup(pts, values, sigma, cutoff, overlap)

    def close(self):
        if getattr(self, "h", None):
            rbf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, rtol=1e-10, restart=30, precision=RBF_FP64, max_iters=10000,
              inner_rtol=1e-4, max_outer=60, lambda0=None, ok=(RBF_OK,)) -> Result:
        o = default_opts(rtol=rtol, restart=restart, precision=precision, max_iters=max_iters,
                         inner_rtol=inner_rtol, max_outer=max_outer)
        w, info, st = rbf_solve(self.h, self.n, o, lambda0, ok)
        return Result(w, info.as_dict(), st)

    def evaluate(self, targets) -> np.ndarray:
        return rbf_evaluate(self.h, targets)

    def binning(self):
        return rbf_binning(self.h, self.n)

    def grid(self):
        return rbf_grid(self.h)

    def neighbor_counts(self):
        return rbf_neighbor_counts(self.h, self.n)
