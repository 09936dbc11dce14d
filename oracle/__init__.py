"""ctypes wrapper of the CPU FP64 oracle (oracle/rbf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rbf_oracle.c")
# RBF_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; the process must preload the
# ASan runtime, see SANITIZE_FLAGS' users in tests/)
SANITIZE = os.environ.get("RBF_ORACLE_SANITIZE") == "1"
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                  "-fno-omit-frame-pointer", "-g"]
LIB = os.path.join(HERE, "librbf_oracle_san.so" if SANITIZE else "librbf_oracle.so")

STATUS = {0: "ORC_OK", 1: "ORC_EINVAL", 2: "ORC_EDUPLICATE", 3: "ORC_ENOMEM",
          5: "ORC_ENOTPD", 6: "ORC_ENOCONV", 7: "ORC_EBREAKDOWN", 8: "ORC_ENAN",
          9: "ORC_ESTATE"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
               *(SANITIZE_FLAGS if SANITIZE else []),
               "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        lp = C.POINTER(C.c_longlong)
        vp = C.c_void_p
        L.orc_create.argtypes = [dp, C.c_longlong, C.c_double, C.c_double, C.c_int,
                                 C.POINTER(vp)]
        L.orc_destroy.argtypes = [vp]
        L.orc_destroy.restype = None
        L.orc_grid.argtypes = [vp, dp, lp]
        L.orc_binning.argtypes = [vp, ip, ip, lp]
        L.orc_matvec.argtypes = [vp, dp, dp, ip]
        L.orc_evaluate.argtypes = [vp, dp, dp, C.c_longlong, dp]
        L.orc_evaluate_counts.argtypes = [vp, dp, dp, C.c_longlong, dp, ip]
        L.orc_rasm_setup.argtypes = [vp]
        L.orc_rasm_apply.argtypes = [vp, dp, dp]
        L.orc_rasm_block.argtypes = [vp, C.c_longlong, lp, ip, ip, dp]
        L.orc_rasm_block_size.argtypes = [vp, C.c_longlong, ip, ip]
        L.orc_gmres.argtypes = [vp, dp, C.c_int, C.c_double, C.c_int, dp, dp, vp, dp,
                                C.c_int]
        L.orc_rel_residual.argtypes = [vp, dp, dp, dp]
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_set_geometry.argtypes = [vp, C.c_double, C.c_double, C.c_double]
        L.orc_subdomains.argtypes = [vp, lp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_longlong)) if a is not None else None


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int),
                ("rel_residual", C.c_double), ("history_len", C.c_int)]


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    rel_residual: float
    history: np.ndarray


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


class Problem:
    """One interpolation problem held by the oracle."""

    def __init__(self, points, sigma: float, cutoff: float, overlap: int = 1):
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
        self.n = pts.shape[0]
        self.sigma, self.cutoff, self.overlap = float(sigma), float(cutoff), int(overlap)
        h = C.c_void_p()
        rc = lib().orc_create(_dp(pts), self.n, self.sigma, self.cutoff, self.overlap,
                              C.byref(h))
        if rc:
            raise OracleError(rc, "orc_create")
        self._h = h
        g = np.zeros(4)
        nc = np.zeros(2, dtype=np.int64)
        lib().orc_grid(self._h, _dp(g), _lp(nc))
        self.x0, self.y0, self.L, self.invL = (float(v) for v in g)
        self.ncx, self.ncy = int(nc[0]), int(nc[1])
        self.ncells = self.ncx * self.ncy

    def set_geometry(self, B: float, D: float, T: float = 0.0):
        """Subdomain boxes of side B, overlapping squares of side D, matvec
        truncation square of side T (0: the radial cutoff)."""
        rc = lib().orc_set_geometry(self._h, float(B), float(D), float(T))
        if rc:
            raise OracleError(rc, "orc_set_geometry")

    def subdomains(self):
        nxy = np.zeros(2, dtype=np.int64)
        lib().orc_subdomains(self._h, _lp(nxy))
        return int(nxy[0]), int(nxy[1])

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def binning(self):
        cell_of = np.empty(self.n, dtype=np.int32)
        perm = np.empty(self.n, dtype=np.int32)
        cs = np.empty(self.ncells + 1, dtype=np.int64)
        rc = lib().orc_binning(self._h, _ip(cell_of), _ip(perm), _lp(cs))
        if rc:
            raise OracleError(rc, "orc_binning")
        return cell_of, perm, cs

    def matvec(self, w, with_counts: bool = False):
        w = np.ascontiguousarray(w, dtype=np.float64)
        y = np.empty(self.n)
        nnb = np.empty(self.n, dtype=np.int32) if with_counts else None
        rc = lib().orc_matvec(self._h, _dp(w), _dp(y), _ip(nnb))
        if rc:
            raise OracleError(rc, "orc_matvec")
        return (y, nnb) if with_counts else y

    def evaluate(self, lam, targets, with_counts: bool = False):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        t = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 2)
        out = np.empty(t.shape[0])
        nnb = np.empty(t.shape[0], dtype=np.int32) if with_counts else None
        rc = lib().orc_evaluate_counts(self._h, _dp(lam), _dp(t), t.shape[0], _dp(out), _ip(nnb))
        if rc:
            raise OracleError(rc, "orc_evaluate")
        return (out, nnb) if with_counts else out

    def rasm_setup(self):
        rc = lib().orc_rasm_setup(self._h)
        if rc:
            raise OracleError(rc, "orc_rasm_setup")

    def rasm_apply(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        z = np.empty(self.n)
        rc = lib().orc_rasm_apply(self._h, _dp(v), _dp(z))
        if rc:
            raise OracleError(rc, "orc_rasm_apply")
        return z

    def rasm_block(self, cell: int, with_factor: bool = True):
        k = C.c_int()
        kc = C.c_int()
        rc = lib().orc_rasm_block_size(self._h, cell, C.byref(k), C.byref(kc))
        if rc:
            raise OracleError(rc, "orc_rasm_block_size")
        mem = np.empty(max(k.value, 1), dtype=np.int64)
        L = np.empty((k.value, k.value), dtype=np.float64) if with_factor else None
        rc = lib().orc_rasm_block(self._h, cell, _lp(mem), C.byref(k), C.byref(kc),
                                  _dp(L))
        if rc:
            raise OracleError(rc, "orc_rasm_block")
        # stored column-major: transpose the row-major view
        return mem[: k.value], kc.value, (L.T.copy() if L is not None else None)

    def gmres(self, f, restart: int = 30, rtol: float = 1e-10, max_iters: int = 10000,
              x0=None, raise_on_error: bool = True):
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.empty(self.n)
        x0a = np.ascontiguousarray(x0, dtype=np.float64) if x0 is not None else None
        info = _Info()
        hist = np.zeros(4096)
        rc = lib().orc_gmres(self._h, _dp(f), restart, rtol, max_iters, _dp(x0a), _dp(x),
                             C.cast(C.byref(info), C.c_void_p), _dp(hist), hist.size)
        if rc and raise_on_error and rc != 6:
            raise OracleError(rc, "orc_gmres")
        return x, SolveInfo(rc, info.iterations, info.restarts, info.rel_residual,
                            hist[: info.history_len].copy())

    def rel_residual(self, f, x) -> float:
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = C.c_double()
        rc = lib().orc_rel_residual(self._h, _dp(f), _dp(x), C.byref(out))
        if rc:
            raise OracleError(rc, "orc_rel_residual")
        return out.value
