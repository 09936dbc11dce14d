"""The list matvec's table-driven exponential on the GPU, pair by pair, bit for
bit against its step-by-step host emulation (every fused multiply-add rounded
once, the table entries 2^(j/32) correctly rounded; the emulation and its
accuracy bound are pinned in test_capi_cpu.py) (-m gpu).

A unit weight on one source s makes the product's entry at every target i
within the cutoff of s exactly fl(2^(beta d2_is / 32) * norm): the other terms
are exact zeros, so the two partial sums add one exponential to a zero.  The
squared distance is rounded as in every product (dy*dy first, then one fused
multiply-add), beta = -32 / (2 sigma^2 ln 2) is formed in extended precision
and rounded once, as the library forms it.  Several sources of a jittered
lattice at h/sigma = 0.8 give targets over the whole cutoff range, so the
table index and the power of two take many values (Section 2.3, the
truncated Gaussian product).
"""
import math
import sys

import numpy as np
import pytest

import paper_0909_5413_amd as R
from tests.test_capi_cpu import _device_exp2_scaled, _fma

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_list_exponential_bit_exact():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    n_side = 40
    rng = np.random.default_rng(5413 + 77)
    h = 2.0 / n_side
    xs = -1 + (np.arange(n_side) + 0.5) * h
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel()], 1) + rng.uniform(-0.1 * h, 0.1 * h, (n_side ** 2, 2))
    n = pts.shape[0]
    sigma = h / 0.8
    cutoff = 6.0 * sigma
    rc2 = cutoff * cutoff
    ln2 = np.longdouble("0.693147180559945309417232121458176568")
    sl = np.longdouble(sigma)
    beta = float(np.longdouble(-16.0) / (sl * sl * ln2))
    norm = 1.0 / (2.0 * math.pi * sigma * sigma)
    say("list exponential", "n", n, "sigma", sigma)
    hd = R.rbf_setup(pts, np.zeros(n), sigma, cutoff, 1)
    try:
        checked = 0
        ks = set()
        for s in (0, 417, 820, 1203, n - 1):
            w = torch.zeros(n, dtype=torch.float64, device="cuda")
            w[s] = 1.0
            y = torch.empty_like(w)
            R.rbf_matvec_device(hd, w, y, R.RBF_FP64, R.RBF_ORDER_ORIGINAL)
            torch.cuda.synchronize()
            got = y.cpu().numpy()
            for i in range(n):
                dx = float(pts[i, 0] - pts[s, 0])
                dy = float(pts[i, 1] - pts[s, 1])
                d2 = _fma(dx, dx, dy * dy)
                if d2 <= rc2:
                    want = _device_exp2_scaled(d2, beta) * norm
                    assert got[i] == want, (s, i, d2, got[i], want)
                    ks.add(round(d2 * beta))
                    checked += 1
                else:
                    assert got[i] == 0.0, (s, i, d2, got[i])
        say("pairs checked", checked, "distinct k", len(ks))
        assert checked > 500 and len(ks) > 200
    finally:
        R.rbf_destroy(hd)
