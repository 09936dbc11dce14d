"""Tolerances of the GPU-vs-oracle comparisons, each derived from the
arithmetic it covers (test helpers; they call only the oracle)."""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53


def residual_gate(P, f, lam, rtol: float) -> float:
    """Bar for the oracle's true relative residual of weights a GPU solve
    returned with its own residual <= rtol.

    Both sides evaluate ||f - A lam|| / ||f|| in FP64 with different summation
    orders.  Each product (A lam)_i sums at most k in-cutoff terms (k the
    largest neighbour count), so either evaluation is off from the exact
    residual by at most (k + 4) u (|A| |lam|)_i per row: k additions, and per
    term the exponential's error (libm's within 1 ulp; the GPU's table-driven
    one within 5.2e-16 relative, 4.7 u: its polynomial 1.41e-16, the table
    entry and three roundings) and the product's rounding; the two together
    by twice that.
    The bar is rtol plus that difference in norm, relative to ||f||."""
    scale = P.matvec(np.abs(lam))
    _, nnb = P.matvec(np.ones_like(lam), with_counts=True)
    k = int(nnb.max())
    return rtol + 2 * (k + 4) * U64 * np.linalg.norm(scale) / np.linalg.norm(f)
