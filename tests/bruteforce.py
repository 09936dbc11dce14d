"""Independent O(N^2) reference pieces for pinning the oracle (tests only).

Nothing here calls the oracle or the GPU library.  The in-cutoff decision is
the same one both implementations take (squared distance rounded as
fma(dx, dx, dy*dy), compared with cutoff*cutoff); numpy has no fused
multiply-add, so pairs whose two-rounding value lies within a few ulps of the
threshold are re-decided in exact rational arithmetic.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def fma_exact(a: float, b: float, c: float) -> float:
    """Correctly rounded a*b + c (Python int division rounds correctly)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def pair_d2(px, py, qx, qy):
    """Two-rounding squared distances between all pairs (rows p, columns q)."""
    dx = px[:, None] - qx[None, :]
    dy = py[:, None] - qy[None, :]
    return dx * dx + dy * dy, dx, dy


def cutoff_mask(px, py, qx, qy, cutoff: float) -> np.ndarray:
    """Boolean matrix: fma(dx, dx, dy*dy) <= cutoff*cutoff for every pair."""
    rc2 = cutoff * cutoff
    d2, dx, dy = pair_d2(px, py, qx, qy)
    mask = d2 <= rc2
    near = np.abs(d2 - rc2) <= 8 * np.spacing(rc2)
    for i, j in zip(*np.nonzero(near)):
        exact = fma_exact(float(dx[i, j]), float(dx[i, j]), float(dy[i, j]) * float(dy[i, j]))
        mask[i, j] = exact <= rc2
    return mask


def gaussian(d2, sigma: float):
    """Normalised 2-D Gaussian exp(-d^2/(2 sigma^2)) / (2 pi sigma^2)."""
    return np.exp(-d2 / (2.0 * sigma * sigma)) / (2.0 * np.pi * sigma * sigma)


def dense_matrix(points, sigma: float, cutoff: float | None):
    """Dense interpolation matrix; truncated at the cutoff unless cutoff is None."""
    x, y = points[:, 0], points[:, 1]
    d2, _, _ = pair_d2(x, y, x, y)
    a = gaussian(d2, sigma)
    if cutoff is not None:
        a = np.where(cutoff_mask(x, y, x, y, cutoff), a, 0.0)
    return a


def cells_of(points, cutoff: float):
    """Cell coordinates on the grid anchored at the minimum corner, side = cutoff."""
    x0, y0 = points[:, 0].min(), points[:, 1].min()
    inv = 1.0 / cutoff
    cx = np.floor((points[:, 0] - x0) * inv).astype(np.int64)
    cy = np.floor((points[:, 1] - y0) * inv).astype(np.int64)
    return cx, cy, int(cx.max()) + 1, int(cy.max()) + 1


def rasm_dense(points, sigma: float, cutoff: float, overlap: int = 1):
    """Explicit M^{-1} = sum_c Rt_c^T inv(A_c) R_c with numpy.linalg.inv.

    A_c is the untruncated Gaussian on the points of the (2*overlap+1)^2 block
    of cells around cell c; only the rows of c's own points are kept.
    """
    n = points.shape[0]
    cx, cy, ncx, ncy = cells_of(points, cutoff)
    minv = np.zeros((n, n))
    for c_y in range(ncy):
        for c_x in range(ncx):
            own = np.nonzero((cx == c_x) & (cy == c_y))[0]
            if own.size == 0:
                continue
            sub = np.nonzero((np.abs(cx - c_x) <= overlap) & (np.abs(cy - c_y) <= overlap))[0]
            pts = points[sub]
            d2, _, _ = pair_d2(pts[:, 0], pts[:, 1], pts[:, 0], pts[:, 1])
            inv = np.linalg.inv(gaussian(d2, sigma))
            pos = {int(g): k for k, g in enumerate(sub)}
            rows = [pos[int(g)] for g in own]
            minv[np.ix_(own, sub)] = inv[rows, :]
    return minv


def boxes(points, B: float):
    """Subdomain boxes of side B on the grid anchored at the minimum corner:
    box index of every point, the box grid's size and every box's centre."""
    x0, y0 = points[:, 0].min(), points[:, 1].min()
    inv = 1.0 / B
    nbx = int(np.floor((points[:, 0].max() - x0) * inv)) + 1
    nby = int(np.floor((points[:, 1].max() - y0) * inv)) + 1
    bx = np.clip(np.floor((points[:, 0] - x0) * inv), 0, nbx - 1).astype(np.int64)
    by = np.clip(np.floor((points[:, 1] - y0) * inv), 0, nby - 1).astype(np.int64)
    cx = x0 + (np.arange(nbx) + 0.5) * B
    cy = y0 + (np.arange(nby) + 0.5) * B
    return by * nbx + bx, nbx, nby, cx, cy


def sorted_order(points, cutoff: float):
    """Position of every point in the (cell, index) order of the cells of side
    cutoff."""
    cx, cy, ncx, _ = cells_of(points, cutoff)
    key = (cy * ncx + cx) * points.shape[0] + np.arange(points.shape[0])
    rank = np.empty(points.shape[0], dtype=np.int64)
    rank[np.argsort(key)] = np.arange(points.shape[0])
    return rank


def box_members(points, cutoff: float, B: float, D: float, b: int):
    """Members of box b: its own points and every point within D/2 of its centre
    along both axes; the others first, then the own ones, each in the (cell,
    index) order of the cells of side cutoff."""
    box, nbx, _, cx, cy = boxes(points, B)
    own = box == b
    inside = ((np.abs(points[:, 0] - cx[b % nbx]) <= 0.5 * D)
              & (np.abs(points[:, 1] - cy[b // nbx]) <= 0.5 * D))
    rank = sorted_order(points, cutoff)
    other = np.nonzero(inside & ~own)[0]
    mine = np.nonzero(own)[0]
    return np.concatenate([other[np.argsort(rank[other])], mine[np.argsort(rank[mine])]]), len(mine)


def box_truncation_mask(points, targets, B: float, T: float):
    """mask[t, j]: source j lies in the square of side T centred on the box of
    target t (boxes of side B over `points`, targets clamped to the grid)."""
    x0, y0 = points[:, 0].min(), points[:, 1].min()
    _, nbx, nby, cx, cy = boxes(points, B)
    inv = 1.0 / B
    tbx = np.clip(np.floor((targets[:, 0] - x0) * inv), 0, nbx - 1).astype(np.int64)
    tby = np.clip(np.floor((targets[:, 1] - y0) * inv), 0, nby - 1).astype(np.int64)
    h = 0.5 * T
    return ((np.abs(points[None, :, 0] - cx[tbx][:, None]) <= h)
            & (np.abs(points[None, :, 1] - cy[tby][:, None]) <= h))


def rasm_dense_boxes(points, sigma: float, cutoff: float, B: float, D: float):
    """Explicit M^{-1} of RASM over the boxes, numpy.linalg.inv of each
    untruncated local matrix, only the rows of the box's own points kept."""
    n = points.shape[0]
    box, nbx, nby, _, _ = boxes(points, B)
    minv = np.zeros((n, n))
    for b in range(nbx * nby):
        mem, kc = box_members(points, cutoff, B, D, b)
        if kc == 0:
            continue
        pts = points[mem]
        d2, _, _ = pair_d2(pts[:, 0], pts[:, 1], pts[:, 0], pts[:, 1])
        inv = np.linalg.inv(gaussian(d2, sigma))
        minv[np.ix_(mem[len(mem) - kc:], mem)] = inv[len(mem) - kc:, :]
    return minv
