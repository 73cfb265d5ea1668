"""Independent geometry for brute-force checks on tiny inputs.

Written separately from the generator's rasterizer: overlaps are decided by
the separating-axis test on convex polygons (interiors meet iff no edge normal
of either polygon separates them, touching counts as separated) and by
segment distances for discs.  The label of Sec. 4, Eq. labeling_op, restricted
to the grid (Sec. 4.1 encoding), is then: proposition p labels trajectory t
iff some sampled footprint of t and some region of p overlap a common cell.
"""
from __future__ import annotations

import numpy as np

import gen


def footprint_polys(poses: np.ndarray) -> np.ndarray:
    """(n, 4, 2) corners of the 4.5 x 2.0 rectangles centred on poses."""
    hl, hw = gen.FOOT_LEN / 2.0, gen.FOOT_WID / 2.0
    local = np.array([[hl, hw], [-hl, hw], [-hl, -hw], [hl, -hw]])
    c, s = np.cos(poses[:, 2]), np.sin(poses[:, 2])
    rot = np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)  # (n, 2, 2)
    return poses[:, None, :2] + np.einsum("nij,kj->nki", rot, local)


def cell_polys(n: int, res: float) -> np.ndarray:
    """(n*n, 4, 2) corners of every cell, row-major ids."""
    iy, ix = np.divmod(np.arange(n * n), n)
    x0, y0 = ix * res, iy * res
    return np.stack([np.stack([x0, y0], -1), np.stack([x0 + res, y0], -1),
                     np.stack([x0 + res, y0 + res], -1), np.stack([x0, y0 + res], -1)], 1)


def _axes(poly):
    e = np.roll(poly, -1, axis=-2) - poly
    return np.stack([-e[..., 1], e[..., 0]], -1)  # edge normals, (..., 4, 2)


def sat_overlap(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Positive-area overlap of convex polygons; A (a, 4, 2), B (b, 4, 2) -> (a, b) bool."""
    Aa = A[:, None, :, :]
    Bb = B[None, :, :, :]
    ok = np.ones((A.shape[0], B.shape[0]), bool)
    for axes in (_axes(A)[:, None], _axes(B)[None, :]):
        for k in range(4):
            ax = axes[..., k, :]
            pa = np.einsum("abvk,abk->abv", np.broadcast_to(Aa, (A.shape[0], B.shape[0], 4, 2)),
                           np.broadcast_to(ax, (A.shape[0], B.shape[0], 2)))
            pb = np.einsum("abvk,abk->abv", np.broadcast_to(Bb, (A.shape[0], B.shape[0], 4, 2)),
                           np.broadcast_to(ax, (A.shape[0], B.shape[0], 2)))
            lo = np.maximum(pa.min(-1), pb.min(-1))
            hi = np.minimum(pa.max(-1), pb.max(-1))
            ok &= lo < hi
    return ok


def _seg_dist(p, a, b):
    """Distance from points p (..., 2) to segments a-b (..., 2)."""
    ab = b - a
    t = np.clip(np.sum((p - a) * ab, -1) / np.sum(ab * ab, -1), 0.0, 1.0)
    q = a + t[..., None] * ab
    return np.linalg.norm(p - q, axis=-1)


def point_in_convex(p, poly):
    """p (m, 2) inside closed convex polygon poly (4, 2) given counter-clockwise or clockwise."""
    e = np.roll(poly, -1, 0) - poly
    r = p[:, None, :] - poly[None, :, :]
    cr = e[None, :, 0] * r[..., 1] - e[None, :, 1] * r[..., 0]
    return np.all(cr >= 0, 1) | np.all(cr <= 0, 1)


def disc_cell_overlap(cx, cy, r, cells):
    """Positive-area overlap of a disc with each cell square: the centre is
    inside the square, or some edge passes closer than r."""
    c = np.array([cx, cy])
    x0, y0 = cells[:, 0, 0], cells[:, 0, 1]
    x1, y1 = cells[:, 2, 0], cells[:, 2, 1]
    inside = (cx > x0) & (cx < x1) & (cy > y0) & (cy < y1)
    d = np.full(len(cells), np.inf)
    for k in range(4):
        a = cells[:, k, :]
        b = cells[:, (k + 1) % 4, :]
        d = np.minimum(d, _seg_dist(np.broadcast_to(c, a.shape), a, b))
    return inside | (d < r)


def shape_poly(kind, cx, cy, a, b):
    if kind != 0:
        raise ValueError("not a rectangle")
    return np.array([[cx - a, cy - b], [cx + a, cy - b], [cx + a, cy + b], [cx - a, cy + b]])


def brute_cover_footprints(poses, n, res):
    """Cells overlapped by any footprint: bool (n*n,)."""
    cells = cell_polys(n, res)
    F = footprint_polys(poses)
    out = np.zeros(n * n, bool)
    for i in range(0, len(F), 64):
        out |= sat_overlap(F[i:i + 64], cells).any(0)
    return out


def brute_cover_shape(kind, cx, cy, a, b, n, res):
    cells = cell_polys(n, res)
    if kind == 0:
        return sat_overlap(shape_poly(kind, cx, cy, a, b)[None], cells)[0]
    return disc_cell_overlap(cx, cy, a, cells)


def poly_poly_dist(A, B):
    """Distance between closed convex polygons A, B (4, 2) each."""
    if sat_overlap(A[None], B[None])[0, 0]:
        return 0.0
    best = np.inf
    for P, Q in ((A, B), (B, A)):
        for k in range(4):
            a, b = Q[k], Q[(k + 1) % 4]
            best = min(best, float(_seg_dist(P, np.broadcast_to(a, P.shape), np.broadcast_to(b, P.shape)).min()))
    return best


def poly_disc_dist(A, cx, cy, r):
    c = np.array([[cx, cy]])
    if point_in_convex(c, A)[0]:
        return 0.0
    d = min(float(_seg_dist(c[0], A[k], A[(k + 1) % 4])) for k in range(4))
    return max(0.0, d - r)
