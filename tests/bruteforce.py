"""Independent brute-force references used to pin the oracle.

dense_H: the system operator of Section 2.3 (Eq. 8) computed voxel by voxel:
the length of the segment S->P inside each closed voxel box, by clipping the
segment's parameter range against the box's slabs (Liang-Barsky).  This uses
no plane-crossing list and no midpoint rule, so it checks Siddon's method of
the oracle from a different direction.
"""
from __future__ import annotations

import numpy as np


def _slab(s, d, lo, hi):
    if d == 0.0:
        return (-np.inf, np.inf) if (lo <= s <= hi) else (np.inf, -np.inf)
    t0, t1 = (lo - s) / d, (hi - s) / d
    return (min(t0, t1), max(t0, t1))


def grid_edges(geom):
    x = -geom.nx * geom.dx / 2 + np.arange(geom.nx + 1) * geom.dx
    y = -geom.ny * geom.dy / 2 + np.arange(geom.ny + 1) * geom.dy
    nz = geom.nz if geom.kind == 1 else 1
    z = -nz * geom.dz / 2 + np.arange(nz + 1) * geom.dz
    return x, y, z


def ray_row(geom, S, P):
    """One row of H: intersection lengths of S->P with every voxel."""
    is3d = geom.kind == 1
    xe, ye, ze = grid_edges(geom)
    D = np.asarray(P, float) - np.asarray(S, float)
    if not is3d:
        D[2] = 0.0
    L = np.linalg.norm(D)
    nz = geom.nz if is3d else 1
    row = np.zeros(nz * geom.ny * geom.nx)
    xs = [_slab(S[0], D[0], xe[i], xe[i + 1]) for i in range(geom.nx)]
    ys = [_slab(S[1], D[1], ye[j], ye[j + 1]) for j in range(geom.ny)]
    zs = [_slab(S[2], D[2], ze[k], ze[k + 1]) for k in range(nz)] if is3d else [(-np.inf, np.inf)]
    for k in range(nz):
        for j in range(geom.ny):
            for i in range(geom.nx):
                lo = max(0.0, xs[i][0], ys[j][0], zs[k][0])
                hi = min(1.0, xs[i][1], ys[j][1], zs[k][1])
                if hi > lo:
                    row[(k * geom.ny + j) * geom.nx + i] = (hi - lo) * L
    return row


def box_chord(geom, S, P):
    """Length of S->P inside the whole grid box (closed form)."""
    is3d = geom.kind == 1
    xe, ye, ze = grid_edges(geom)
    D = np.asarray(P, float) - np.asarray(S, float)
    if not is3d:
        D[2] = 0.0
    lo, hi = 0.0, 1.0
    for a, (e0, e1) in enumerate([(xe[0], xe[-1]), (ye[0], ye[-1]), (ze[0], ze[-1])]):
        if a == 2 and not is3d:
            continue
        t0, t1 = _slab(S[a], D[a], e0, e1)
        lo, hi = max(lo, t0), min(hi, t1)
    return max(hi - lo, 0.0) * np.linalg.norm(D)


def disk_chord(S, P, cx, cy, R, zlo=-np.inf, zhi=np.inf):
    """Length of S->P inside the cylinder x^2+y^2<=R^2 (axis z, centre cx,cy), z in [zlo,zhi]."""
    S = np.asarray(S, float)
    D = np.asarray(P, float) - S
    px, py = S[..., 0] - cx, S[..., 1] - cy
    A = D[..., 0] ** 2 + D[..., 1] ** 2
    B = 2 * (px * D[..., 0] + py * D[..., 1])
    C = px * px + py * py - R * R
    disc = B * B - 4 * A * C
    ok = disc > 0
    sq = np.sqrt(np.where(ok, disc, 0))
    lo = np.where(ok, (-B - sq) / (2 * A), 0)
    hi = np.where(ok, (-B + sq) / (2 * A), 0)
    if np.isfinite(zlo):
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (zlo - S[..., 2]) / D[..., 2]
            t1 = (zhi - S[..., 2]) / D[..., 2]
        lo = np.maximum(lo, np.minimum(t0, t1))
        hi = np.minimum(hi, np.maximum(t0, t1))
    lo, hi = np.maximum(lo, 0), np.minimum(hi, 1)
    return np.maximum(hi - lo, 0) * np.linalg.norm(D, axis=-1)
