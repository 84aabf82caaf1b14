"""Scanner geometry for the synthetic DEAM workloads.

The system operator h(x, y) of the forward model (Section 2.3, Eq. 8) is
defined by a third-generation fan-beam scanner (2D) or a helical cone-beam
scanner with a cylindrical detector (3D).  The paper names the scanner type
(a helical fan-beam CT system, Section 2.3 and Section 3) but not its
parameters, so this module fixes one convention that the oracle and the GPU
library each implement on their own:

* Voxel (ix, iy, iz) covers [x0 + ix*dx, x0 + (ix+1)*dx] x [...] x [...],
  with x0 = -nx*dx/2, y0 = -ny*dy/2, z0 = -nz*dz/2; storage index
  (iz*ny + iy)*nx + ix (x fastest).
* View v: beta = beta0 + 2*pi*v/views_per_rot; source
  S = (sid*cos(beta), sid*sin(beta), z_s(v)); central direction
  u = -(cos(beta), sin(beta), 0);
  z_s(v) = (v - (n_views-1)/2) * feed_per_rot / views_per_rot.
* Channel k: gamma_k = (k - (n_cols-1)/2 - col_offset) * dgamma (equiangular
  arc centred on the source); row r: zeta_r = (r - (n_rows-1)/2) * drow_iso *
  sdd/sid.  Detector cell centre P = S + sdd*R(gamma_k)u + (0, 0, zeta_r).
* One ray per detector cell, the segment S -> P; ray index
  (v*n_rows + r)*n_cols + k (channel fastest).

This module only describes the scanner and produces ray end points for the
measurement simulation; it contains no part of the reconstruction method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

FAN2D = 0
HELICAL3D = 1


@dataclass(frozen=True)
class Geometry:
    kind: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    n_views: int
    n_rows: int
    n_cols: int
    sid: float
    sdd: float
    dgamma: float
    col_offset: float
    drow_iso: float
    beta0: float
    views_per_rot: float
    feed_per_rot: float

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_rows * self.n_cols

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def image_shape(self):
        return (self.nz, self.ny, self.nx) if self.kind == HELICAL3D else (self.ny, self.nx)

    @property
    def sino_shape(self):
        if self.kind == HELICAL3D:
            return (self.n_views, self.n_rows, self.n_cols)
        return (self.n_views, self.n_cols)

    def box_diagonal(self) -> float:
        """Length of the diagonal of the voxel grid (mm): the longest chord."""
        ex, ey = self.nx * self.dx, self.ny * self.dy
        ez = self.nz * self.dz if self.kind == HELICAL3D else 0.0
        return math.sqrt(ex * ex + ey * ey + ez * ez)

    def as_dict(self):
        return asdict(self)


def fan_dgamma(nx, ny, dx, dy, sid, n_cols):
    """Channel pitch so that the fan covers the circle circumscribing the grid."""
    r_fov = 0.5 * math.hypot(nx * dx, ny * dy)
    return 2.0 * math.asin(r_fov / sid) / n_cols


def fan2d(n, d, n_views, n_cols, sid=570.0, sdd=1040.0):
    return Geometry(kind=FAN2D, nx=n, ny=n, nz=1, dx=d, dy=d, dz=1.0,
                    n_views=n_views, n_rows=1, n_cols=n_cols, sid=sid, sdd=sdd,
                    dgamma=fan_dgamma(n, n, d, d, sid, n_cols), col_offset=0.0,
                    drow_iso=1.0, beta0=0.0, views_per_rot=float(n_views),
                    feed_per_rot=0.0)


def helical3d(n, d, nz, dz, n_rows, n_cols, views_per_rot, n_rot, pitch,
              drow_iso, sid=570.0, sdd=1040.0):
    feed = pitch * n_rows * drow_iso
    return Geometry(kind=HELICAL3D, nx=n, ny=n, nz=nz, dx=d, dy=d, dz=dz,
                    n_views=int(views_per_rot * n_rot), n_rows=n_rows,
                    n_cols=n_cols, sid=sid, sdd=sdd,
                    dgamma=fan_dgamma(n, n, d, d, sid, n_cols), col_offset=0.0,
                    drow_iso=drow_iso, beta0=0.0,
                    views_per_rot=float(views_per_rot), feed_per_rot=feed)


def ray_endpoints(g: Geometry, views=None):
    """Source and detector-cell points (mm) of the rays of the given views.

    Returns (S, P), each of shape (n, 3), in ray-index order restricted to
    ``views`` (default: all views).
    """
    views = np.arange(g.n_views) if views is None else np.asarray(views)
    beta = g.beta0 + 2.0 * np.pi * views / g.views_per_rot
    cb, sb = np.cos(beta), np.sin(beta)
    zs = (views - (g.n_views - 1) / 2.0) * g.feed_per_rot / g.views_per_rot
    gam = (np.arange(g.n_cols) - (g.n_cols - 1) / 2.0 - g.col_offset) * g.dgamma
    cg, sg = np.cos(gam), np.sin(gam)
    zeta = (np.arange(g.n_rows) - (g.n_rows - 1) / 2.0) * g.drow_iso * g.sdd / g.sid
    if g.kind == FAN2D:
        zeta = np.zeros(1)
    nv, nr, nc = len(views), len(zeta), g.n_cols
    # central direction u = -(cb, sb); rotated by gamma: R(g)u
    ux, uy = -cb[:, None], -sb[:, None]
    dxv = cg[None, :] * ux - sg[None, :] * uy
    dyv = sg[None, :] * ux + cg[None, :] * uy
    S = np.empty((nv, nr, nc, 3))
    P = np.empty((nv, nr, nc, 3))
    S[..., 0] = (g.sid * cb)[:, None, None]
    S[..., 1] = (g.sid * sb)[:, None, None]
    S[..., 2] = zs[:, None, None] if g.kind == HELICAL3D else 0.0
    P[..., 0] = S[..., 0] + g.sdd * dxv[:, None, :]
    P[..., 1] = S[..., 1] + g.sdd * dyv[:, None, :]
    P[..., 2] = S[..., 2] + zeta[None, :, None]
    return S.reshape(-1, 3), P.reshape(-1, 3)
