"""Continuous phantoms with closed-form chords, and their rasterisation.

A phantom is a list of objects, each with a material and a parent material.
Its attenuation map is additive:
    mu(x, E) = sum_k [mu_{m_k}(E) - mu_{parent_k}(E)] * 1[x in object_k],
so an object that lies inside its parent replaces the parent's material
there.  The line integral of such a map along a ray is the sum of the
objects' chords weighted by the same differences, which makes the simulated
measurements exact for the continuous object (no voxel model).

Shapes: elliptic cylinders with axis along z (ellipses in 2D) and finite
circular cylinders with any axis (the pedicle screws of the helical
workload).  A blob phantom (sums of Gaussians in the two basis components)
has a closed-form line integral too.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .physics import mu as material_mu, ENERGY_KEV, basis_mu

_EPS = 1e-300


def _quad_interval(A, B, C):
    """Interval where A a^2 + B a + C <= 0 (A > 0); empty -> (0, 0)."""
    disc = B * B - 4.0 * A * C
    ok = (disc > 0.0) & (A > 0.0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    den = np.where(ok, 2.0 * A, 1.0)
    lo = np.where(ok, (-B - sq) / den, 0.0)
    hi = np.where(ok, (-B + sq) / den, 0.0)
    return lo, hi


def _slab_interval(s, d, lo_b, hi_b):
    """Ray parameters where lo_b <= s + a d <= hi_b."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (lo_b - s) / d
        t1 = (hi_b - s) / d
    par = d == 0.0
    inside = (s >= lo_b) & (s <= hi_b)
    lo = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(t0, t1))
    hi = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(t0, t1))
    return lo, hi


@dataclass
class EllipticCylinder:
    """Ellipse (cx, cy, semi-axes a, b, rotation theta) extruded over [zlo, zhi]."""
    cx: float
    cy: float
    a: float
    b: float
    material: str
    parent: str
    theta: float = 0.0
    zlo: float = -math.inf
    zhi: float = math.inf

    def chord(self, S, P):
        D = P - S
        c, s = math.cos(self.theta), math.sin(self.theta)
        px, py = S[:, 0] - self.cx, S[:, 1] - self.cy
        q0x = (c * px + s * py) / self.a
        q0y = (-s * px + c * py) / self.b
        q1x = (c * D[:, 0] + s * D[:, 1]) / self.a
        q1y = (-s * D[:, 0] + c * D[:, 1]) / self.b
        A = q1x * q1x + q1y * q1y
        B = 2.0 * (q0x * q1x + q0y * q1y)
        C = q0x * q0x + q0y * q0y - 1.0
        lo, hi = _quad_interval(A, B, C)
        if math.isfinite(self.zlo) or math.isfinite(self.zhi):
            zl, zh = _slab_interval(S[:, 2], D[:, 2], self.zlo, self.zhi)
            lo, hi = np.maximum(lo, zl), np.minimum(hi, zh)
        lo, hi = np.maximum(lo, 0.0), np.minimum(hi, 1.0)
        return np.maximum(hi - lo, 0.0) * np.linalg.norm(D, axis=1)

    def contains(self, X):
        c, s = math.cos(self.theta), math.sin(self.theta)
        px, py = X[..., 0] - self.cx, X[..., 1] - self.cy
        u = (c * px + s * py) / self.a
        v = (-s * px + c * py) / self.b
        inside = u * u + v * v <= 1.0
        if X.shape[-1] > 2:
            inside &= (X[..., 2] >= self.zlo) & (X[..., 2] <= self.zhi)
        return inside

    def bbox(self):
        r = max(self.a, self.b)
        return (self.cx - r, self.cx + r, self.cy - r, self.cy + r, self.zlo, self.zhi)


@dataclass
class Cylinder:
    """Finite circular cylinder: centre, unit axis, radius, half-length."""
    center: tuple
    axis: tuple
    radius: float
    half_length: float
    material: str
    parent: str

    def chord(self, S, P):
        D = P - S
        c = np.asarray(self.center, dtype=np.float64)
        a = np.asarray(self.axis, dtype=np.float64)
        a = a / np.linalg.norm(a)
        w = S - c
        wa = w[:, 0] * a[0] + w[:, 1] * a[1] + w[:, 2] * a[2]
        da = D[:, 0] * a[0] + D[:, 1] * a[1] + D[:, 2] * a[2]
        q0 = w - wa[:, None] * a
        q1 = D - da[:, None] * a
        A = (q1 * q1).sum(axis=1)
        B = 2.0 * (q0 * q1).sum(axis=1)
        C = (q0 * q0).sum(axis=1) - self.radius ** 2
        lo, hi = _quad_interval(A, B, C)
        zl, zh = _slab_interval(wa, da, -self.half_length, self.half_length)
        lo, hi = np.maximum(np.maximum(lo, zl), 0.0), np.minimum(np.minimum(hi, zh), 1.0)
        return np.maximum(hi - lo, 0.0) * np.linalg.norm(D, axis=1)

    def contains(self, X):
        c = np.asarray(self.center, dtype=np.float64)
        a = np.asarray(self.axis, dtype=np.float64)
        a = a / np.linalg.norm(a)
        w = X - c
        t = w[..., 0] * a[0] + w[..., 1] * a[1] + w[..., 2] * a[2]
        r2 = (w * w).sum(axis=-1) - t * t
        return (r2 <= self.radius ** 2) & (np.abs(t) <= self.half_length)

    def bbox(self):
        c = np.asarray(self.center, dtype=np.float64)
        a = np.asarray(self.axis, dtype=np.float64)
        a = a / np.linalg.norm(a)
        ext = np.abs(a) * self.half_length + self.radius
        return (c[0] - ext[0], c[0] + ext[0], c[1] - ext[1], c[1] + ext[1],
                c[2] - ext[2], c[2] + ext[2])


METALS = ("titanium", "steel")


@dataclass
class MaterialPhantom:
    objects: list
    materials: list = field(default_factory=list)

    def __post_init__(self):
        mats = []
        for o in self.objects:
            for m in (o.material, o.parent):
                if m not in mats:
                    mats.append(m)
        self.materials = mats

    def mu_table(self, e_kev=ENERGY_KEV):
        return np.stack([material_mu(m, e_kev) for m in self.materials])

    def path_lengths(self, S, P):
        """Signed material path lengths (n, n_materials) in mm."""
        L = np.zeros((S.shape[0], len(self.materials)))
        for o in self.objects:
            ch = o.chord(S, P)
            L[:, self.materials.index(o.material)] += ch
            L[:, self.materials.index(o.parent)] -= ch
        return L

    def metal_objects(self):
        return [o for o in self.objects if o.material in METALS]


@dataclass
class BlobPhantom:
    """c_i(x) = base_i * 1[x in box] + sum_k A_ik exp(-|x-m_k|^2 / (2 s_k^2)), 2D only.

    The base term covers the voxel grid (a box of half-widths hx, hy)."""
    base: np.ndarray      # (2,)
    amp: np.ndarray       # (2, K)
    centers: np.ndarray   # (K, 2)
    sigma: np.ndarray     # (K,)
    hx: float
    hy: float

    def basis_line_integrals(self, S, P):
        D = P - S
        Ln = np.linalg.norm(D[:, :2], axis=1)
        e = D[:, :2] / Ln[:, None]
        out = np.zeros((S.shape[0], 2))
        # box chord for the constant part
        lx, hx_ = _slab_interval(S[:, 0], D[:, 0], -self.hx, self.hx)
        ly, hy_ = _slab_interval(S[:, 1], D[:, 1], -self.hy, self.hy)
        lo = np.maximum(np.maximum(lx, ly), 0.0)
        hi = np.minimum(np.minimum(hx_, hy_), 1.0)
        box = np.maximum(hi - lo, 0.0) * Ln
        out += box[:, None] * self.base[None, :]
        for k in range(len(self.sigma)):
            w = self.centers[k][None, :] - S[:, :2]
            t = (w * e).sum(axis=1)
            d2 = (w * w).sum(axis=1) - t * t
            s = self.sigma[k]
            # full-line integral; the ray end points lie far outside every blob
            li = s * math.sqrt(2.0 * math.pi) * np.exp(-np.maximum(d2, 0.0) / (2.0 * s * s))
            out += li[:, None] * self.amp[:, k][None, :]
        return out

    def sample(self, X):
        """Values of (c1, c2) at points X (..., 2)."""
        inside = (np.abs(X[..., 0]) <= self.hx) & (np.abs(X[..., 1]) <= self.hy)
        out = np.zeros(X.shape[:-1] + (2,))
        out += inside[..., None] * self.base
        for k in range(len(self.sigma)):
            d2 = ((X - self.centers[k]) ** 2).sum(-1)
            out += np.exp(-d2 / (2.0 * self.sigma[k] ** 2))[..., None] * self.amp[:, k]
        return out


def random_blobs(seed, n_blobs, radius, geom, base=(0.05, 0.01)):
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(0, 1, n_blobs))
    th = rng.uniform(0, 2 * np.pi, n_blobs)
    centers = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    sigma = rng.uniform(8.0, 25.0, n_blobs)
    amp = np.stack([rng.uniform(0.05, 0.4, n_blobs), rng.uniform(0.0, 0.15, n_blobs)])
    return BlobPhantom(base=np.asarray(base, dtype=np.float64), amp=amp, centers=centers,
                       sigma=sigma, hx=geom.nx * geom.dx / 2, hy=geom.ny * geom.dy / 2)


def voxel_centres(geom):
    x = (np.arange(geom.nx) + 0.5) * geom.dx - geom.nx * geom.dx / 2
    y = (np.arange(geom.ny) + 0.5) * geom.dy - geom.ny * geom.dy / 2
    return x, y


def metal_fraction(phantom: MaterialPhantom, geom, ss: int):
    """Fraction of each voxel covered by metal, from ss^d sub-samples."""
    from .geometry import HELICAL3D
    is3d = geom.kind == HELICAL3D
    nz = geom.nz if is3d else 1
    frac = np.zeros((nz, geom.ny, geom.nx))
    x0, y0 = -geom.nx * geom.dx / 2, -geom.ny * geom.dy / 2
    z0 = -geom.nz * geom.dz / 2
    offs = (np.arange(ss) + 0.5) / ss
    for o in phantom.metal_objects():
        bx0, bx1, by0, by1, bz0, bz1 = o.bbox()
        ix0 = max(int(math.floor((bx0 - x0) / geom.dx)), 0)
        ix1 = min(int(math.ceil((bx1 - x0) / geom.dx)), geom.nx)
        iy0 = max(int(math.floor((by0 - y0) / geom.dy)), 0)
        iy1 = min(int(math.ceil((by1 - y0) / geom.dy)), geom.ny)
        if is3d:
            iz0 = max(int(math.floor((max(bz0, z0 - 1) - z0) / geom.dz)), 0)
            iz1 = min(int(math.ceil((min(bz1, -z0 + 1) - z0) / geom.dz)), geom.nz)
        else:
            iz0, iz1 = 0, 1
        if ix0 >= ix1 or iy0 >= iy1 or iz0 >= iz1:
            continue
        xs = x0 + (np.arange(ix0, ix1)[:, None] + offs[None, :]).ravel() * geom.dx
        ys = y0 + (np.arange(iy0, iy1)[:, None] + offs[None, :]).ravel() * geom.dy
        if is3d:
            zs = z0 + (np.arange(iz0, iz1)[:, None] + offs[None, :]).ravel() * geom.dz
            Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
            pts = np.stack([X, Y, Z], axis=-1)
            inside = o.contains(pts).astype(np.float64)
            inside = inside.reshape(iz1 - iz0, ss, iy1 - iy0, ss, ix1 - ix0, ss)
            f = inside.mean(axis=(1, 3, 5))
        else:
            Y, X = np.meshgrid(ys, xs, indexing="ij")
            pts = np.stack([X, Y], axis=-1)
            inside = o.contains(pts).astype(np.float64)
            inside = inside.reshape(iy1 - iy0, ss, ix1 - ix0, ss)
            f = inside.mean(axis=(1, 3))[None]
        sub = frac[iz0:iz1, iy0:iy1, ix0:ix1]
        frac[iz0:iz1, iy0:iy1, ix0:ix1] = np.minimum(sub + f, 1.0)
    return frac if is3d else frac[0]


def basis_image(phantom: MaterialPhantom, geom, I0, ss: int = 4):
    """Basis images (2, V) of a 2D phantom: each of ss x ss sub-samples of a
    pixel takes the basis fractions of the material of the innermost object
    containing it (the objects are listed outermost first), averaged."""
    from .physics import material_in_basis
    coef = {m: material_in_basis(m, I0) for m in phantom.materials}
    coef.setdefault("air", np.zeros(2))
    x0, y0 = -geom.nx * geom.dx / 2, -geom.ny * geom.dy / 2
    offs = (np.arange(ss) + 0.5) / ss
    xs = x0 + (np.arange(geom.nx)[:, None] + offs[None, :]).ravel() * geom.dx
    ys = y0 + (np.arange(geom.ny)[:, None] + offs[None, :]).ravel() * geom.dy
    X = np.stack(np.meshgrid(xs, ys, indexing="xy"), axis=-1)       # (ny*ss, nx*ss, 2)
    first = phantom.objects[0].parent if phantom.objects else "air"
    out = np.zeros(X.shape[:2] + (2,))
    out[...] = coef.get(first, np.zeros(2))
    for o in phantom.objects:
        inside = o.contains(X)
        out[inside] = coef[o.material]
    out = out.reshape(geom.ny, ss, geom.nx, ss, 2).mean(axis=(1, 3))
    return np.ascontiguousarray(out.reshape(-1, 2).T)
