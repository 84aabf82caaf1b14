"""The synthetic DEAM workloads and their seeded inputs.

Each workload stands in for the paper's scanner and patient data (Section 3:
a water phantom with steel rods on a Philips Brilliance Big Bore, and a
clinical helical head-and-neck scan with 816 channels and 16 x 0.75 mm
collimation), which are not available.  The shapes follow those scans:
816-channel fan-beam and 16-row helical geometries, ~1 mm voxels, a
water-equivalent body with bone and titanium/steel implants, and 90/140 kVp
spectra with 1-keV bins from 20 to 140 keV.

``make_inputs(name)`` returns a dict with
    geom        Geometry
    I0, mu      (2, n_energy) spectra (photons per ray) and basis attenuation (1/mm)
    d           (2, n_rays) float32 Poisson counts (low, high)
    gbar        (2, n_rays) float64 expected counts of the continuous phantom
    metal       uint8 image, 1 where >= half of the voxel is metal
    t           metal-trace threshold (mm of metal path)
    c0          (2, n_voxels) float64 initial basis images (cold start)
    Z           (2,) float64 normalisers of the surrogate update
    n_iter      iteration count of the workload
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import geometry as G
from .physics import ENERGY_KEV, basis_mu, spectra, water_in_basis, mu as material_mu
from .phantoms import (EllipticCylinder as E, Cylinder, MaterialPhantom, basis_image,
                       metal_fraction, random_blobs, voxel_centres)


def geometry_for(name: str) -> G.Geometry:
    if name == "fan128":        # 128^2 at 1 mm, 180 views over 360 deg, 256 channels
        return G.fan2d(128, 1.0, 180, 256)
    if name == "fan512":        # 512^2 at 0.98 mm, 984 views, 816 channels
        return G.fan2d(512, 0.98, 984, 816)
    if name == "helical":       # 512^2 x 64, 16 x 816 detector, 1152 views/rot, 4 rot, pitch 0.5
        return G.helical3d(512, 0.98, 64, 1.0, 16, 816, 1152, 4, 0.5, 4.0 / 3.0)
    if name == "fan256":        # 256^2 at 1 mm, 360 views x 512 channels
        return G.fan2d(256, 1.0, 360, 512)
    if name == "fan64":         # small fan-beam case for quick checks
        return G.fan2d(64, 1.0, 64, 96)
    if name == "helical_small":  # small helical case: 64^2 x 16, 4 rows x 96 channels
        return G.helical3d(64, 1.0, 16, 1.0, 4, 96, 48, 2, 0.75, 2.0)
    if name == "helical_mid":   # 96^2 x 24, 8 rows x 168 channels, 320 views/rot x 2, pitch 0.75
        return G.helical3d(96, 1.0, 24, 1.0, 8, 168, 320, 2, 0.75, 1.5)
    raise KeyError(name)


WORKLOADS = {
    # name: (I0, seed, iterations)
    "fan128": (1e5, 1, 20),
    "fan512": (2e5, 2, 50),
    "helical": (2e5, 3, 30),
    "fan256": (1e5, 40, 20),
    "fan64": (1e5, 11, 20),
    "helical_small": (1e5, 13, 10),
    "helical_mid": (1e5, 14, 20),
}


# Penalty of the penalised iteration (Eqs. 6-7), (lambda, delta) per workload.
# The paper gives no values.  delta = 0.005 in basis units (about 0.5% of the
# water value of the first component).  lambda makes the penalty's curvature
# in its quadratic regime, 4 lambda sum_{x~} w(x,x~), equal to the median
# data curvature Z_1 b^_1 over the field of view at the cold start, rounded:
#   fan64          Z_1 b^_1 ~ 6.0e5, sum w = 6.83 (1 mm)        -> 2.2e4
#   fan512         Z_1 b^_1 ~ 8.7e4, sum w = 6.97 (0.98 mm)     -> 3.1e3
#   helical_small  Z_1 b^_1 ~ 2.4e5, sum w = 19.1 (26 nbrs)     -> 3.1e3
#   helical        Z_1 b^_1 ~ 8.5e4, sum w = 19.4 (26 nbrs)     -> 1.1e3
PENALTY = {
    "fan64": (2.2e4, 0.005),
    "fan512": (3.1e3, 0.005),
    "helical_small": (3.1e3, 0.005),
    "helical": (1.1e3, 0.005),
}


def mar_params(geom, I0, e_kev=ENERGY_KEV):
    """Parameters of the MAR initialisation (Section 2.2).  water_j is the
    spectrum-weighted attenuation of water (1/mm); the classes of the prior
    image are relative to it: air below 0.5, soft tissue below 1.5, bone
    above; metal at 5 or more in the high-energy image (cortical bone is ~3.9x
    water; a titanium rod of 3 mm radius reconstructs at 5.9-8.6x after beam
    hardening and partial-volume blur).  eps (line-integral units, ~0.3 mm of water)
    keeps the NMAR normalisation finite outside the object.  t is the
    metal-trace threshold of the workloads."""
    w = material_mu("water", e_kev)
    water = (I0 @ w) / I0.sum(axis=1)
    return dict(t=0.5 * min(geom.dx, geom.dy), water=water, air_frac=0.5, bone_frac=1.5,
                metal_frac=5.0, eps=0.01)


def phantom_for(name: str) -> MaterialPhantom:
    if name in ("fan128", "fan64"):
        s = 1.0 if name == "fan128" else 0.5
        return MaterialPhantom([
            E(0, 0, 50 * s, 50 * s, "water", "air"),
            E(25 * s, 0, 7.5 * s, 7.5 * s, "bone", "water"),
            E(-25 * s, 0, 7.5 * s, 7.5 * s, "bone", "water"),
            E(0, 25 * s, 3 * s, 3 * s, "titanium", "water"),
        ])
    if name == "fan512":
        objs = [E(0, 0, 200, 140, "fat", "air"), E(0, 0, 190, 130, "water", "fat"),
                E(0, -80, 35, 25, "bone", "water", theta=0.1)]
        for sx in (-1, 1):
            objs += [E(sx * 95, 0, 30, 30, "cortical_bone", "water"),
                     E(sx * 95, 0, 24, 24, "trabecular_bone", "cortical_bone"),
                     E(sx * 95, 0, 10, 8, "steel", "trabecular_bone", theta=sx * 0.3)]
        return MaterialPhantom(objs)
    if name == "helical":
        return spine_phantom(1.0, 32.0, 12.0)
    if name == "helical_small":
        return spine_phantom(0.12, 8.0, 3.0)
    if name == "helical_mid":
        return spine_phantom(0.18, 12.0, 4.5)
    raise KeyError(name)


def spine_phantom(s, zhalf, zscrew):
    """The helical workloads' phantom, in-plane lengths scaled by s: an
    elliptic body (fat around water) over |z| <= zhalf, a vertebral body
    (cortical shell, trabecular core), a posterior arch around the canal, and
    four titanium screws converging at 15 degrees, at z = -zscrew and zscrew."""
    zl, zh = -zhalf, zhalf
    objs = [E(0, 0, 180 * s, 130 * s, "fat", "air", zlo=zl, zhi=zh),
            E(0, 0, 170 * s, 120 * s, "water", "fat", zlo=zl, zhi=zh),
            E(0, -20 * s, 24 * s, 24 * s, "cortical_bone", "water", zlo=zl, zhi=zh),
            E(0, -20 * s, 22 * s, 22 * s, "trabecular_bone", "cortical_bone", zlo=zl, zhi=zh),
            E(0, -55 * s, 20 * s, 14 * s, "cortical_bone", "water", zlo=zl, zhi=zh),
            E(0, -55 * s, 9 * s, 7 * s, "water", "cortical_bone", zlo=zl, zhi=zh)]
    ang = math.radians(15.0)
    zpos = (-zscrew, zscrew)
    for sx in (-1, 1):
        d = (-sx * math.sin(ang), math.cos(ang), 0.0)
        for z in zpos:
            start = (sx * 18.0 * s, -75.0 * s, z)
            half = 22.5 * s
            c = (start[0] + half * d[0], start[1] + half * d[1], z)
            objs.append(Cylinder(c, d, max(2.5 * s, 1.0), half, "titanium", "water"))
    return MaterialPhantom(objs)


def _views_chunks(n_views, per):
    return [np.arange(a, min(a + per, n_views)) for a in range(0, n_views, per)]


def bowtie(geom, b1_edge=25.0, b2_edge=2.0):
    """A bowtie filter as its path lengths (mm) in the two basis materials per
    detector channel, shape (2, n_cols): zero on the central channel, growing
    as (gamma / gamma_max)^2 to (b1_edge, b2_edge) at the ends of the fan."""
    k = np.arange(geom.n_cols)
    gam = (k - 0.5 * (geom.n_cols - 1) - geom.col_offset) * geom.dgamma
    s = (gam / np.abs(gam).max()) ** 2
    return np.stack([b1_edge * s, b2_edge * s])


def expected_counts(geom, phantom, I0, threads=None, bt=None):
    """Expected counts (2, n_rays) of the continuous phantom, float64; with a
    bowtie bt (2, n_cols) each ray sees the spectra attenuated by the filter
    path of its channel."""
    if isinstance(phantom, MaterialPhantom):
        mu_t = phantom.mu_table()
        lengths = phantom.path_lengths
    else:
        mu_t = basis_mu()
        lengths = phantom.basis_line_integrals
    keep = I0.sum(axis=0) > 0
    mu_k, I0_k = mu_t[:, keep], I0[:, keep]
    per = max(1, 200_000 // (geom.n_rows * geom.n_cols))
    chunks = _views_chunks(geom.n_views, per)
    out = np.empty((2, geom.n_rays))

    def work(views):
        # plain ufunc sums (no BLAS): safe to run from several threads and
        # bitwise identical on every host
        S, P = G.ray_endpoints(geom, views)
        Lm = lengths(S, P)                      # (n, n_materials) path lengths
        A = np.zeros((Lm.shape[0], mu_k.shape[1]))
        for m in range(Lm.shape[1]):
            A += Lm[:, m:m + 1] * mu_k[m][None, :]   # line integral per energy
        if bt is not None:
            kk = np.arange(A.shape[0]) % geom.n_cols
            bmu = basis_mu()[:, keep]
            A += bt[0][kk][:, None] * bmu[0][None, :] + bt[1][kk][:, None] * bmu[1][None, :]
        np.negative(A, out=A)
        np.exp(A, out=A)
        a = views[0] * geom.n_rows * geom.n_cols
        for j in range(2):
            out[j, a:a + A.shape[0]] = (A * I0_k[j][None, :]).sum(axis=1)

    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, chunks))
    return out


def make_inputs(name: str, seed=None, i0=None, with_data=True, with_bowtie=False):
    geom = geometry_for(name)
    i0_d, seed_d, n_iter = WORKLOADS[name]
    seed = seed_d if seed is None else seed
    i0 = i0_d if i0 is None else i0
    I0 = spectra(i0)
    mu = basis_mu()
    inp = dict(name=name, geom=geom, I0=I0, mu=mu, energies=ENERGY_KEV.copy(),
               n_iter=n_iter, seed=seed)
    ph = phantom_for(name)
    ss = 4 if geom.kind == G.FAN2D else 2
    frac = metal_fraction(ph, geom, ss)
    inp["metal"] = (frac >= 0.5).astype(np.uint8).reshape(-1)
    inp["t"] = 0.5 * min(geom.dx, geom.dy)
    inp["c0"] = cold_start(geom, I0)
    inp["Z"] = surrogate_Z(geom, mu, I0)
    bt = bowtie(geom) if with_bowtie else None
    if bt is not None:
        inp["bt"] = bt
    if with_data:
        gbar = expected_counts(geom, ph, I0, bt=bt)
        rng = np.random.default_rng(seed)
        inp["gbar"] = gbar
        inp["d"] = rng.poisson(gbar).astype(np.float32)
    return inp


def cold_start(geom, I0):
    """Water (in basis fractions) inside the disk inscribed in the grid, zero outside."""
    w = water_in_basis(I0)
    x, y = voxel_centres(geom)
    r = 0.5 * min(geom.nx * geom.dx, geom.ny * geom.dy)
    disk = (x[None, :] ** 2 + y[:, None] ** 2) <= r * r
    nz = geom.nz if geom.kind == G.HELICAL3D else 1
    disk = np.broadcast_to(disk, (nz,) + disk.shape).reshape(-1)
    return np.stack([w[0] * disk, w[1] * disk]).astype(np.float64)


def surrogate_Z(geom, mu, I0):
    """Z_i = 2 * max_E mu_i(E) * (longest chord of the grid), over the energies
    where some spectrum is non-zero; with this choice the weights
    h(x,y) mu_i(E) / Z_i of any ray sum to at most one."""
    keep = I0.sum(axis=0) > 0
    return 2.0 * mu[:, keep].max(axis=1) * geom.box_diagonal()


def unrolled_phantom(seed, scale=1.0):
    """Seeded phantom of the unrolled-reconstruction workload: a water disk of
    radius 90 mm with two bone disks and one to three metal rods (diameter
    3-12 mm, titanium or steel) inside it; lengths scaled by `scale`."""
    rng = np.random.default_rng(seed)
    objs = [E(0, 0, 90 * scale, 90 * scale, "water", "air")]
    placed = []

    def spot(r):
        for _ in range(1000):
            rr = (70 * scale - r) * math.sqrt(rng.uniform())
            th = rng.uniform(0, 2 * math.pi)
            x, y = rr * math.cos(th), rr * math.sin(th)
            if all(math.hypot(x - a, y - b) > r + q + 2 * scale for a, b, q in placed):
                placed.append((x, y, r))
                return x, y
        raise RuntimeError("no room for the insert")

    for _ in range(2):
        r = 12 * scale
        x, y = spot(r)
        objs.append(E(x, y, r, r, "bone", "water"))
    for _ in range(int(rng.integers(1, 4))):
        r = 0.5 * rng.uniform(3, 12) * scale
        x, y = spot(r)
        objs.append(E(x, y, r, r, "titanium" if rng.uniform() < 0.5 else "steel", "water"))
    return MaterialPhantom(objs)


def unrolled_inputs(seed, name="fan256", i0=1e5):
    """One case of the unrolled-reconstruction workload on a fan-beam
    geometry: Poisson data of unrolled_phantom(seed), the metal mask, the
    cold start, Z, the truth in the basis and the non-metal voxels."""
    geom = geometry_for(name)
    I0 = spectra(i0)
    mu = basis_mu()
    scale = geom.nx * geom.dx / 256.0
    ph = unrolled_phantom(seed, scale)
    frac = metal_fraction(ph, geom, 4)
    metal = (frac >= 0.5).astype(np.uint8).reshape(-1)
    gbar = expected_counts(geom, ph, I0)
    rng = np.random.default_rng(seed)
    d = rng.poisson(gbar).astype(np.float32)
    return dict(name=name, geom=geom, I0=I0, mu=mu, d=d, gbar=gbar, metal=metal,
                t=0.5 * min(geom.dx, geom.dy), c0=cold_start(geom, I0), Z=surrogate_Z(geom, mu, I0),
                c_true=basis_image(ph, geom, I0), keep=(frac.reshape(-1) == 0).astype(np.float64),
                seed=seed)


def blob_inputs(name="fan256", seed_c=4, seed_true=40, i0=1e5, n_blobs=20):
    """Gradient workload: smooth positive basis images (Gaussian-blob sums).

    Returns the evaluation point c (blobs sampled at voxel centres, seed_c) and
    Poisson data of an independent blob phantom (seed_true), simulated from its
    closed-form line integrals."""
    geom = geometry_for(name)
    I0 = spectra(i0)
    mu = basis_mu()
    ph_c = random_blobs(seed_c, n_blobs, 100.0 * geom.nx / 256, geom)
    ph_t = random_blobs(seed_true, n_blobs, 100.0 * geom.nx / 256, geom)
    x, y = voxel_centres(geom)
    X = np.stack(np.meshgrid(x, y, indexing="xy"), axis=-1)
    c = ph_c.sample(X).reshape(-1, 2).T.copy()
    gbar = expected_counts(geom, ph_t, I0)
    rng = np.random.default_rng(seed_true)
    d = rng.poisson(gbar).astype(np.float32)
    return dict(name=name, geom=geom, I0=I0, mu=mu, c=c, d=d, gbar=gbar,
                Z=surrogate_Z(geom, mu, I0))
