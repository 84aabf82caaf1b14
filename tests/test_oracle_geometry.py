"""Pins of the oracle's system operator h(x,y) (Section 2.3, Eq. 8) against
closed forms and brute force that share no code with it."""
import math

import numpy as np
import pytest

from workloads import geometry as G
from workloads.geometry import ray_endpoints
from tests.bruteforce import ray_row, box_chord, disk_chord


def small_fan(nx=8, ny=8, dx=1.0, dy=1.0):
    return G.Geometry(kind=0, nx=nx, ny=ny, nz=1, dx=dx, dy=dy, dz=1.0, n_views=8, n_rows=1,
                      n_cols=16, sid=20.0, sdd=40.0, dgamma=0.05, col_offset=0.0, drow_iso=1.0,
                      beta0=0.1, views_per_rot=8.0, feed_per_rot=0.0)


def small_box3d():
    return G.Geometry(kind=1, nx=6, ny=5, nz=4, dx=1.0, dy=1.2, dz=0.8, n_views=8, n_rows=3,
                      n_cols=16, sid=20.0, sdd=40.0, dgamma=0.05, col_offset=0.0, drow_iso=1.0,
                      beta0=0.1, views_per_rot=8.0, feed_per_rot=2.0)


def random_rays(rng, n, is3d, radius=15.0):
    out = []
    for _ in range(n):
        a = rng.uniform(0, 2 * np.pi)
        b = a + np.pi + rng.uniform(-0.6, 0.6)
        S = np.array([radius * math.cos(a), radius * math.sin(a), rng.uniform(-3, 3) if is3d else 0.0])
        P = np.array([radius * math.cos(b), radius * math.sin(b), rng.uniform(-3, 3) if is3d else 0.0])
        out.append((S, P))
    return out


def dense_from_siddon(orc, g, S, P):
    idx, ln = orc.siddon(g, S, P)
    row = np.zeros(g.n_voxels)
    np.add.at(row, idx, ln)
    return row


@pytest.mark.parametrize("geom_fn", [small_fan, lambda: small_fan(7, 5, 1.3, 0.7), small_box3d])
def test_siddon_matches_voxelwise_clipping(orc, geom_fn):
    """T1: each h(x,y) equals the segment length inside the closed voxel box."""
    g = geom_fn()
    rng = np.random.default_rng(0)
    rays = random_rays(rng, 40, g.kind == 1)
    # axis-parallel rays (off the grid planes)
    rays += [(np.array([0.31, -15.0, 0.2]), np.array([0.31, 15.0, 0.2])),
             (np.array([-15.0, -1.77, -0.4]), np.array([15.0, -1.77, -0.4]))]
    # diagonal rays through grid corners (coincident x and y crossings)
    # (z = 0.13 keeps the 3D variants off the z planes: a ray lying in a grid
    # plane is assigned to one side by the midpoint rule, while closed boxes
    # would count it on both)
    rays += [(np.array([-10.0, -10.0, 0.13]), np.array([10.0, 10.0, 0.13])),
             (np.array([-10.0, 11.0, 0.13]), np.array([11.0, -10.0, 0.13]))]
    for S, P in rays:
        ref = ray_row(g, S, P)
        got = dense_from_siddon(orc, g, S, P)
        assert np.allclose(got, ref, rtol=0, atol=1e-12), (S, P)


def test_siddon_z_parallel_ray(orc):
    g = small_box3d()
    S, P = np.array([0.3, 0.45, -10.0]), np.array([0.3, 0.45, 10.0])
    ref = ray_row(g, S, P)
    got = dense_from_siddon(orc, g, S, P)
    assert np.allclose(got, ref, atol=1e-12)
    assert abs(got.sum() - g.nz * g.dz) < 1e-12


@pytest.mark.parametrize("name", ["fan64", "helical_small"])
def test_row_sum_is_box_chord(orc, name):
    """T2: sum_x h(x,y) is the length of the ray inside the grid box."""
    from workloads import geometry_for
    g = geometry_for(name)
    ones = np.ones(g.n_voxels)
    l = orc.forward(g, ones)[0]
    S, P = ray_endpoints(g)
    ref = np.array([box_chord(g, S[i], P[i]) for i in range(g.n_rays)])
    assert np.abs(l - ref).max() < 1e-10


def offset_fan():
    """Anisotropic pixels, a channel offset and a start angle (all conventions exercised)."""
    return G.Geometry(kind=0, nx=40, ny=30, nz=1, dx=1.2, dy=0.8, dz=1.0, n_views=30, n_rows=1,
                      n_cols=64, sid=200.0, sdd=380.0, dgamma=G.fan_dgamma(40, 30, 1.2, 0.8, 200.0, 64) * 1.1,
                      col_offset=0.37, drow_iso=1.0, beta0=0.41, views_per_rot=30.0, feed_per_rot=0.0)


@pytest.mark.parametrize("name,cx,cy,R", [("fan128", 17.3, -9.1, 21.0), ("fan64", -5.0, 8.0, 9.5),
                                          ("offset", 6.1, -3.3, 7.0)])
def test_pixelised_disk_chord_bracket(orc, name, cx, cy, R):
    """T3: the pixelised disk (pixel on iff its centre is inside) lies between
    the disks of radius R-a and R+a, a = half pixel diagonal, so its projection
    is bracketed by the closed-form chords of those disks.  The rays come from
    the workload geometry (an independent numpy implementation), which also
    pins the source/detector conventions."""
    from workloads import geometry_for
    g = offset_fan() if name == "offset" else geometry_for(name)
    x = (np.arange(g.nx) + 0.5) * g.dx - g.nx * g.dx / 2
    y = (np.arange(g.ny) + 0.5) * g.dy - g.ny * g.dy / 2
    img = (((x[None, :] - cx) ** 2 + (y[:, None] - cy) ** 2) <= R * R).astype(np.float64)
    l = orc.forward(g, img.reshape(-1))[0]
    S, P = ray_endpoints(g)
    a = 0.5 * math.hypot(g.dx, g.dy)
    lo = disk_chord(S, P, cx, cy, R - a)
    hi = disk_chord(S, P, cx, cy, R + a)
    assert np.all(l >= lo - 1e-9) and np.all(l <= hi + 1e-9)
    # and the bracket is informative: most rays through the disk are strictly inside it
    assert (l > 0).sum() > 0.1 * g.n_rays


def test_helical_cylinder_chord_bracket(orc):
    """T3 in 3D: a z-aligned voxelised cylinder spanning all slices."""
    from workloads import geometry_for
    g = geometry_for("helical_small")
    cx, cy, R = 3.0, -4.0, 11.0
    x = (np.arange(g.nx) + 0.5) * g.dx - g.nx * g.dx / 2
    y = (np.arange(g.ny) + 0.5) * g.dy - g.ny * g.dy / 2
    disk = (((x[None, :] - cx) ** 2 + (y[:, None] - cy) ** 2) <= R * R).astype(np.float64)
    img = np.broadcast_to(disk, (g.nz,) + disk.shape).reshape(-1)
    l = orc.forward(g, img)[0]
    S, P = ray_endpoints(g)
    a = 0.5 * math.hypot(g.dx, g.dy)
    zl, zh = -g.nz * g.dz / 2, g.nz * g.dz / 2
    lo = disk_chord(S, P, cx, cy, R - a, zl, zh)
    hi = disk_chord(S, P, cx, cy, R + a, zl, zh)
    assert np.all(l >= lo - 1e-9) and np.all(l <= hi + 1e-9)
    assert (l > 0).sum() > 0.1 * g.n_rays


def test_rot90_shifts_views(orc):
    """T4: np.rot90 maps f to f(R x) with R the +90 degree rotation, so the
    sinogram of the rotated image is the original shifted by a quarter turn."""
    from workloads import geometry_for
    g = geometry_for("fan64")
    assert g.n_views % 4 == 0
    rng = np.random.default_rng(3)
    img = rng.random((g.ny, g.nx))
    s0 = orc.forward(g, img.reshape(-1))[0].reshape(g.n_views, g.n_cols)
    s1 = orc.forward(g, np.rot90(img).copy().reshape(-1))[0].reshape(g.n_views, g.n_cols)
    assert np.abs(s1 - np.roll(s0, -g.n_views // 4, axis=0)).max() < 1e-10 * np.abs(s0).max()


@pytest.mark.parametrize("name", ["fan64", "helical_small"])
def test_adjoint_identity(orc, name):
    """T5: <H x, y> = <x, H^T y> for random x, y (the backprojector is the
    transpose of the forward projector)."""
    from workloads import geometry_for
    g = geometry_for(name)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, g.n_voxels))
    y = rng.standard_normal((2, g.n_rays))
    lhs = np.sum(orc.forward(g, x) * y)
    rhs = np.sum(x * orc.backproject(g, y))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(orc.forward(g, np.abs(x))).sum() * np.abs(y).max())


@pytest.mark.parametrize("geom_fn", [small_fan, small_box3d])
def test_backprojection_matches_dense_transpose(orc, geom_fn):
    """The oracle backprojector equals the transpose of the brute-force dense H
    (2D fan and a 3D helical box)."""
    g = geom_fn()
    S, P = ray_endpoints(g)
    H = np.stack([ray_row(g, S[i], P[i]) for i in range(g.n_rays)])
    rng = np.random.default_rng(7)
    w = rng.standard_normal(g.n_rays)
    assert np.allclose(orc.backproject(g, w)[0], H.T @ w, atol=1e-11)
    c = rng.standard_normal(g.n_voxels)
    assert np.allclose(orc.forward(g, c)[0], H @ c, atol=1e-11)


@pytest.mark.parametrize("name", ["fan64", "helical_small"])
def test_forward_rays_equals_forward(orc, name):
    """The sampled-ray projector (the reference of the full-size checks) returns,
    bit for bit, the selected columns of the whole-sinogram projection, for a
    ray list in arbitrary order with repeats and both ends of the range."""
    from workloads import geometry_for
    g = geometry_for(name)
    rng = np.random.default_rng(17)
    img = rng.standard_normal((2, g.n_voxels))
    full = orc.forward(g, img)
    rays = np.concatenate([[g.n_rays - 1, 0], rng.integers(0, g.n_rays, 500), [7, 7]])
    sel = orc.forward_rays(g, img, rays)
    assert sel.shape == (2, rays.size)
    assert np.array_equal(sel, full[:, rays])
