"""GPU parity: every C-ABI call against the FP64 CPU oracle on the same seeded
inputs.  Each result is checked twice (tests/errors.py): relative L2 over the
whole array, and element-wise, max |x - x_o| relative to max |x_o|.  Bounds:
  mixed precision: projections, g and weights <= 1e-5; images after 20
                   iterations <= 1e-4; masks bit-exact;
  fp64:            <= 1e-10 (projections, weights, images).
"""
import numpy as np
import pytest
import torch

from workloads import make_inputs, geometry_for
from workloads import geometry as G
from tests.errors import rel_l2 as rel, rel_max, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda"


def odd_fan():
    """Non-square grid, anisotropic pixels, channel offset, odd sizes."""
    return G.Geometry(kind=0, nx=45, ny=37, nz=1, dx=1.1, dy=0.9, dz=1.0, n_views=37, n_rows=1,
                      n_cols=71, sid=300.0, sdd=560.0, dgamma=G.fan_dgamma(45, 37, 1.1, 0.9, 300.0, 71) * 1.05,
                      col_offset=0.25, drow_iso=1.0, beta0=0.3, views_per_rot=37.0, feed_per_rot=0.0)


def odd_helix():
    return G.Geometry(kind=1, nx=35, ny=29, nz=11, dx=1.0, dy=1.2, dz=0.9, n_views=50, n_rows=5,
                      n_cols=61, sid=250.0, sdd=480.0, dgamma=G.fan_dgamma(35, 29, 1.0, 1.2, 250.0, 61),
                      col_offset=-0.3, drow_iso=1.5, beta0=0.7, views_per_rot=24.0, feed_per_rot=4.0)


def wide_fan():
    """A 520 x 500 grid: enough 32 x 32 tiles (17 x 16) for the backprojector
    to take whole-CU tiles, with ragged tiles on two edges; 60 views.

    Mixed plans walk in FP32 grid coordinates relative to the grid corner, so
    a segment's split point carries an error of about the FP32 spacing at the
    coordinate (6e-5 pixel at 520).  The errors of a voxel's terms are
    independent, so a backprojection's relative error grows with the grid
    extent and falls with the square root of the views per voxel: about 7e-6
    here, against 7e-7 for 128 x 128 with 180 views."""
    return G.Geometry(kind=0, nx=520, ny=500, nz=1, dx=0.9, dy=0.95, dz=1.0, n_views=60, n_rows=1,
                      n_cols=601, sid=600.0, sdd=1100.0,
                      dgamma=G.fan_dgamma(520, 500, 0.9, 0.95, 600.0, 601), col_offset=0.25,
                      drow_iso=1.0, beta0=0.4, views_per_rot=60.0, feed_per_rot=0.0)


def axis_fan():
    """Degenerate rays: an odd channel count with no offset and views every
    45 degrees from 0, so the central channel runs exactly along an axis
    (slope 0, on a pixel boundary of the even grid) or exactly along a
    diagonal through pixel corners (slope 1)."""
    return G.Geometry(kind=0, nx=48, ny=48, nz=1, dx=1.0, dy=1.0, dz=1.0, n_views=8, n_rows=1,
                      n_cols=65, sid=200.0, sdd=400.0, dgamma=G.fan_dgamma(48, 48, 1.0, 1.0, 200.0, 65),
                      col_offset=0.0, drow_iso=1.0, beta0=0.0, views_per_rot=8.0, feed_per_rot=0.0)


GEOMS = {
    "fan64": lambda: geometry_for("fan64"),
    "fan128": lambda: geometry_for("fan128"),
    "wide_fan": wide_fan,
    "helical_small": lambda: geometry_for("helical_small"),
    "odd_fan": odd_fan,
    "odd_helix": odd_helix,
}


@pytest.fixture(scope="module")
def spectra():
    inp = make_inputs("fan64", with_data=False)
    return inp["I0"], inp["mu"]


def plan_for(g, spectra, prec):
    from paper_2202_00116_amd.plan import Plan
    return Plan(g, spectra[0], spectra[1], prec)


@pytest.mark.parametrize("gname", list(GEOMS))
@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
def test_forward(orc, spectra, gname, prec, tol):
    g = GEOMS[gname]()
    plan = plan_for(g, spectra, prec)
    rng = np.random.default_rng(1)
    c = rng.uniform(0.0, 1.0, (2, g.n_voxels))
    ref = orc.forward(g, c)
    l = plan.forward(torch.tensor(c, dtype=plan.dtype, device=DEV)).cpu().numpy()
    # the oracle is fed the values the GPU sees (rounded to the plan precision)
    ref = orc.forward(g, c.astype(np.float32).astype(np.float64)) if prec == "mixed" else ref
    assert_close(l, ref, tol, what=f"{gname} {prec} forward")
    l1 = plan.forward(torch.tensor(c[:1], dtype=plan.dtype, device=DEV)).cpu().numpy()
    assert_close(l1, ref[:1], tol, what=f"{gname} {prec} forward 1 ch")


@pytest.mark.parametrize("gname", list(GEOMS))
@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
@pytest.mark.parametrize("nch", [1, 2, 4])
def test_backproject(orc, spectra, gname, prec, tol, nch):
    g = GEOMS[gname]()
    plan = plan_for(g, spectra, prec)
    rng = np.random.default_rng(2)
    # non-negative weights (as the AM weights are): error relative to the result
    w = rng.uniform(0.0, 1.0, (nch, g.n_rays))
    if prec == "mixed":
        w = w.astype(np.float32).astype(np.float64)
    ref = orc.backproject(g, w)
    b = plan.backproject(torch.tensor(w, dtype=plan.dtype, device=DEV)).cpu().numpy()
    assert_close(b, ref, tol, what=f"{gname} {prec} {nch} ch backproject")
    # signed weights: the sums cancel, so the error is measured against H^T |w|
    ws = rng.standard_normal((nch, g.n_rays))
    if prec == "mixed":
        ws = ws.astype(np.float32).astype(np.float64)
    ref = orc.backproject(g, ws)
    scale = np.linalg.norm(orc.backproject(g, np.abs(ws)))
    b = plan.backproject(torch.tensor(ws, dtype=plan.dtype, device=DEV)).cpu().numpy()
    smax = np.abs(orc.backproject(g, np.abs(ws))).max()
    print(gname, prec, nch, "signed backproject err / |H^T|w||", np.linalg.norm(b - ref) / scale,
          "max err / max H^T|w|", np.abs(b - ref).max() / smax)
    assert np.linalg.norm(b - ref) <= tol * scale
    assert np.abs(b - ref).max() <= tol * smax


@pytest.mark.parametrize("gname", ["fan64", "helical_small", "odd_helix"])
def test_adjoint_identity_gpu(spectra, gname):
    g = GEOMS[gname]()
    plan = plan_for(g, spectra, "mixed")
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.uniform(0, 1, (2, g.n_voxels)), dtype=torch.float32, device=DEV)
    y = torch.tensor(rng.uniform(0, 1, (2, g.n_rays)), dtype=torch.float32, device=DEV)
    lhs = (plan.forward(x).double() * y.double()).sum().item()
    rhs = (x.double() * plan.backproject(y).double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
@pytest.mark.parametrize("mode", [0, 1])
def test_poly_mean(orc, prec, tol, mode):
    inp = make_inputs("fan64")
    g = inp["geom"]
    plan = plan_for(g, (inp["I0"], inp["mu"]), prec)
    rng = np.random.default_rng(4)
    l = orc.forward(g, inp["c0"] * rng.uniform(0.8, 1.2, inp["c0"].shape))
    if prec == "mixed":
        l = l.astype(np.float32).astype(np.float64)
    mask = (rng.random(g.n_rays) < 0.2).astype(np.uint8)
    w_o, g_o, obj_o = orc.poly_mean(inp["I0"], inp["mu"], l, inp["d"], mask, mode=mode)
    w, gg, obj = plan.poly_mean(torch.tensor(l, dtype=plan.dtype, device=DEV),
                                torch.tensor(inp["d"], device=DEV),
                                torch.tensor(mask, device=DEV), mode=mode, want_g=True,
                                want_obj=True)
    assert_close(gg.cpu().numpy(), g_o, tol, what=f"{prec} mode {mode} g")
    if mode == 1:
        # u_i = sum_j (d_j/g_j - 1) a_ij cancels where d ~ g (Poisson noise of
        # a few 1e-3), so the relative L2 bound is 10 tol, and the element-wise
        # error is measured against the scale of its terms, sum_j (d_j/g_j + 1) a_ij
        w_np = w.cpu().numpy()
        wa, _, _ = orc.poly_mean(inp["I0"], inp["mu"], l, inp["d"], mask, mode=0)
        scale = wa[:2] + wa[2:]
        em = np.abs(w_np - w_o).max() / np.abs(scale).max()
        print(prec, "GRAD weights rel L2", rel(w_np, w_o), "max err / max scale", em)
        assert rel(w_np, w_o) <= 10 * tol and em <= tol
    else:
        assert_close(w.cpu().numpy(), w_o, tol, what=f"{prec} mode {mode} weights")
    assert abs(obj.item() - obj_o.sum()) <= (1e-6 if prec == "mixed" else 1e-10) * abs(obj_o.sum())


@pytest.mark.parametrize("name", ["fan64", "fan128", "helical_small"])
def test_metal_trace_bit_exact(orc, name):
    inp = make_inputs(name, with_data=False)
    g = inp["geom"]
    mask_o, T_o = orc.metal_trace(g, inp["metal"], inp["t"])
    plan = plan_for(g, (inp["I0"], inp["mu"]), "mixed")
    mask, T = plan.metal_trace(torch.tensor(inp["metal"], device=DEV), inp["t"], want_T=True)
    T = T.cpu().numpy()
    margin = np.abs(T_o - inp["t"]).min()
    print(name, "trace margin", margin, "T err", np.abs(T - T_o).max())
    assert np.abs(T - T_o).max() < 1e-10
    assert np.array_equal(mask.cpu().numpy(), mask_o)
    assert mask_o.sum() > 0


@pytest.mark.parametrize("name,n", [("fan64", 20), ("fan128", 20), ("helical_small", 8)])
@pytest.mark.parametrize("prec,tol", [("mixed", 1e-4), ("fp64", 1e-10)])
def test_iterate(orc, name, n, prec, tol):
    inp = make_inputs(name)
    g = inp["geom"]
    mask_o, _ = orc.metal_trace(g, inp["metal"], inp["t"])
    c_o, h_o = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask_o, inp["Z"], inp["c0"], n)
    plan = plan_for(g, (inp["I0"], inp["mu"]), prec)
    c = torch.tensor(inp["c0"], device=DEV)
    hist = torch.zeros(n, dtype=torch.float64, device=DEV)
    plan.iterate(c, torch.tensor(inp["d"], device=DEV), torch.tensor(mask_o, device=DEV),
                 inp["Z"], n, hist)
    c = c.cpu().numpy()
    h = hist.cpu().numpy()
    print(name, prec, "hist rel", np.abs(h - h_o).max() / h_o[0])
    assert_close(c, c_o, tol, what=f"{name} {prec} image after {n} iterations")
    assert np.abs(h - h_o).max() <= (1e-5 if prec == "mixed" else 1e-9) * h_o[0]


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-4), ("fp64", 1e-10)])
def test_iterate_wide_fan(orc, prec, tol):
    """Whole-CU backprojector tiles with ragged edges through the iteration
    (the packed four-channel accumulation), against the oracle."""
    from workloads.configs import cold_start, expected_counts, surrogate_Z, unrolled_phantom
    from workloads.phantoms import metal_fraction
    from workloads.physics import basis_mu, spectra
    g = wide_fan()
    I0, mu = spectra(1e5), basis_mu()
    ph = unrolled_phantom(7, scale=2.0)
    d = np.random.default_rng(8).poisson(expected_counts(g, ph, I0)).astype(np.float32)
    metal = (metal_fraction(ph, g, 4) >= 0.5).astype(np.uint8).reshape(-1)
    mask_o, _ = orc.metal_trace(g, metal, 0.45)
    assert mask_o.sum() > 0
    c0, Z, n = cold_start(g, I0), surrogate_Z(g, mu, I0), 5
    c_o, h_o = orc.iterate(g, I0, mu, d, mask_o, Z, c0, n)
    plan = plan_for(g, (I0, mu), prec)
    c = torch.tensor(c0, device=DEV)
    hist = torch.zeros(n, dtype=torch.float64, device=DEV)
    plan.iterate(c, torch.tensor(d, device=DEV), torch.tensor(mask_o, device=DEV), Z, n, hist)
    c, h = c.cpu().numpy(), hist.cpu().numpy()
    print("wide_fan", prec, "hist rel", np.abs(h - h_o).max() / h_o[0])
    assert_close(c, c_o, tol, what=f"wide_fan {prec} image")
    assert np.abs(h - h_o).max() <= (1e-5 if prec == "mixed" else 1e-9) * h_o[0]


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
def test_degenerate_rays(orc, spectra, prec, tol):
    """Rays along the grid's central lines and diagonals.  A ray within
    rounding of a grid line may run in either adjacent row (the crossing of an
    almost parallel line is ill-conditioned), so what is compared is what does
    not depend on that choice: line integrals of an image that is symmetric
    about both central lines, backprojections away from the central rows and
    columns, sums of mirror pairs on them, and the adjoint identity (the
    forward and backward walks must choose alike)."""
    g = axis_fan()
    plan = plan_for(g, spectra, prec)
    rng = np.random.default_rng(41)
    img = rng.uniform(0, 1, (2, g.ny, g.nx))
    img = img + img[:, ::-1, :]
    img = img + img[:, :, ::-1]
    img = img.reshape(2, -1)
    if prec == "mixed":
        img = img.astype(np.float32).astype(np.float64)
    l = plan.forward(torch.tensor(img, dtype=plan.dtype, device=DEV)).cpu().numpy()
    assert_close(l, orc.forward(g, img), tol, what=f"axis_fan {prec} forward")
    w = rng.uniform(0, 1, (1, g.n_rays))
    if prec == "mixed":
        w = w.astype(np.float32).astype(np.float64)
    b = plan.backproject(torch.tensor(w, dtype=plan.dtype, device=DEV)).cpu().numpy()[0].reshape(g.ny, g.nx)
    b_o = orc.backproject(g, w)[0].reshape(g.ny, g.nx)
    hy, hx = g.ny // 2, g.nx // 2
    off = np.ones((g.ny, g.nx), bool)
    off[hy - 1:hy + 1, :] = False
    off[:, hx - 1:hx + 1] = False
    scale = np.abs(b_o).max()
    assert np.abs(b - b_o)[off].max() <= tol * 10 * scale
    # rows hy-1, hy in pairs (away from the central columns), columns hx-1, hx
    # in pairs (away from the central rows), and the 2 x 2 centre as a whole
    cols = np.r_[0:hx - 1, hx + 1:g.nx]
    rows = np.r_[0:hy - 1, hy + 1:g.ny]
    rp, rp_o = b[hy - 1:hy + 1, cols].sum(0), b_o[hy - 1:hy + 1, cols].sum(0)
    cp, cp_o = b[rows, hx - 1:hx + 1].sum(1), b_o[rows, hx - 1:hx + 1].sum(1)
    assert np.abs(rp - rp_o).max() <= tol * 10 * scale
    assert np.abs(cp - cp_o).max() <= tol * 10 * scale
    centre, centre_o = b[hy - 1:hy + 1, hx - 1:hx + 1].sum(), b_o[hy - 1:hy + 1, hx - 1:hx + 1].sum()
    assert abs(centre - centre_o) <= tol * 10 * scale
    x = torch.tensor(rng.uniform(0, 1, (1, g.n_voxels)), dtype=plan.dtype, device=DEV)
    y = torch.tensor(rng.uniform(0, 1, (1, g.n_rays)), dtype=plan.dtype, device=DEV)
    lhs = (plan.forward(x).double() * y.double()).sum().item()
    rhs = (x.double() * plan.backproject(y).double()).sum().item()
    assert abs(lhs - rhs) <= (1e-5 if prec == "mixed" else 1e-12) * abs(lhs)


def random_fan(seed):
    """A seeded 2D fan: grids of 3 to 90 pixels a side, anisotropic pixels, a
    random channel offset and start angle, few to many views and channels.
    Short chords, empty common interiors of a wave and chords that start or
    end on the wave's first or last plane all occur."""
    r = np.random.default_rng(seed)
    nx, ny = int(r.integers(3, 91)), int(r.integers(3, 91))
    dx, dy = float(r.uniform(0.5, 1.5)), float(r.uniform(0.5, 1.5))
    n_cols = int(r.integers(7, 200))
    n_views = int(r.integers(3, 40))
    rad = 0.5 * np.hypot(nx * dx, ny * dy)
    sid = float(r.uniform(1.5, 6.0)) * rad
    sdd = sid + rad * float(r.uniform(1.1, 3.0))      # the detector lies beyond the grid
    return G.Geometry(kind=0, nx=nx, ny=ny, nz=1, dx=dx, dy=dy, dz=1.0, n_views=n_views, n_rows=1,
                      n_cols=n_cols, sid=sid, sdd=sdd,
                      dgamma=G.fan_dgamma(nx, ny, dx, dy, sid, n_cols) * float(r.uniform(0.7, 1.2)),
                      col_offset=float(r.uniform(-0.5, 0.5)), drow_iso=1.0,
                      beta0=float(r.uniform(0, 2 * np.pi)), views_per_rot=float(r.uniform(n_views, 2 * n_views)),
                      feed_per_rot=0.0)


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
def test_random_fans(orc, spectra, prec, tol):
    """Forward and backprojection on 12 seeded random fans against the oracle."""
    for seed in range(200, 212):
        g = random_fan(seed)
        plan = plan_for(g, spectra, prec)
        rng = np.random.default_rng(seed)
        c = rng.uniform(0, 1, (2, g.n_voxels))
        w = rng.uniform(0, 1, (2, g.n_rays))
        if prec == "mixed":
            c = c.astype(np.float32).astype(np.float64)
            w = w.astype(np.float32).astype(np.float64)
        l = plan.forward(torch.tensor(c, dtype=plan.dtype, device=DEV)).cpu().numpy()
        b = plan.backproject(torch.tensor(w, dtype=plan.dtype, device=DEV)).cpu().numpy()
        tag = f"seed {seed} {g.nx}x{g.ny} {g.n_views}x{g.n_cols} {prec}"
        assert_close(l, orc.forward(g, c), tol, what=tag + " forward")
        assert_close(b, orc.backproject(g, w), tol, what=tag + " backproject")


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-4), ("fp64", 1e-10)])
def test_random_fans_iterate(orc, prec, tol):
    """Three DEAM iterations (the packed four-channel backprojection) on four
    seeded random fans, data from a phantom scaled to the grid, against the
    oracle."""
    from workloads.configs import cold_start, expected_counts, surrogate_Z, unrolled_phantom
    from workloads.phantoms import metal_fraction
    from workloads.physics import basis_mu, spectra as make_spectra
    I0, mu = make_spectra(1e5), basis_mu()
    for seed in range(220, 224):
        g = random_fan(seed)
        ph = unrolled_phantom(seed, scale=0.45 * min(g.nx * g.dx, g.ny * g.dy) / 90.0)
        d = np.random.default_rng(seed).poisson(expected_counts(g, ph, I0)).astype(np.float32)
        metal = (metal_fraction(ph, g, 4) >= 0.5).astype(np.uint8).reshape(-1)
        mask_o, _ = orc.metal_trace(g, metal, 0.5 * min(g.dx, g.dy))
        c0, Z, n = cold_start(g, I0), surrogate_Z(g, mu, I0), 3
        c_o, h_o = orc.iterate(g, I0, mu, d, mask_o, Z, c0, n)
        plan = plan_for(g, (I0, mu), prec)
        c = torch.tensor(c0, device=DEV)
        hist = torch.zeros(n, dtype=torch.float64, device=DEV)
        plan.iterate(c, torch.tensor(d, device=DEV), torch.tensor(mask_o, device=DEV), Z, n, hist)
        eh = float(np.abs(hist.cpu().numpy() - h_o).max() / h_o[0])
        tag = f"seed {seed} {g.nx}x{g.ny} {g.n_views}x{g.n_cols} {prec}"
        print(f"{tag}: objective {eh:.2e}, trace rays {int(mask_o.sum())}")
        assert_close(c.cpu().numpy(), c_o, tol, what=tag + " image")
        assert eh <= (1e-5 if prec == "mixed" else 1e-9), seed


def random_helix(seed):
    """A seeded helical scan: grids of 4 to 48 pixels a side and 2 to 14
    slices, 1 to 9 detector rows, a feed of up to a collimation per turn (or
    none), random offsets and start angle."""
    r = np.random.default_rng(seed)
    nx, ny, nz = int(r.integers(4, 49)), int(r.integers(4, 49)), int(r.integers(2, 15))
    dx, dy, dz = float(r.uniform(0.6, 1.4)), float(r.uniform(0.6, 1.4)), float(r.uniform(0.6, 1.6))
    n_rows, n_cols = int(r.integers(1, 10)), int(r.integers(9, 120))
    n_views = int(r.integers(8, 60))
    rad = 0.5 * np.hypot(nx * dx, ny * dy)
    sid = float(r.uniform(1.5, 6.0)) * rad
    sdd = sid + rad * float(r.uniform(1.1, 3.0))
    drow = float(r.uniform(0.5, 2.0))
    vpr = float(r.uniform(0.3 * n_views, n_views))
    feed = 0.0 if seed % 4 == 0 else float(r.uniform(0.2, 1.0)) * n_rows * drow
    return G.Geometry(kind=1, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, n_views=n_views,
                      n_rows=n_rows, n_cols=n_cols, sid=sid, sdd=sdd,
                      dgamma=G.fan_dgamma(nx, ny, dx, dy, sid, n_cols) * float(r.uniform(0.8, 1.2)),
                      col_offset=float(r.uniform(-0.5, 0.5)), drow_iso=drow,
                      beta0=float(r.uniform(0, 2 * np.pi)), views_per_rot=vpr, feed_per_rot=feed)


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
def test_random_helices(orc, spectra, prec, tol):
    """Forward and backprojection on 8 seeded random helical scans against
    the oracle."""
    for seed in range(300, 308):
        g = random_helix(seed)
        plan = plan_for(g, spectra, prec)
        rng = np.random.default_rng(seed)
        c = rng.uniform(0, 1, (2, g.n_voxels))
        w = rng.uniform(0, 1, (2, g.n_rays))
        if prec == "mixed":
            c = c.astype(np.float32).astype(np.float64)
            w = w.astype(np.float32).astype(np.float64)
        l = plan.forward(torch.tensor(c, dtype=plan.dtype, device=DEV)).cpu().numpy()
        b = plan.backproject(torch.tensor(w, dtype=plan.dtype, device=DEV)).cpu().numpy()
        tag = f"seed {seed} {g.nx}x{g.ny}x{g.nz} {g.n_views}x{g.n_rows}x{g.n_cols} {prec}"
        assert_close(l, orc.forward(g, c), tol, what=tag + " forward")
        assert_close(b, orc.backproject(g, w), tol, what=tag + " backproject")


def test_iterate_is_deterministic_and_resumable(spectra):
    inp = make_inputs("fan64")
    g = inp["geom"]
    plan = plan_for(g, (inp["I0"], inp["mu"]), "mixed")
    d = torch.tensor(inp["d"], device=DEV)
    c_a = torch.tensor(inp["c0"], device=DEV)
    plan.iterate(c_a, d, None, inp["Z"], 6)
    c_b = torch.tensor(inp["c0"], device=DEV)
    plan.iterate(c_b, d, None, inp["Z"], 3)
    plan.iterate(c_b, d, None, inp["Z"], 3)
    assert torch.equal(c_a, c_b)
    w = torch.rand((4, g.n_rays), device=DEV)
    assert torch.equal(plan.backproject(w), plan.backproject(w))


def test_update(orc, spectra):
    g = geometry_for("fan64")
    plan = plan_for(g, spectra, "fp64")
    rng = np.random.default_rng(6)
    b = rng.uniform(0.5, 2.0, (4, g.n_voxels))
    b[0, :10] = 0.0
    b[3, 20:30] = 0.0
    c = rng.standard_normal((2, g.n_voxels))
    Z = np.array([7.0, 30.0])
    ref = orc.update(b, Z, c)
    ct = torch.tensor(c, device=DEV)
    plan.update(ct, torch.tensor(b, device=DEV), Z)
    assert np.abs(ct.cpu().numpy() - ref).max() < 1e-14
