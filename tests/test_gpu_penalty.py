"""Penalised DEAM on the GPU (Eqs. 6-7): the penalty value, the penalised
c-step (FP64 Newton) against the oracle's bisection on identical inputs, the
penalised iteration against the oracle, the objective's decrease, and a
sampled check at the full helical size in the benchmark's launch
configuration."""
import numpy as np
import pytest
import torch

from workloads import make_inputs, PENALTY
from workloads import geometry as Gw
from tests.errors import rel_l2, rel_max

pytestmark = pytest.mark.gpu
DEV = "cuda"


def rel(a, b):
    """The larger of the relative L2 error and the element-wise error (max-abs
    relative to max |b|): a bound on it bounds both."""
    return max(rel_l2(a, b), rel_max(a, b))


def _plan(g, inp, prec):
    from paper_2202_00116_amd.plan import Plan
    return Plan(g, inp["I0"], inp["mu"], prec)


def ragged_fan():
    """A 2D grid that is not a multiple of the 32 x 32 update tile."""
    return Gw.Geometry(kind=0, nx=45, ny=37, nz=1, dx=0.9, dy=1.1, dz=1.0, n_views=16, n_rows=1,
                       n_cols=96, sid=300.0, sdd=600.0, dgamma=0.004, col_offset=0.25,
                       drow_iso=1.0, beta0=0.0, views_per_rot=16.0, feed_per_rot=0.0)


def ragged_box():
    """A 3D grid with ragged x/y tiles and anisotropic voxels."""
    return Gw.Geometry(kind=1, nx=40, ny=33, nz=5, dx=1.0, dy=0.8, dz=1.5, n_views=16, n_rows=4,
                       n_cols=64, sid=300.0, sdd=600.0, dgamma=0.006, col_offset=0.0,
                       drow_iso=1.0, beta0=0.0, views_per_rot=16.0, feed_per_rot=4.0)


def _synthetic(g, seed, skip=True):
    """Smooth-plus-noise iterate and positive backprojections of realistic size."""
    rng = np.random.default_rng(seed)
    V = g.n_voxels
    ix = np.arange(V) % g.nx
    base = 0.5 + 0.3 * np.sin(ix / 5.0)
    c = np.stack([base + 0.02 * rng.standard_normal(V), 0.04 + 0.01 * rng.standard_normal(V)])
    b = rng.uniform(5e4, 2e5, (4, V))
    if skip:
        b[0, rng.uniform(size=V) < 0.05] = 0.0
        b[3, rng.uniform(size=V) < 0.05] = -1.0
    return c, b


@pytest.mark.parametrize("geo", ["fan64", "helical_small", "ragged_fan", "ragged_box"])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_update_penalized_matches_oracle(orc, geo, prec):
    inp = make_inputs("fan64", with_data=False)
    g = {"ragged_fan": ragged_fan, "ragged_box": ragged_box}.get(geo, lambda: Gw_geom(geo))()
    plan = _plan(g, inp, prec)
    c, b = _synthetic(g, 81)
    dt = torch.float32 if prec == "mixed" else torch.float64
    bt = torch.tensor(b, dtype=dt, device=DEV)
    b_used = bt.cpu().numpy().astype(np.float64)          # what the kernel reads
    Z = inp["Z"]
    for lam, delta in ((0.0, 0.01), (2e4, 0.01), (3e5, 0.002)):
        ref = orc.update_pen(g, b_used, Z, lam, delta, c)
        out, cp = plan.update_penalized(torch.tensor(c, device=DEV), bt, Z, lam, delta, want_proj=True)
        out = out.cpu().numpy()
        err = np.abs(out - ref).max()
        print(f"{geo} {prec} lam={lam:g}: max |gpu - oracle| = {err:.3e}")
        assert err <= 1e-12 * np.abs(ref).max()
        assert np.array_equal(cp.cpu().numpy(), out.astype(cp.cpu().numpy().dtype))
        skip = ~((b_used[:2] > 0) & (b_used[2:] > 0))
        assert np.array_equal(out[skip], c[skip])


def Gw_geom(name):
    from workloads.configs import geometry_for
    return geometry_for(name)


def test_update_penalized_lambda_zero_matches_update():
    inp = make_inputs("fan64", with_data=False)
    g = inp["geom"]
    plan = _plan(g, inp, "fp64")
    c, b = _synthetic(g, 82)
    ct = torch.tensor(c, device=DEV)
    bt = torch.tensor(b, device=DEV)
    ref = ct.clone()
    plan.update(ref, bt, inp["Z"])
    out = plan.update_penalized(ct, bt, inp["Z"], 0.0, 0.01)
    # Newton stops after a step below 1e-13 (|c| + 1e-3): the same bound as against the oracle
    assert (out - ref).abs().max().item() <= 1e-12 * ref.abs().max().item()


@pytest.mark.parametrize("geo", ["fan64", "helical_small", "ragged_box"])
def test_penalty_value_matches_oracle(orc, geo):
    inp = make_inputs("fan64", with_data=False)
    g = ragged_box() if geo == "ragged_box" else Gw_geom(geo)
    c, _ = _synthetic(g, 83)
    for prec in ("mixed", "fp64"):
        plan = _plan(g, inp, prec)
        for lam, delta in ((1.0, 0.01), (7e3, 0.002)):
            got = plan.penalty(torch.tensor(c, device=DEV), lam, delta).item()
            ref = orc.penalty(g, c, lam, delta)
            assert got == pytest.approx(ref, rel=1e-12)


def test_penalized_entry_points_reject_bad_arguments():
    from paper_2202_00116_amd._lib import DeamError
    inp = make_inputs("fan64", with_data=False)
    g = inp["geom"]
    plan = _plan(g, inp, "mixed")
    c = torch.zeros((2, g.n_voxels), dtype=torch.float64, device=DEV)
    b = torch.ones((4, g.n_voxels), dtype=torch.float32, device=DEV)
    for lam, delta in ((-1.0, 0.01), (1.0, 0.0), (float("nan"), 0.01), (1.0, float("inf"))):
        with pytest.raises(DeamError, match="VALUE"):
            plan.update_penalized(c, b, inp["Z"], lam, delta)
        with pytest.raises(DeamError, match="VALUE"):
            plan.penalty(c, lam, delta)
    # output overlapping the input iterate
    import ctypes as C
    from paper_2202_00116_amd import _lib as L
    Zh = np.ascontiguousarray(inp["Z"], dtype=np.float64)
    rc = plan.lib.deam_update_penalized(plan._p, C.c_void_p(c.data_ptr()), C.c_void_p(c.data_ptr() + 8),
                                        None, C.c_void_p(b.data_ptr()), Zh.ctypes.data_as(C.c_void_p),
                                        1.0, 0.01, None)
    assert rc == -7


@pytest.mark.parametrize("name,prec,n,tol", [("fan64", "fp64", 8, 1e-9), ("fan64", "mixed", 20, 1e-4),
                                             ("helical_small", "fp64", 3, 1e-9),
                                             ("helical_small", "mixed", 10, 1e-4)])
def test_iterate_penalized_matches_oracle(orc, name, prec, n, tol):
    inp = make_inputs(name)
    g = inp["geom"]
    lam, delta = PENALTY[name]
    plan = _plan(g, inp, prec)
    mask_o = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    ref, href = orc.iterate_pen(g, inp["I0"], inp["mu"], inp["d"], mask_o, inp["Z"], lam, delta,
                                inp["c0"], n)
    c = torch.tensor(inp["c0"], device=DEV)
    h = torch.zeros(n, dtype=torch.float64, device=DEV)
    plan.iterate_penalized(c, torch.tensor(inp["d"], device=DEV), torch.tensor(mask_o, device=DEV),
                           inp["Z"], lam, delta, n, h)
    e = rel(c.cpu().numpy(), ref)
    eh = np.abs(h.cpu().numpy() - href).max() / abs(href[0])
    print(f"{name} {prec} {n} it.: image rel {e:.3e}, objective rel {eh:.3e}")
    assert e <= tol
    assert eh <= (1e-12 if prec == "fp64" else 1e-6)
    # the penalty acts: the result differs from the unpenalised iterate
    cu, _ = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask_o, inp["Z"], inp["c0"], n)
    assert rel(ref, cu) > 10 * tol


def test_fp64_penalized_objective_decreases():
    inp = make_inputs("fan64")
    g = inp["geom"]
    plan = _plan(g, inp, "fp64")
    M = torch.tensor(inp["metal"], device=DEV)
    mask = plan.metal_trace(M, inp["t"])
    d = torch.tensor(inp["d"], device=DEV)
    for lam, delta in (PENALTY["fan64"], (3e5, 0.02)):
        c = torch.tensor(inp["c0"], device=DEV)
        h = torch.zeros(12, dtype=torch.float64, device=DEV)
        plan.iterate_penalized(c, d, mask, inp["Z"], lam, delta, 12, h)
        h = h.cpu().numpy()
        assert np.all(np.diff(h) < 0), h


def test_iterate_penalized_lambda_zero_matches_iterate():
    inp = make_inputs("fan64")
    g = inp["geom"]
    plan = _plan(g, inp, "fp64")
    d = torch.tensor(inp["d"], device=DEV)
    a = torch.tensor(inp["c0"], device=DEV)
    b = a.clone()
    plan.iterate(a, d, None, inp["Z"], 4)
    plan.iterate_penalized(b, d, None, inp["Z"], 0.0, 0.01, 4)
    assert (a - b).abs().max().item() <= 1e-12 * a.abs().max().item()


def test_update_penalized_full_helical_sampled(orc):
    """The 512 x 512 x 64 helical grid in the benchmark's launch configuration
    (mixed plan): sampled voxels (random, faces, edges, corners) against the
    oracle's per-voxel c-step on the same synthetic iterate and backprojections."""
    from workloads.configs import geometry_for
    g = geometry_for("helical")
    inp = make_inputs("fan64", with_data=False)
    lam, delta = PENALTY["helical"]
    plan = _plan(g, inp, "mixed")
    rng = np.random.default_rng(84)
    V = g.n_voxels
    c, b = _synthetic(g, 85)
    bt = torch.tensor(b, dtype=torch.float32, device=DEV)
    b_used = bt.cpu().numpy().astype(np.float64)
    out = plan.update_penalized(torch.tensor(c, device=DEV), bt, inp["Z"], lam, delta).cpu().numpy()
    nx, ny, nz = g.nx, g.ny, g.nz
    corners = [((z * ny) + y) * nx + x for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
    edges = [((z * ny) + y) * nx + x for z in (0, nz // 2, nz - 1) for y in (0, 31, 32, ny - 1)
             for x in (0, 31, 32, 255, nx - 1)]
    sel = np.unique(np.concatenate([rng.choice(V, 20000, replace=False), corners, edges]))
    ref = orc.update_pen_voxels(g, b_used, inp["Z"], lam, delta, c, sel)
    err = np.abs(out[:, sel] - ref).max()
    print(f"helical full size: {len(sel)} sampled voxels, max |gpu - oracle| = {err:.3e}")
    assert err <= 1e-12 * np.abs(ref).max()
    moved = np.abs(out[:, sel] - orc.update(b_used[:, sel], inp["Z"], c[:, sel])).max()
    assert moved > 1e-6
