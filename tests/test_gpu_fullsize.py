"""Parity at the benchmark sizes, with the launch configuration bench.py times.

fan512 (2D, 512^2, 984 x 816 rays): the oracle runs the whole problem: metal
mask (bit-exact), forward projection, backprojection, two full DEAM iterations
and the 20 iterations of the stated image tolerance.  helical (512^2 x 64, 4608 x 16 x 816 rays): the oracle computes
sampled rays one by one (line integrals, metal trace, expected counts);
properties that hold at any size (adjoint identity, monotone objective) cover
the rest."""
import numpy as np
import pytest
import torch

from workloads import make_inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
DEV = "cuda"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) / np.linalg.norm(np.asarray(b, float)))


@pytest.fixture(scope="module")
def fan512():
    return make_inputs("fan512")


@pytest.fixture(scope="module")
def helical():
    return make_inputs("helical")


def test_fan512_full(orc, fan512):
    from paper_2202_00116_amd.plan import Plan
    inp = fan512
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], "mixed")
    mask_o, T_o = orc.metal_trace(g, inp["metal"], inp["t"])
    mask, T = plan.metal_trace(torch.tensor(inp["metal"], device=DEV), inp["t"], want_T=True)
    assert np.array_equal(mask.cpu().numpy(), mask_o)
    assert np.abs(T.cpu().numpy() - T_o).max() < 1e-9
    print("fan512 trace margin", np.abs(T_o - inp["t"]).min(), "metal rays", int(mask_o.sum()))
    # forward projection of the starting image
    c32 = inp["c0"].astype(np.float32).astype(np.float64)
    l_o = orc.forward(g, c32)
    l = plan.forward(torch.tensor(c32, dtype=torch.float32, device=DEV)).cpu().numpy()
    print("fan512 forward rel", rel(l, l_o))
    assert rel(l, l_o) <= 1e-5
    # backprojection of non-negative weights
    rng = np.random.default_rng(21)
    w = rng.uniform(0, 1, (4, g.n_rays)).astype(np.float32).astype(np.float64)
    b_o = orc.backproject(g, w)
    b = plan.backproject(torch.tensor(w, dtype=torch.float32, device=DEV)).cpu().numpy()
    print("fan512 backproject rel", rel(b, b_o))
    assert rel(b, b_o) <= 1e-5
    # two DEAM iterations from the cold start, with the objective history
    c_o, h_o = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask_o, inp["Z"], inp["c0"], 2)
    c = torch.tensor(inp["c0"], device=DEV)
    hist = torch.zeros(2, dtype=torch.float64, device=DEV)
    plan.iterate(c, torch.tensor(inp["d"], device=DEV), mask, inp["Z"], 2, hist)
    print("fan512 2-iteration image rel", rel(c.cpu().numpy(), c_o))
    assert rel(c.cpu().numpy(), c_o) <= 1e-5
    assert np.abs(hist.cpu().numpy() - h_o).max() <= 1e-6 * h_o[0]


def test_fan512_20_iterations_against_oracle(orc, fan512):
    """The stated image tolerance at the benchmark size: 20 DEAM iterations
    from the cold start, both GPU precisions against the oracle's 20
    iterations on the same inputs (image and objective history)."""
    from paper_2202_00116_amd.plan import Plan
    inp = fan512
    g = inp["geom"]
    n = 20
    mask_o, _ = orc.metal_trace(g, inp["metal"], inp["t"])
    c_o, h_o = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask_o, inp["Z"], inp["c0"], n)
    d = torch.tensor(inp["d"], device=DEV)
    mask = torch.tensor(mask_o, device=DEV)
    for prec, tol, htol in (("mixed", 1e-4, 1e-5), ("fp64", 1e-10, 1e-10)):
        plan = Plan(g, inp["I0"], inp["mu"], prec)
        c = torch.tensor(inp["c0"], device=DEV)
        hist = torch.zeros(n, dtype=torch.float64, device=DEV)
        plan.iterate(c, d, mask, inp["Z"], n, hist)
        e = rel(c.cpu().numpy(), c_o)
        eh = float(np.abs(hist.cpu().numpy() - h_o).max() / h_o[0])
        print(f"fan512 {prec} 20 iterations: image rel {e:.3e}, objective rel {eh:.3e}")
        assert e <= tol and eh <= htol


def test_fan512_objective_monotone_50_iterations(fan512):
    """The masked I-divergence never increases over the workload's 50
    iterations (mixed precision, bench configuration)."""
    from paper_2202_00116_amd.plan import Plan
    inp = fan512
    plan = Plan(inp["geom"], inp["I0"], inp["mu"], "mixed")
    mask = plan.metal_trace(torch.tensor(inp["metal"], device=DEV), inp["t"])
    c = torch.tensor(inp["c0"], device=DEV)
    hist = torch.zeros(50, dtype=torch.float64, device=DEV)
    plan.iterate(c, torch.tensor(inp["d"], device=DEV), mask, inp["Z"], 50, hist)
    h = hist.cpu().numpy()
    assert np.all(np.diff(h) <= 1e-7 * h[:-1]), h
    assert h[-1] < 0.2 * h[0]


def test_fan512_mixed_tracks_fp64_over_50_iterations(fan512):
    """Mixed precision against the all-FP64 GPU path (itself checked against
    the oracle) after the workload's 50 iterations."""
    from paper_2202_00116_amd.plan import Plan
    inp = fan512
    d = torch.tensor(inp["d"], device=DEV)
    out = {}
    for prec in ("mixed", "fp64"):
        plan = Plan(inp["geom"], inp["I0"], inp["mu"], prec)
        mask = plan.metal_trace(torch.tensor(inp["metal"], device=DEV), inp["t"])
        c = torch.tensor(inp["c0"], device=DEV)
        plan.iterate(c, d, mask, inp["Z"], 50)
        out[prec] = c.cpu().numpy()
    print("fan512 50 iterations mixed vs fp64", rel(out["mixed"], out["fp64"]))
    assert rel(out["mixed"], out["fp64"]) <= 1e-4


def test_helical_sampled(orc, helical):
    from paper_2202_00116_amd.plan import Plan
    inp = helical
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], "mixed")
    rng = np.random.default_rng(31)
    rays = np.sort(rng.choice(g.n_rays, 4000, replace=False))
    rays_t = torch.tensor(rays, device=DEV)
    # metal trace on sampled rays (FP64 both sides)
    mask, T = plan.metal_trace(torch.tensor(inp["metal"], device=DEV), inp["t"], want_T=True)
    T_o = orc.forward_rays(g, inp["metal"].astype(np.float64), rays)[0]
    assert np.abs(T[rays_t].cpu().numpy() - T_o).max() < 1e-9
    assert np.array_equal(mask[rays_t].cpu().numpy(), (T_o >= inp["t"]).astype(np.uint8))
    assert int(mask.sum().item()) > 0
    # line integrals of a random image on sampled rays
    c = rng.uniform(0, 1, (2, g.n_voxels)).astype(np.float32)
    l = plan.forward(torch.tensor(c, device=DEV))[:, rays_t].cpu().numpy()
    l_o = orc.forward_rays(g, c.astype(np.float64), rays)
    print("helical sampled forward rel", rel(l, l_o))
    assert rel(l, l_o) <= 1e-5
    # expected counts and weights on the sampled rays, from the GPU's line integrals
    lt = plan.forward(torch.tensor(inp["c0"], dtype=torch.float32, device=DEV))
    d = torch.tensor(inp["d"], device=DEV)
    w, gg, _ = plan.poly_mean(lt, d, mask, want_g=True)
    w_o, g_o, _ = orc.poly_mean(inp["I0"], inp["mu"], lt[:, rays_t].double().cpu().numpy(),
                                inp["d"][:, rays], mask[rays_t].cpu().numpy())
    assert rel(gg[:, rays_t].cpu().numpy(), g_o) <= 1e-5
    assert rel(w[:, rays_t].cpu().numpy(), w_o) <= 1e-5


def test_helical_adjoint_and_monotone(helical):
    from paper_2202_00116_amd.plan import Plan
    inp = helical
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], "mixed")
    rng = np.random.default_rng(32)
    x = torch.tensor(rng.uniform(0, 1, (2, g.n_voxels)), dtype=torch.float32, device=DEV)
    y = torch.tensor(rng.uniform(0, 1, (2, g.n_rays)), dtype=torch.float32, device=DEV)
    lhs = (plan.forward(x).double() * y.double()).sum().item()
    rhs = (x.double() * plan.backproject(y).double()).sum().item()
    print("helical adjoint", abs(lhs - rhs) / abs(lhs))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # the same with data only on views where the slabs' irradiation windows
    # open and close (the scan's ends and a block in the middle): rays that
    # the backprojector's view culling dropped wrongly would be a large share
    # of this product
    yv = y.view(2, g.n_views, -1).clone()
    keep = torch.zeros(g.n_views, dtype=torch.bool, device=DEV)
    keep[:256] = True
    keep[-256:] = True
    keep[g.n_views // 2 - 64:g.n_views // 2 + 64] = True
    yv[:, ~keep] = 0
    yv = yv.view(2, -1)
    lhs = (plan.forward(x).double() * yv.double()).sum().item()
    rhs = (x.double() * plan.backproject(yv).double()).sum().item()
    print("helical adjoint (window-edge views)", abs(lhs - rhs) / abs(lhs))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    mask = plan.metal_trace(torch.tensor(inp["metal"], device=DEV), inp["t"])
    c = torch.tensor(inp["c0"], device=DEV)
    hist = torch.zeros(4, dtype=torch.float64, device=DEV)
    plan.iterate(c, torch.tensor(inp["d"], device=DEV), mask, inp["Z"], 4, hist)
    h = hist.cpu().numpy()
    assert np.all(np.diff(h) <= 1e-7 * h[:-1]), h
