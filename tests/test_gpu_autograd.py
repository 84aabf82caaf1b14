"""Hand-written adjoint of the Poisson NLL (and of c -> g) behind
torch.autograd.Function, checked against the FP64 oracle gradient and against
FP64 central finite differences (h = 1e-3)."""
import numpy as np
import pytest
import torch

from workloads import blob_inputs, make_inputs
from tests.errors import rel_l2, rel_max

pytestmark = pytest.mark.gpu
DEV = "cuda"


def rel(a, b):
    """The larger of the relative L2 error and the element-wise error (max-abs
    relative to max |b|): a bound on it bounds both."""
    return max(rel_l2(a, b), rel_max(a, b))


@pytest.fixture(scope="module")
def blobs():
    return blob_inputs("fan256")


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-4), ("fp64", 1e-10)])
def test_nll_gradient_matches_oracle(orc, blobs, prec, tol):
    from paper_2202_00116_amd.plan import Plan
    from paper_2202_00116_amd.autograd import DEAMNLL
    inp = blobs
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], prec)
    c_np = inp["c"] if prec == "fp64" else inp["c"].astype(np.float32).astype(np.float64)
    L_o, grad_o = orc.nll_grad(g, inp["I0"], inp["mu"], inp["d"], None, c_np)
    c = torch.tensor(c_np, dtype=plan.dtype, device=DEV, requires_grad=True)
    loss = DEAMNLL.apply(c, plan, torch.tensor(inp["d"], device=DEV), None)
    loss.backward()
    print(prec, "loss rel", abs(loss.item() - L_o) / abs(L_o), "grad rel", rel(c.grad.cpu().numpy(), grad_o))
    assert abs(loss.item() - L_o) <= (1e-7 if prec == "mixed" else 1e-12) * abs(L_o)
    assert rel(c.grad.cpu().numpy(), grad_o) <= tol


def test_nll_gradient_finite_differences(blobs):
    """FP64 GPU path: central differences of L along 16 random single-voxel axes
    per component and 4 random directions."""
    from paper_2202_00116_amd.plan import Plan
    from paper_2202_00116_amd.autograd import DEAMNLL
    inp = blobs
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], "fp64")
    d = torch.tensor(inp["d"], device=DEV)
    c0 = torch.tensor(inp["c"], device=DEV)
    c = c0.clone().requires_grad_(True)
    DEAMNLL.apply(c, plan, d, None).backward()
    grad = c.grad.detach()
    rng = np.random.default_rng(41)
    h = 1e-3
    dirs = []
    for i in range(2):
        for x in rng.choice(g.n_voxels, 16, replace=False):
            e = torch.zeros_like(c0)
            e[i, x] = 1.0
            dirs.append(e)
    for _ in range(4):
        dirs.append(torch.tensor(rng.standard_normal((2, g.n_voxels)) / np.sqrt(2 * g.n_voxels), device=DEV))
    gmax = grad.abs().max().item()
    for e in dirs:
        fp = DEAMNLL.apply(c0 + h * e, plan, d, None).item()
        fm = DEAMNLL.apply(c0 - h * e, plan, d, None).item()
        fd = (fp - fm) / (2 * h)
        an = (grad * e).sum().item()
        assert abs(fd - an) <= 1e-6 * gmax + 1e-6 * abs(an), (fd, an)


def test_poly_forward_vjp_matches_nll(blobs):
    """Autograd through PolyForward with the NLL written in torch gives the same
    gradient as the fused DEAMNLL adjoint (FP64)."""
    from paper_2202_00116_amd.plan import Plan
    from paper_2202_00116_amd.autograd import DEAMNLL, PolyForward
    inp = blobs
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], "fp64")
    d = torch.tensor(inp["d"], device=DEV)
    c1 = torch.tensor(inp["c"], device=DEV, requires_grad=True)
    gg = PolyForward.apply(c1, plan)
    loss1 = (gg - d.double() * torch.log(gg)).sum()
    loss1.backward()
    c2 = torch.tensor(inp["c"], device=DEV, requires_grad=True)
    loss2 = DEAMNLL.apply(c2, plan, d, None)
    loss2.backward()
    assert abs(loss1.item() - loss2.item()) <= 1e-11 * abs(loss2.item())
    assert rel(c1.grad.cpu().numpy(), c2.grad.cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-10)])
def test_poly_forward_vjp_matches_oracle(orc, blobs, prec, tol):
    """PolyForward against the oracle: the expected counts g, and the backward
    pass (VJP-mode weights u_i = -sum_j v_j a_ij, then the backprojection) for
    an upstream v = dloss/dg > 0 (the weights are then all negative, so the
    backprojection does not cancel), element by element."""
    from paper_2202_00116_amd.plan import Plan
    from paper_2202_00116_amd.autograd import PolyForward
    inp = blobs
    g = inp["geom"]
    plan = Plan(g, inp["I0"], inp["mu"], prec)
    c = torch.tensor(inp["c"], dtype=plan.dtype, device=DEV, requires_grad=True)
    gg = PolyForward.apply(c, plan)
    rng = np.random.default_rng(77)
    v = rng.uniform(0.5, 1.5, (2, g.n_rays)) / inp["d"].mean()
    (gg * torch.tensor(v, dtype=gg.dtype, device=DEV)).sum().backward()
    # the oracle takes the line integrals the GPU used (the plan's projection)
    l = plan.forward(c.detach()).double().cpu().numpy()
    v_used = torch.tensor(v, dtype=plan.dtype).double().numpy()
    u_o, g_o, _ = orc.poly_mean(inp["I0"], inp["mu"], l, np.zeros((2, g.n_rays)), None,
                                mode=orc.W_VJP, v=v_used)
    grad_o = orc.backproject(g, u_o)
    e_g, e_grad = rel(gg.detach().cpu().numpy(), g_o), rel(c.grad.cpu().numpy(), grad_o)
    print(f"{prec} PolyForward: g {e_g:.3e}, VJP {e_grad:.3e}")
    assert e_g <= tol and e_grad <= tol


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_single_bin_beer_lambert(orc, prec):
    """One energy bin (Eq. 8 reduces to Beer-Lambert): g_j = I0_j exp(-mu.l),
    element by element against the oracle's FP64 exp.  Mixed plans evaluate
    exp as the hardware 2^x of the argument scaled by log2(e): with the line
    integrals given in FP32 (both sides), the FP32 roundings of mu (1 unit of
    2^-24 relative), log2(e) (1), the scaled integrals (1), the product mu_2 k_2
    (1) and the fused sum (1) shift the exponent by at most 5 * 2^-24 * x
    (x = mu.l; d(2^-a)/2^-a = ln 2 da and a = x log2(e)); the hardware 2^x
    (1 ulp), I0 (1) and its product (1) add 3 units, with 2 to spare:
    |g - g_o| / g_o <= 2^-24 (5 x + 5)."""
    from paper_2202_00116_amd.plan import Plan
    g = make_inputs("fan64", with_data=False)["geom"]
    I0 = np.array([[7e4], [1.3e5]])
    mu = np.array([[0.021], [0.057]])
    plan = Plan(g, I0, mu, prec)
    rng = np.random.default_rng(19)
    l = rng.uniform(0, 40, (2, g.n_rays))
    if prec == "mixed":
        l = l.astype(np.float32).astype(np.float64)
    d = rng.uniform(0, 1e5, (2, g.n_rays)).astype(np.float32)
    _, gg, _ = plan.poly_mean(torch.tensor(l, dtype=plan.dtype, device=DEV),
                              torch.tensor(d, device=DEV), None, want_g=True)
    gg = gg.double().cpu().numpy()
    x = mu[0, 0] * l[0] + mu[1, 0] * l[1]
    ref = I0[:, :1] * np.exp(-x)[None, :]
    _, g_o, _ = orc.poly_mean(I0, mu, l, d.astype(np.float64))
    assert np.allclose(g_o, ref, rtol=1e-14)
    e = np.abs(gg - g_o) / g_o
    bound = (2.0 ** -24) * (5.0 * x + 5.0) if prec == "mixed" else 1e-14 * (1.0 + x)
    print(f"{prec} single bin: max rel {e.max():.3e}, max of rel / bound {(e / bound).max():.3f}")
    assert np.all(e <= bound)


def test_gradcheck_small():
    """torch.autograd.gradcheck of DEAMNLL on a small FP64 problem."""
    from paper_2202_00116_amd.plan import Plan
    from paper_2202_00116_amd.autograd import DEAMNLL
    inp = make_inputs("fan64")
    plan = Plan(inp["geom"], inp["I0"], inp["mu"], "fp64")
    d = torch.tensor(inp["d"], device=DEV)
    mask = torch.zeros(plan.R, dtype=torch.uint8, device=DEV)
    mask[::7] = 1
    c = torch.tensor(inp["c0"] * 0.95, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: DEAMNLL.apply(x, plan, d, mask), (c,), eps=1e-4,
                                    atol=1e-4, rtol=1e-6, fast_mode=True)
