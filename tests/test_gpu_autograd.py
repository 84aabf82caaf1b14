"""Hand-written adjoint of the Poisson NLL (and of c -> g) behind
torch.autograd.Function, checked against the FP64 oracle gradient and against
FP64 central finite differences (h = 1e-3)."""
import numpy as np
import pytest
import torch

from workloads import blob_inputs, make_inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


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
