"""Ordered-subset DEAM on the GPU (deam_iterate_os) against the oracle's
ordered-subset iteration: interleaved view subsets that divide the view count
and that do not, 2D and helical, both precisions; one subset is deam_iterate
bit for bit; argument errors."""
import numpy as np
import pytest
import torch

from workloads import make_inputs
from tests.errors import rel_l2, rel_max

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _plan(inp, prec):
    from paper_2202_00116_amd.plan import Plan
    return Plan(inp["geom"], inp["I0"], inp["mu"], prec)


def rel(a, b):
    """The larger of the relative L2 error and the element-wise error (max-abs
    relative to max |b|): a bound on it bounds both."""
    return max(rel_l2(a, b), rel_max(a, b))


@pytest.mark.parametrize("name,n_sub,n_iter", [("fan64", 4, 5), ("fan64", 5, 3),
                                               ("helical_small", 3, 3), ("helical_small", 7, 2)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_iterate_os_matches_oracle(orc, name, n_sub, n_iter, prec, tol):
    inp = make_inputs(name)
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    ref, href = orc.iterate_os(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"],
                               n_sub, n_iter)
    plan = _plan(inp, prec)
    c = torch.tensor(inp["c0"], device=DEV)
    h = torch.zeros(n_iter, dtype=torch.float64, device=DEV)
    plan.iterate_os(c, torch.tensor(inp["d"], device=DEV), torch.tensor(mask, device=DEV), inp["Z"],
                    n_sub, n_iter, h)
    e = rel(c.cpu().numpy(), ref)
    eh = float(np.abs(h.cpu().numpy() - href).max() / abs(href[0]))
    print(f"{name} {prec} S={n_sub} {n_iter} epochs: image rel {e:.3e}, objective rel {eh:.3e}")
    assert e <= tol and eh <= tol
    # without the history the iterates are the same
    c2 = torch.tensor(inp["c0"], device=DEV)
    plan.iterate_os(c2, torch.tensor(inp["d"], device=DEV), torch.tensor(mask, device=DEV), inp["Z"],
                    n_sub, n_iter)
    assert torch.equal(c, c2)


@pytest.mark.parametrize("name", ["fan64", "helical_small"])
def test_one_subset_is_iterate(name):
    inp = make_inputs(name)
    plan = _plan(inp, "mixed")
    d = torch.tensor(inp["d"], device=DEV)
    a = torch.tensor(inp["c0"], device=DEV)
    b = a.clone()
    ha = torch.zeros(3, dtype=torch.float64, device=DEV)
    hb = torch.zeros(3, dtype=torch.float64, device=DEV)
    plan.iterate(a, d, None, inp["Z"], 3, ha)
    plan.iterate_os(b, d, None, inp["Z"], 1, 3, hb)
    assert torch.equal(a, b) and torch.equal(ha, hb)


def test_iterate_os_full_fan512_one_epoch(orc):
    """The 512 x 512 benchmark workload, 8 subsets, one epoch."""
    inp = make_inputs("fan512")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    ref, _ = orc.iterate_os(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], 8, 1)
    plan = _plan(inp, "mixed")
    c = torch.tensor(inp["c0"], device=DEV)
    plan.iterate_os(c, torch.tensor(inp["d"], device=DEV), torch.tensor(mask, device=DEV), inp["Z"],
                    8, 1)
    # eight updates of the image: relative L2 1e-5, element-wise the image
    # bound 1e-4
    e2, em = rel_l2(c.cpu().numpy(), ref), rel_max(c.cpu().numpy(), ref)
    print(f"fan512 mixed S=8, 1 epoch: image rel L2 {e2:.3e}, max-abs/max {em:.3e}")
    assert e2 <= 1e-5 and em <= 1e-4


def test_iterate_os_rejects_bad_subsets():
    from paper_2202_00116_amd._lib import DeamError
    inp = make_inputs("fan64", with_data=False)
    plan = _plan(inp, "mixed")
    c = torch.zeros((2, plan.V), dtype=torch.float64, device=DEV)
    d = torch.ones((2, plan.R), dtype=torch.float32, device=DEV)
    for n_sub in (0, inp["geom"].n_views + 1):
        with pytest.raises(DeamError, match="VALUE"):
            plan.iterate_os(c, d, None, inp["Z"], n_sub, 1)
