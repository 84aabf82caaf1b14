"""deam_poly_mean_noalloc (no workspace, no allocation) against deam_poly_mean
through the C ABI: bit for bit on two calls in a row on one GPU, the second
on a smaller problem (so its scratch holds the first call's partials), in
every weight mode; sizes beyond the scratch are rejected before launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from workloads import make_inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _vp(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _inputs(name, prec, seed):
    from paper_2202_00116_amd.plan import Plan
    inp = make_inputs(name)
    plan = Plan(inp["geom"], inp["I0"], inp["mu"], prec)
    rng = np.random.default_rng(seed)
    c = inp["c0"] * rng.uniform(0.8, 1.2, inp["c0"].shape)
    l = plan.forward(torch.tensor(c, dtype=plan.dtype, device=DEV))
    d = torch.tensor(inp["d"], device=DEV)
    mask = (torch.rand(plan.R, device=DEV) < 0.1).to(torch.uint8)
    v4 = torch.randn((4, plan.R), dtype=plan.dtype, device=DEV)
    return plan, l, d, mask, v4


def _run(plan, l, d, mask, mode, v, noalloc):
    from paper_2202_00116_amd import _lib as L
    nw = 4 if mode == L.W_AM else 2
    w = torch.full((nw, plan.R), float("nan"), dtype=plan.dtype, device=DEV)
    g = torch.full((2, plan.R), float("nan"), dtype=plan.dtype, device=DEV)
    obj = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    if noalloc:
        rc = plan.lib.deam_poly_mean_noalloc(plan._p, _vp(l), _vp(d), _vp(mask), mode, _vp(v),
                                             _vp(w), _vp(g), _vp(obj), _stream())
    else:
        ws, n = plan.workspace(L.OP_POLY_MEAN)
        rc = plan.lib.deam_poly_mean(plan._p, _vp(l), _vp(d), _vp(mask), mode, _vp(v), _vp(w),
                                     _vp(g), _vp(obj), ws, n, _stream())
    assert rc == 0, plan.lib.deam_last_error()
    torch.cuda.synchronize()
    return w, g, obj


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_matches_workspace_entry_point(prec):
    from paper_2202_00116_amd import _lib as L
    big = _inputs("fan128", prec, 1)
    small = _inputs("fan64", prec, 2)
    for mode in (L.W_AM, L.W_GRAD, L.W_VJP, L.W_STEP_VJP):
        for plan, l, d, mask, v4 in (big, small):      # the second call is smaller
            v = None if mode in (L.W_AM, L.W_GRAD) else (v4[:2].contiguous() if mode == L.W_VJP else v4)
            a = _run(plan, l, d, mask, mode, v, noalloc=True)
            b = _run(plan, l, d, mask, mode, v, noalloc=False)
            assert torch.equal(a[0], b[0]), (prec, mode)
            assert torch.equal(a[1], b[1]), (prec, mode)
            if mode in (L.W_AM, L.W_GRAD):
                assert torch.equal(a[2], b[2]) and torch.isfinite(a[2]).all(), (prec, mode)


def test_noalloc_rejects_too_many_rays():
    """A plan with more rays than the scratch serves is refused before
    anything is enqueued (the outputs keep their values)."""
    from paper_2202_00116_amd.plan import Plan
    from workloads import geometry as G
    inp = make_inputs("fan64", with_data=False)
    g = G.Geometry(kind=1, nx=8, ny=8, nz=8, dx=1.0, dy=1.0, dz=1.0, n_views=512, n_rows=256,
                   n_cols=520, sid=200.0, sdd=400.0, dgamma=G.fan_dgamma(8, 8, 1.0, 1.0, 200.0, 520),
                   col_offset=0.0, drow_iso=0.05, beta0=0.0, views_per_rot=512.0, feed_per_rot=1.0)
    plan = Plan(g, inp["I0"], inp["mu"], "mixed")
    assert plan.R > 67_100_672
    t = torch.zeros(8, device=DEV)
    rc = plan.lib.deam_poly_mean_noalloc(plan._p, _vp(t), _vp(t), None, 0, None, _vp(t), None,
                                         None, _stream())
    assert rc == -6
    assert b"deam_poly_mean_noalloc" in plan.lib.deam_last_error()
    torch.cuda.synchronize()
    assert torch.equal(t, torch.zeros(8, device=DEV))
