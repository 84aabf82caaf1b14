"""Edge cases and error paths of the widening entry points on the GPU: zero
iterations leave the iterate untouched, NULL pointers and bad sizes are
rejected before anything is enqueued, and a rejected call leaves its outputs
alone."""
import ctypes as C

import numpy as np
import pytest
import torch

from workloads import make_inputs, PENALTY

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def setup():
    from paper_2202_00116_amd.plan import Plan
    inp = make_inputs("fan64")
    plan = Plan(inp["geom"], inp["I0"], inp["mu"], "mixed")
    return inp, plan


def test_zero_iterations_are_no_ops(setup):
    from paper_2202_00116_amd.plan import Plan, iterate_dual
    inp, plan = setup
    d = torch.tensor(inp["d"], device=DEV)
    c0 = torch.tensor(inp["c0"], device=DEV)
    lam, delta = PENALTY["fan64"]
    for run in (lambda c: plan.iterate_penalized(c, d, None, inp["Z"], lam, delta, 0),
                lambda c: plan.iterate_os(c, d, None, inp["Z"], 4, 0)):
        c = c0.clone()
        run(c)
        assert torch.equal(c, c0)
    lo, hi = np.zeros_like(inp["I0"]), np.zeros_like(inp["I0"])
    lo[0], hi[1] = inp["I0"][0], inp["I0"][1]
    plo = Plan(inp["geom"], lo, inp["mu"], "mixed")
    phi = Plan(inp["geom"], hi, inp["mu"], "mixed")
    c = c0.clone()
    iterate_dual(plo, phi, c, d, None, d, None, inp["Z"], 0)
    assert torch.equal(c, c0)


def _vp(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def test_null_pointers_are_rejected(setup):
    from paper_2202_00116_amd._lib import DeamMarParams
    inp, plan = setup
    lib = plan.lib
    Zh = np.ascontiguousarray(inp["Z"], dtype=np.float64)
    Zp = Zh.ctypes.data_as(C.c_void_p)
    c = torch.tensor(inp["c0"], device=DEV)
    d = torch.tensor(inp["d"], device=DEV)
    b = torch.ones((4, plan.V), dtype=torch.float32, device=DEV)
    ws, n = plan.workspace(7)
    ERR_NULL = -1
    assert lib.deam_update_penalized(plan._p, None, _vp(c), None, _vp(b), Zp, 1.0, 0.01, None) == ERR_NULL
    assert lib.deam_penalty(plan._p, _vp(c), 1.0, 0.01, None, ws, n, None) == ERR_NULL
    assert lib.deam_iterate_penalized(plan._p, _vp(c), None, None, Zp, 1.0, 0.01, 1, None, ws, n,
                                      None) == ERR_NULL
    assert lib.deam_iterate_os(plan._p, None, _vp(d), None, Zp, 2, 1, None, ws, n, None) == ERR_NULL
    assert lib.deam_dilate_mask(plan._p, None, 1, None, None) == ERR_NULL
    assert lib.deam_fbp(plan._p, None, 1, None, ws, n, None) == ERR_NULL
    P = DeamMarParams()
    assert lib.deam_mar_init(plan._p, _vp(d), C.byref(P), None, None, None, ws, n, None) == ERR_NULL
    assert lib.deam_plan_set_bowtie(None, None) == ERR_NULL
    # the iterate is untouched by all of these
    assert torch.equal(c, torch.tensor(inp["c0"], device=DEV))


def test_small_workspace_is_rejected(setup):
    inp, plan = setup
    lib = plan.lib
    Zh = np.ascontiguousarray(inp["Z"], dtype=np.float64)
    c = torch.tensor(inp["c0"], device=DEV)
    d = torch.tensor(inp["d"], device=DEV)
    ws, n = plan.workspace(7)
    rc = lib.deam_iterate_penalized(plan._p, _vp(c), _vp(d), None, Zh.ctypes.data_as(C.c_void_p),
                                    1.0, 0.01, 1, None, ws, C.c_size_t(n.value - 256), None)
    assert rc == -4
    rc = lib.deam_iterate_os(plan._p, _vp(c), _vp(d), None, Zh.ctypes.data_as(C.c_void_p), 2, 1, None,
                             ws, C.c_size_t(16), None)
    assert rc == -4
    assert torch.equal(c, torch.tensor(inp["c0"], device=DEV))


def test_workspace_sizes_of_new_operations(setup):
    _, plan = setup
    from paper_2202_00116_amd import _lib as L
    for op in (L.OP_PENALTY, L.OP_ITERATE_PENALIZED, L.OP_FBP, L.OP_MAR_INIT):
        assert plan.workspace_bytes(op) > 0
    with pytest.raises(L.DeamError, match="VALUE"):
        plan.workspace_bytes(10)


def test_dilate_rejects_overlap_and_radius(setup):
    from paper_2202_00116_amd._lib import DeamError
    inp, plan = setup
    m = torch.zeros(plan.R, dtype=torch.uint8, device=DEV)
    with pytest.raises(DeamError, match="VALUE"):
        plan.dilate_mask(m, -1)
    with pytest.raises(DeamError, match="VALUE"):
        plan.dilate_mask(m, plan.geom.n_cols + 1)
    rc = plan.lib.deam_dilate_mask(plan._p, _vp(m), 1, C.c_void_p(m.data_ptr() + 1), None)
    assert rc == -7
