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


def test_iterate_c_proj_and_host_history(setup):
    """deam_iterate's c_proj is the final iterate in the plan precision (also
    with zero iterations), and deam_iterate_sync returns the same history in
    host memory, bit for bit, after waiting for the device."""
    from paper_2202_00116_amd.plan import Plan
    inp = setup[0]
    d = torch.tensor(inp["d"], device=DEV)
    for prec in ("mixed", "fp64"):
        plan = Plan(inp["geom"], inp["I0"], inp["mu"], prec)
        c_a = torch.tensor(inp["c0"], device=DEV)
        cp = torch.full((2, plan.V), float("nan"), dtype=plan.dtype, device=DEV)
        h_a = torch.zeros(3, dtype=torch.float64, device=DEV)
        plan.iterate(c_a, d, None, inp["Z"], 3, h_a, c_proj=cp)
        assert torch.equal(cp, c_a.to(plan.dtype))
        c_b = torch.tensor(inp["c0"], device=DEV)
        cp_b = torch.empty_like(cp)
        h_b = plan.iterate_sync(c_b, d, None, inp["Z"], 3, c_proj=cp_b)
        assert torch.equal(c_a, c_b) and torch.equal(cp, cp_b)
        assert np.array_equal(h_a.cpu().numpy(), h_b)
        c0 = torch.tensor(inp["c0"], device=DEV)
        cp0 = torch.full_like(cp, float("nan"))
        assert plan.iterate_sync(c0, d, None, inp["Z"], 0, c_proj=cp0).size == 0
        assert torch.equal(cp0, c0.to(plan.dtype))


def test_validate_inputs(setup):
    from paper_2202_00116_amd._lib import DeamError
    inp, plan = setup
    c = torch.tensor(inp["c0"], device=DEV)
    d = torch.tensor(inp["d"], device=DEV)
    assert plan.validate_inputs(c, d) == (0, 0)
    assert plan.validate_inputs(None, d) == (0, 0)
    c[1, 17] = float("nan")
    c[0, 3] = float("inf")
    d[0, 5] = -1.0
    d[1, 9] = float("nan")
    d[1, 11] = -0.0          # -0 is a valid count
    with pytest.raises(DeamError, match="VALUE"):
        plan.validate_inputs(c, d)
    bad = (C.c_int64 * 2)()
    ws, n = plan.workspace(2)
    rc = plan.lib.deam_validate_inputs(plan._p, _vp(c), _vp(d), bad, ws, n, None)
    assert rc == -7 and (bad[0], bad[1]) == (2, 2)
    assert b"non-finite" in plan.lib.deam_last_error()
    assert plan.lib.deam_validate_inputs(plan._p, _vp(c), _vp(d), bad, ws, C.c_size_t(8), None) == -4
