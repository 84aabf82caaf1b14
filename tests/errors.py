"""Error measures of the parity tests.

Every result is compared in two ways: the relative L2 error over the whole
array, ||x - x_o|| / ||x_o||, and the element-wise error, the largest
|x - x_o| relative to max |x_o|.  The first is what accumulates from
independent rounding errors; the second catches an error confined to a
few elements (a wrong voxel, an edge tile, a weak ray) that the first would
average away."""
import numpy as np


def rel_l2(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300))


def errors(a, b):
    return rel_l2(a, b), rel_max(a, b)


def assert_close(a, b, tol, tol_max=None, what=""):
    """Both errors within their bounds (tol_max defaults to tol); prints them."""
    e2, em = errors(a, b)
    tm = tol if tol_max is None else tol_max
    print(f"{what}: rel L2 {e2:.3e} (<= {tol:.1e}), max-abs/max {em:.3e} (<= {tm:.1e})", flush=True)
    assert e2 <= tol, (what, "rel L2", e2, tol)
    assert em <= tm, (what, "max-abs/max", em, tm)
    return e2, em
