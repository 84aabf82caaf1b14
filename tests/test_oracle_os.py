"""Pins of the oracle's ordered-subset DEAM (views split into interleaved
subsets; one DEAM step per subset):

* one subset is the DEAM iteration, bit for bit;
* in 2D, the step of subset s is the DEAM step of the fan-beam scan made of
  that subset's views alone (start angle shifted by s views, n_sub times the
  angular step), with its counts and mask;
* the subsets speed up the first epochs: the objective after one epoch of
  four subsets is below that after one DEAM iteration.
"""
import dataclasses
import math

import numpy as np
import pytest

from workloads import make_inputs


def _subset_geometry(g, n_sub, s):
    n = len(range(s, g.n_views, n_sub))
    return dataclasses.replace(g, n_views=n, beta0=g.beta0 + 2.0 * math.pi * s / g.views_per_rot,
                               views_per_rot=g.views_per_rot / n_sub)


def _subset_rays(g, n_sub, s):
    per = g.n_rows * g.n_cols
    v = np.arange(s, g.n_views, n_sub)
    return (v[:, None] * per + np.arange(per)[None, :]).reshape(-1)


def test_one_subset_is_deam(orc):
    inp = make_inputs("helical_small")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    args = (g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"])
    c1, h1 = orc.iterate(*args, inp["c0"], 3)
    c2, h2 = orc.iterate_os(*args, inp["c0"], 1, 3)
    assert np.array_equal(c1, c2) and np.array_equal(h1, h2)


@pytest.mark.parametrize("n_sub", [2, 3, 5])
def test_subset_step_is_deam_on_the_subset_scan(orc, n_sub):
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    c = inp["c0"].copy()
    for s in range(n_sub):
        gs = _subset_geometry(g, n_sub, s)
        rays = _subset_rays(g, n_sub, s)
        c, _ = orc.iterate(gs, inp["I0"], inp["mu"], np.ascontiguousarray(inp["d"][:, rays]),
                           np.ascontiguousarray(mask[rays]), inp["Z"], c, 1)
    ref, h = orc.iterate_os(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], n_sub, 1)
    assert np.abs(c - ref).max() <= 1e-12 * np.abs(ref).max()
    assert h[0] == pytest.approx(orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, inp["c0"]),
                                 rel=1e-12)


def test_subsets_speed_up_the_first_epoch(orc):
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    args = (g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"])
    c1, _ = orc.iterate(*args, inp["c0"], 1)
    c4, _ = orc.iterate_os(*args, inp["c0"], 4, 1)
    f = lambda c: orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c)  # noqa: E731
    assert f(c4) < f(c1) < f(inp["c0"])
