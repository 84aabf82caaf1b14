"""Pins of the oracle's two-scan DEAM (a system operator and a metal trace
per spectrum, Section 2.1) and of the trace dilation:

* with the same geometry and trace for both scans it is the DEAM iteration;
* with different scans (the high-energy scan rotated by half a view and its
  detector shifted by a quarter channel) the summed masked I-divergence
  decreases at every iteration (the alternating minimisation still holds);
* dilation: radius 0 is the identity, a single ray grows into a run of
  2r + 1 channels clipped at the detector ends, and random masks agree with
  the union of shifted copies.
"""
import dataclasses
import math

import numpy as np

from workloads import make_inputs


def shifted_scan(g):
    return dataclasses.replace(g, beta0=g.beta0 + math.pi / g.views_per_rot,
                               col_offset=g.col_offset + 0.25)


def test_same_scans_are_deam(orc):
    for name in ("fan64", "helical_small"):
        inp = make_inputs(name)
        g = inp["geom"]
        mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
        ref, href = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], 3)
        c, h = orc.iterate_dual((g, g), inp["I0"], inp["mu"], (inp["d"][0], inp["d"][1]),
                                (mask, mask), inp["Z"], inp["c0"], 3)
        assert np.abs(c - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.allclose(h, href, rtol=1e-12)


def test_different_scans_decrease_the_objective(orc):
    from workloads.configs import expected_counts, phantom_for
    inp = make_inputs("fan64")
    gl = inp["geom"]
    gh = shifted_scan(gl)
    gbar = expected_counts(gh, phantom_for("fan64"), inp["I0"])
    dh = np.random.default_rng(97).poisson(gbar[1]).astype(np.float64)
    ml = orc.metal_trace(gl, inp["metal"], inp["t"])[0]
    mh = orc.metal_trace(gh, inp["metal"], inp["t"])[0]
    assert not np.array_equal(ml, mh)
    c, h = orc.iterate_dual((gl, gh), inp["I0"], inp["mu"], (inp["d"][0], dh), (ml, mh), inp["Z"],
                            inp["c0"], 10)
    assert np.all(np.diff(h) < 0), h


def test_dilate_mask(orc):
    from tests.test_oracle_geometry import small_box3d
    g = small_box3d()
    rng = np.random.default_rng(98)
    m = (rng.uniform(size=g.n_rays) < 0.05).astype(np.uint8)
    assert np.array_equal(orc.dilate_mask(g, m, 0), m)
    one = np.zeros(g.n_rays, np.uint8)
    one[3 * g.n_cols + 1] = 1                                  # channel 1 of row 3
    d = orc.dilate_mask(g, one, 3).reshape(-1, g.n_cols)
    assert d[3, :5].tolist() == [1] * 5 and d[3, 5:].sum() == 0 and d.sum() == 5
    for r in (1, 2, 5):
        M = m.reshape(-1, g.n_cols)
        ref = np.zeros_like(M)
        for s in range(-r, r + 1):
            sh = np.zeros_like(M)
            if s >= 0:
                sh[:, s:] = M[:, :g.n_cols - s]
            else:
                sh[:, :s] = M[:, -s:]
            ref |= sh
        assert np.array_equal(orc.dilate_mask(g, m, r), ref.reshape(-1))
