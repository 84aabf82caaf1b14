"""Pins of the oracle's bowtie filter (energy- and channel-dependent spectra
I0_j(y,E) of Eq. 8), given as the filter's path lengths in the two basis
materials per channel:

* a filter of zero thickness is no filter, bit for bit;
* the per-ray spectrum I0_j(E) exp(-mu_1 b_1k - mu_2 b_2k) gives the same
  energy sums, weights and objective as the plain poly-mean of the line
  integrals shifted by the filter path (l_i + b_ik): the filter acts like
  material on the ray that no voxel holds;
* one energy bin: g_j = I0_j exp(-mu (l + b)), Beer-Lambert;
* DEAM on data simulated with the filter decreases the masked I-divergence.
"""
import numpy as np
import pytest

from workloads import make_inputs, bowtie


def test_zero_filter_is_no_filter(orc):
    inp = make_inputs("fan64")
    g = inp["geom"]
    l = orc.forward(g, inp["c0"])
    bt = np.zeros((2, g.n_cols))
    for mode in (orc.W_AM, orc.W_GRAD):
        a = orc.poly_mean(inp["I0"], inp["mu"], l, inp["d"], None, mode)
        b = orc.poly_mean_bt(inp["I0"], inp["mu"], bt, l, inp["d"], None, mode)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("mode", ["am", "grad", "step"])
def test_filter_is_a_shift_of_the_line_integrals(orc, mode):
    inp = make_inputs("helical_small")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    rng = np.random.default_rng(101)
    bt = np.stack([rng.uniform(0, 30, g.n_cols), rng.uniform(0, 3, g.n_cols)])
    l = orc.forward(g, inp["c0"])
    k = np.arange(g.n_rays) % g.n_cols
    ls = l + bt[:, k]
    m = {"am": orc.W_AM, "grad": orc.W_GRAD, "step": orc.W_STEP_VJP}[mode]
    v = rng.standard_normal((4, g.n_rays)) if mode == "step" else None
    a = orc.poly_mean_bt(inp["I0"], inp["mu"], bt, l, inp["d"], mask, m, v)
    b = orc.poly_mean(inp["I0"], inp["mu"], ls, inp["d"], mask, m, v)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-12 * np.abs(y).max())


def test_single_bin_beer_lambert(orc):
    nE = 5
    I0 = np.zeros((2, nE))
    I0[0, 2], I0[1, 2] = 1e5, 2e5
    mu = np.full((2, nE), 0.02)
    mu[1] = 0.05
    R, n_cols = 12, 4
    rng = np.random.default_rng(102)
    l = rng.uniform(0, 20, (2, R))
    bt = rng.uniform(0, 10, (2, n_cols))
    k = np.arange(R) % n_cols
    _, gg, _ = orc.poly_mean_bt(I0, mu, bt, l, np.ones((2, R)), None)
    att = np.exp(-(0.02 * (l[0] + bt[0, k]) + 0.05 * (l[1] + bt[1, k])))
    assert np.allclose(gg, np.stack([1e5 * att, 2e5 * att]), rtol=1e-14)


def test_deam_with_filter_decreases_objective(orc):
    inp = make_inputs("fan64", with_bowtie=True)
    g = inp["geom"]
    assert np.allclose(inp["bt"], bowtie(g))
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    c, h = orc.iterate_bt(g, inp["I0"], inp["mu"], inp["bt"], inp["d"], mask, inp["Z"], inp["c0"], 10)
    assert np.all(np.diff(h) < 0)
    # ignoring the filter on filtered data is visibly worse
    cw, hw = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], 10)
    assert hw[-1] > 2 * h[-1]
