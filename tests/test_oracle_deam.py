"""Pins of the oracle's DEAM steps against closed forms, invariants of the
alternating minimisation and finite differences (no call of the oracle is
checked against itself)."""
import numpy as np
import pytest

from workloads import make_inputs, geometry_for
from workloads.geometry import ray_endpoints
from tests.bruteforce import ray_row
from tests.test_oracle_geometry import small_fan


def test_single_bin_beer_lambert(orc):
    """T6: one energy bin: g_j = I0_j exp(-mu.l) and -ln(g_j/I0_j) = mu.l (Eq. 8)."""
    rng = np.random.default_rng(1)
    R = 1000
    l = rng.uniform(0, 40, (2, R))
    d = rng.uniform(0, 1e5, (2, R))
    I0 = np.array([[7e4], [1.3e5]])
    mu = np.array([[0.021], [0.057]])
    _, g, _ = orc.poly_mean(I0, mu, l, d)
    ml = mu[0, 0] * l[0] + mu[1, 0] * l[1]
    assert np.allclose(-np.log(g[0] / I0[0, 0]), ml, rtol=1e-13, atol=1e-13)
    assert np.allclose(-np.log(g[1] / I0[1, 0]), ml, rtol=1e-13, atol=1e-13)


def test_flat_attenuation_sums_spectrum(orc):
    """Energy-independent mu: g_j = (sum_E I0_j(E)) exp(-mu.l), which catches a
    dropped or double-counted energy bin."""
    inp = make_inputs("fan64", with_data=False)
    I0 = inp["I0"]
    nE = I0.shape[1]
    mu = np.stack([np.full(nE, 0.02), np.full(nE, 0.05)])
    rng = np.random.default_rng(2)
    l = rng.uniform(0, 30, (2, 500))
    _, g, _ = orc.poly_mean(I0, mu, l, np.ones((2, 500)))
    ref = I0.sum(axis=1)[:, None] * np.exp(-(0.02 * l[0] + 0.05 * l[1]))[None, :]
    assert np.allclose(g, ref, rtol=1e-13)


def test_linear_family_constraint(orc):
    """T7 (Eqs. 9-10): the p-step keeps sum_E p_j = d~_j.  With mu_1 = 1 at every
    energy, w~_1 = sum_j sum_E p_j, so w~_1 = d_L + d_H off the trace and
    g_L + g_H on it (p = q there, Eq. 11), while w^_1 = g_L + g_H always."""
    inp = make_inputs("fan64", with_data=False)
    I0, mu = inp["I0"], inp["mu"].copy()
    mu[0] = 1.0
    rng = np.random.default_rng(3)
    R = 2000
    l = rng.uniform(0, 20, (2, R))
    d = rng.poisson(5e4, (2, R)).astype(float)
    mask = (rng.random(R) < 0.3).astype(np.uint8)
    w, g, _ = orc.poly_mean(I0, mu, l, d, mask)
    off, on = mask == 0, mask == 1
    assert np.allclose(w[0][off], (d[0] + d[1])[off], rtol=1e-13)
    assert np.allclose(w[0][on], (g[0] + g[1])[on], rtol=1e-13)
    assert np.allclose(w[2], g[0] + g[1], rtol=1e-13)
    # on the trace the measured and estimated weights coincide exactly
    assert np.array_equal(w[:2, on], w[2:, on])


def test_idiv_vanishes_on_consistent_data_and_matches_nll(orc):
    """Eq. 5 is zero when d = g, and differs from the NLL sum(g - d ln g) by the
    constant sum(d ln d - d) over the rays off the trace."""
    inp = make_inputs("fan64")
    g = inp["geom"]
    rng = np.random.default_rng(4)
    mask = (rng.random(g.n_rays) < 0.2).astype(np.uint8)
    l = orc.forward(g, inp["c0"])
    _, gg, obj = orc.poly_mean(inp["I0"], inp["mu"], l, inp["d"], mask)
    _, _, obj0 = orc.poly_mean(inp["I0"], inp["mu"], l, gg, mask)
    assert np.abs(obj0).max() < 1e-9 * gg.max()
    _, _, nll = orc.poly_mean(inp["I0"], inp["mu"], l, inp["d"], mask, mode=orc.W_GRAD)
    d = inp["d"].astype(float)
    off = mask == 0
    const = np.sum(np.where(d > 0, d * np.log(np.where(d > 0, d, 1.0)), 0.0)[:, off] - d[:, off])
    assert abs((obj.sum() - nll.sum()) - const) < 1e-9 * abs(const)


def test_consistent_data_is_fixed_point(orc):
    """T8: if d = g(c*) then r = 1, w~ = w^, and the update leaves c* unchanged."""
    inp = make_inputs("fan64", with_data=False)
    g = inp["geom"]
    c = inp["c0"] * 1.1
    l = orc.forward(g, c)
    _, gg, _ = orc.poly_mean(inp["I0"], inp["mu"], l, np.zeros((2, g.n_rays)))
    c1, hist = orc.iterate(g, inp["I0"], inp["mu"], gg, None, inp["Z"], c, 1)
    assert np.abs(c1 - c).max() < 1e-12
    assert hist[0] < 1e-9 * gg.sum()


def test_all_metal_mask_is_noop(orc):
    """T9: with every ray on the trace (p = q everywhere, Eq. 11) the update is
    exactly zero."""
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = np.ones(g.n_rays, dtype=np.uint8)
    c1, hist = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], 2)
    assert np.array_equal(c1, inp["c0"])
    assert np.all(hist == 0.0)


def test_voxels_seen_only_by_corrupt_rays_keep_their_value(orc):
    """Voxels whose every ray lies on the metal trace keep their initial value
    exactly (the metal region is estimated from the initial image)."""
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask, _ = orc.metal_trace(g, inp["metal"], inp["t"])
    seen = orc.backproject(g, (mask == 0).astype(float))[0]
    hidden = seen == 0.0
    assert hidden.sum() > 0
    c1, _ = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], 3)
    assert np.array_equal(c1[:, hidden], inp["c0"][:, hidden])
    assert not np.array_equal(c1[:, ~hidden], inp["c0"][:, ~hidden])


@pytest.mark.parametrize("name,n", [("fan64", 20), ("fan128", 12), ("helical_small", 6)])
@pytest.mark.parametrize("use_mask", [True, False])
def test_masked_idiv_nonincreasing(orc, name, n, use_mask):
    """T10: the masked I-divergence of Eq. 5 never increases across DEAM
    iterations (alternating minimisation with a majorising surrogate)."""
    inp = make_inputs(name)
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0] if use_mask else None
    c, hist = orc.iterate(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], inp["c0"], n)
    final = orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c)
    seq = np.append(hist, final)
    assert np.all(np.diff(seq) <= 1e-12 * seq[:-1]), seq
    assert seq[-1] < 0.9 * seq[0]


def test_monoenergetic_matches_textbook_am(orc):
    """T11: one energy bin reduces DEAM to the alternating minimisation
    algorithm for transmission tomography.  With one bin mu_i cancels in the
    ratio of the backprojections, so every component moves by the same log
    ratio, each with its own normaliser:
        q = I0 exp(-H (mu_1 c_1 + mu_2 c_2)),
        c_i <- c_i - ln( H^T d / H^T q ) / Z_i,
    computed here with the brute-force dense H."""
    g = small_fan()
    S, P = ray_endpoints(g)
    H = np.stack([ray_row(g, S[i], P[i]) for i in range(g.n_rays)])
    rng = np.random.default_rng(11)
    mu1, mu2 = 0.3, 0.12
    c_true = np.stack([rng.uniform(0.5, 1.5, g.n_voxels), rng.uniform(0.0, 0.5, g.n_voxels)])
    I0 = np.array([[1e4], [0.0]])
    mu = np.array([[mu1], [mu2]])
    d = np.stack([rng.poisson(1e4 * np.exp(-H @ (mu1 * c_true[0] + mu2 * c_true[1]))).astype(float),
                  np.zeros(g.n_rays)])
    Z = np.array([2 * mu1 * g.box_diagonal(), 2 * mu2 * g.box_diagonal()])
    c0 = np.stack([np.full(g.n_voxels, 1.0), np.full(g.n_voxels, 0.2)])
    c_orc, _ = orc.iterate(g, I0, mu, d, None, Z, c0, 3)
    c = c0.copy()
    for _ in range(3):
        q = 1e4 * np.exp(-H @ (mu1 * c[0] + mu2 * c[1]))
        bt, bh = H.T @ d[0], H.T @ q
        ok = (bt > 0) & (bh > 0)
        step = np.log(bt[ok] / bh[ok])
        c[0, ok] -= step / Z[0]
        c[1, ok] -= step / Z[1]
    assert np.allclose(c_orc, c, rtol=0, atol=1e-12)
    assert np.abs(c_orc - c0).max() > 1e-3


def test_gradient_matches_finite_differences(orc):
    """T12: dL/dc_i = b~_i - b^_i for the Poisson NLL L = sum (g - d ln g) off the
    trace, against FP64 central differences (h = 1e-3)."""
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask, _ = orc.metal_trace(g, inp["metal"], inp["t"])
    c = inp["c0"] * 0.97
    L0, grad = orc.nll_grad(g, inp["I0"], inp["mu"], inp["d"], mask, c)
    rng = np.random.default_rng(12)
    h = 1e-3
    dirs = []
    for i in range(2):
        for x in rng.choice(np.flatnonzero(np.abs(grad[i]) > 1e-3 * np.abs(grad[i]).max()), 8, replace=False):
            e = np.zeros_like(c)
            e[i, x] = 1.0
            dirs.append(e)
    for _ in range(2):
        dirs.append(rng.standard_normal(c.shape) / np.sqrt(c.size))
    for e in dirs:
        fp = orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c + h * e, mode=orc.W_GRAD)
        fm = orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c - h * e, mode=orc.W_GRAD)
        fd = (fp - fm) / (2 * h)
        an = np.sum(grad * e)
        assert abs(fd - an) <= 1e-5 * np.abs(grad).max() + 1e-6 * abs(an), (fd, an)
    # the I-divergence has the same gradient (it differs by a constant)
    e = dirs[-1]
    fp = orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c + h * e)
    fm = orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c - h * e)
    assert abs((fp - fm) / (2 * h) - np.sum(grad * e)) <= 1e-5 * np.abs(grad).max()


def test_vjp_weights_are_finite_difference_products(orc):
    """W_VJP (adjoint of Eq. 8 for an upstream v_j = dloss/dg_j): the weight
    u_i(y) equals sum_j v_j dg_j/dl_i, with dg_j/dl_i taken by central
    differences of the oracle's expected counts g in l_i (not by the energy
    sums a_ij that the mode uses).  The trace does not enter."""
    inp = make_inputs("fan64", with_data=False)
    I0, mu = inp["I0"], inp["mu"]
    rng = np.random.default_rng(23)
    R = 400
    l = rng.uniform(0, 25, (2, R))
    v = rng.standard_normal((2, R))
    d = rng.uniform(0, 1e5, (2, R))
    mask = (rng.random(R) < 0.3).astype(np.uint8)
    u, _, _ = orc.poly_mean(I0, mu, l, d, mask, mode=orc.W_VJP, v=v)
    h = 1e-3
    for i in range(2):
        lp, lm = l.copy(), l.copy()
        lp[i] += h
        lm[i] -= h
        _, gp, _ = orc.poly_mean(I0, mu, lp, d)
        _, gm, _ = orc.poly_mean(I0, mu, lm, d)
        fd = (v * (gp - gm)).sum(axis=0) / (2 * h)
        scale = (np.abs(v) * np.abs(gp - gm)).sum(axis=0) / (2 * h)
        assert np.all(np.abs(u[i] - fd) <= 1e-6 * scale + 1e-12), i
