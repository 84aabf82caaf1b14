"""Pins of the oracle's vector-Jacobian product of one DEAM iteration
Phi(c) = c - ln(b~(c)/b^(c))/Z (the differentiable unrolled reconstruction):

* central finite differences of the oracle's own iteration map, along single
  voxels and random directions, with and without the metal-trace mask;
* an independent derivative: PyTorch FP64 autograd through the iteration
  written with a dense system matrix (columns = the oracle's projections of
  unit images) on a tiny grid;
* the chain rule through three iterations against finite differences of an
  L2 loss on the third iterate.
"""
import numpy as np
import pytest

from workloads import make_inputs
from tests.test_oracle_geometry import small_fan


def _phi(orc, inp, mask, c):
    return orc.iterate(inp["geom"], inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], c, 1)[0]


def test_step_vjp_matches_finite_differences(orc, use_mask=True):
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0] if use_mask else None
    rng = np.random.default_rng(51)
    c = inp["c0"] * 0.9 + 0.01 * rng.standard_normal(inp["c0"].shape)
    G = rng.standard_normal(c.shape)
    vjp = orc.step_vjp(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], c, G)
    h = 1e-5
    dirs = []
    for i in range(2):
        for x in rng.choice(g.n_voxels, 6, replace=False):
            e = np.zeros_like(c)
            e[i, x] = 1.0
            dirs.append(e)
    for _ in range(3):
        dirs.append(rng.standard_normal(c.shape))
    for e in dirs:
        fd = (np.sum(G * _phi(orc, inp, mask, c + h * e)) - np.sum(G * _phi(orc, inp, mask, c - h * e))) / (2 * h)
        an = np.sum(vjp * e)
        assert abs(fd - an) <= 2e-5 * (abs(an) + np.abs(vjp).max() * np.sqrt(np.sum(e * e))), (fd, an)
    # the Jacobian is not the identity: the data terms contribute
    assert np.abs(vjp - G).max() > 1e-2 * np.abs(G).max()


def test_step_vjp_without_mask_matches_finite_differences(orc):
    test_step_vjp_matches_finite_differences(orc, use_mask=False)


def test_step_vjp_matches_dense_autograd(orc):
    torch = pytest.importorskip("torch")
    g = small_fan()
    V, R = g.n_voxels, g.n_rays
    # dense H from the oracle's projections of unit images
    H = np.zeros((R, V))
    for x in range(V):
        e = np.zeros((1, V))
        e[0, x] = 1.0
        H[:, x] = orc.forward(g, e)[0]
    assert np.abs(H).sum() > 0
    from workloads import physics as P
    I0 = P.spectra(2e3)
    mu = P.basis_mu()
    rng = np.random.default_rng(52)
    c = np.stack([rng.uniform(0.02, 0.08, V), rng.uniform(0.0, 0.02, V)])
    lbar = np.stack([H @ c[0], H @ c[1]])
    gbar = np.stack([(I0[j][:, None] * np.exp(-(mu[0][:, None] * lbar[0] + mu[1][:, None] * lbar[1]))).sum(0)
                     for j in range(2)])
    d = rng.poisson(gbar).astype(np.float64)
    mask = (rng.uniform(size=R) < 0.15).astype(np.uint8)
    Z = 2.0 * np.abs(H).sum(1).max() * np.array([mu[0].max(), mu[1].max()])
    G = rng.standard_normal((2, V))

    Ht = torch.tensor(H)
    I0t, mut = torch.tensor(I0), torch.tensor(mu)
    dt, mt = torch.tensor(d), torch.tensor(mask.astype(bool))
    ct = torch.tensor(c, requires_grad=True)
    l = ct @ Ht.T                                            # (2, R)
    e = torch.exp(-(mut[0][:, None] * l[0] + mut[1][:, None] * l[1]))   # (E, R)
    q = I0t[:, :, None] * e[None]                            # (2, E, R)
    gj = q.sum(1)                                            # (2, R)
    a = torch.stack([(mut[i][None, :, None] * q).sum(1) for i in range(2)])   # (i, j, R)
    r = torch.where(mt[None], torch.ones_like(gj), dt / gj)  # (j, R)
    wt = (r[None] * a).sum(1)                                # (i, R)
    wh = a.sum(1)
    bt = wt @ Ht
    bh = wh @ Ht
    phi = ct - torch.log(bt / bh) / torch.tensor(Z)[:, None]
    (phi * torch.tensor(G)).sum().backward()
    ref = ct.grad.numpy()
    vjp = orc.step_vjp(g, I0, mu, d, mask, Z, c, G)
    assert np.abs(vjp - ref).max() <= 1e-9 * np.abs(ref).max(), np.abs(vjp - ref).max()


def test_unrolled_chain_matches_finite_differences(orc):
    """loss = sum over non-metal voxels of (Phi^3(c0) - c_ref)^2; the gradient
    w.r.t. c0 by three step_vjp calls backwards through the stored iterates."""
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    keep = (np.asarray(inp["metal"]).reshape(-1) == 0).astype(np.float64)
    rng = np.random.default_rng(53)
    c_ref = inp["c0"] + 0.02 * rng.standard_normal(inp["c0"].shape)
    n = 3

    def loss_and_iterates(c0):
        cs = [c0]
        for _ in range(n):
            cs.append(_phi(orc, inp, mask, cs[-1]))
        return np.sum(keep * (cs[-1] - c_ref) ** 2), cs

    c0 = inp["c0"] * 0.95
    L0, cs = loss_and_iterates(c0)
    G = 2.0 * keep * (cs[-1] - c_ref)
    for k in range(n - 1, -1, -1):
        G = orc.step_vjp(g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"], cs[k], G)
    h = 1e-5
    for _ in range(3):
        e = rng.standard_normal(c0.shape)
        fd = (loss_and_iterates(c0 + h * e)[0] - loss_and_iterates(c0 - h * e)[0]) / (2 * h)
        an = np.sum(G * e)
        assert abs(fd - an) <= 1e-4 * abs(an) + 1e-8, (fd, an)
