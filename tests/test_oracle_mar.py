"""Pins of the MAR-initialisation oracle (Section 2.2, Fig. 1, Eq. 4):

* line integrals: Beer-Lambert inversion and the one-photon floor;
* fan-beam FBP: a centred uniform disk from its closed-form chords is
  reconstructed at its attenuation inside and ~0 outside; an off-centre blob
  projected by the system operator (channel offset and start angle non-zero)
  comes back in place and in value;
* prior classes and the metal image at known levels;
* NMAR: a sinogram proportional to (prior projection + eps) along each view is
  a fixed point; normalised data that is linear in the channel is
  interpolated exactly across the trace (also at the detector ends, where the
  nearest value is taken); data off the trace is untouched;
* Eq. 4: the decomposition inverts the spectrum-weighted attenuation, and with
  a single energy bin it is the 2x2 solve with mu_i(E);
* the whole initialisation reduces the metal artifact: against the FBP of a
  metal-free scan of the same phantom, NMAR lowers the error near the metal.

Each pin takes the oracle module as an argument so that the mutation test can
route it to a copy with a planted mistake.
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads.geometry as Gw
from workloads import make_inputs, mar_params, phantom_for


@pytest.fixture(scope="module")
def mo():
    from oracle import mar_oracle
    return mar_oracle


def offset_fan():
    return Gw.Geometry(kind=0, nx=128, ny=128, nz=1, dx=1.0, dy=1.0, dz=1.0, n_views=180, n_rows=1,
                       n_cols=256, sid=570.0, sdd=1040.0,
                       dgamma=Gw.fan_dgamma(128, 128, 1.0, 1.0, 570.0, 256), col_offset=0.25,
                       drow_iso=1.0, beta0=0.3, views_per_rot=180.0, feed_per_rot=0.0)


def wide_fan():
    """A short source distance (a fan of about 2 x 27 degrees), where the cosine
    pre-weight and the 1/L^2 weight matter at first order."""
    return Gw.Geometry(kind=0, nx=128, ny=128, nz=1, dx=1.0, dy=1.0, dz=1.0, n_views=360, n_rows=1,
                       n_cols=384, sid=200.0, sdd=400.0,
                       dgamma=Gw.fan_dgamma(128, 128, 1.0, 1.0, 200.0, 384), col_offset=-0.3,
                       drow_iso=1.0, beta0=-0.7, views_per_rot=360.0, feed_per_rot=0.0)


def _grid(g):
    x = -0.5 * g.nx * g.dx + (np.arange(g.nx) + 0.5) * g.dx
    y = -0.5 * g.ny * g.dy + (np.arange(g.ny) + 0.5) * g.dy
    X, Y = np.meshgrid(x, y, indexing="xy")
    return X.ravel(), Y.ravel()


def test_line_integrals(mo):
    I0 = np.array([[1e4, 3e4, 0.0], [0.0, 2e4, 5e4]])
    a = np.array([[0.0, 1.5, 7.0], [0.3, 2.0, 30.0]])
    tot = I0.sum(axis=1)[:, None]
    d = tot * np.exp(-a)
    p = mo.line_integrals(d, I0)
    assert np.allclose(p[:, :2], a[:, :2], rtol=1e-13, atol=1e-13)
    # below one photon the count is taken as one
    assert p[1, 2] == pytest.approx(math.log(tot[1, 0]), rel=1e-15)
    assert mo.line_integrals(np.zeros((2, 1)), I0)[0, 0] == pytest.approx(math.log(tot[0, 0]))


@pytest.mark.parametrize("geo", ["narrow", "wide"])
def test_fbp_centred_disk_closed_form(mo, geo):
    g = Gw.fan2d(128, 1.0, 180, 256) if geo == "narrow" else wide_fan()
    r, mu0 = 40.0, 0.02
    dist = g.sid * np.abs(np.sin(mo.channel_angles(g)))   # distance of each ray from the centre
    prof = 2.0 * mu0 * np.sqrt(np.maximum(r * r - dist ** 2, 0.0))
    f = mo.fbp(g, np.tile(prof, g.n_views)[None])[0]
    X, Y = _grid(g)
    R = np.hypot(X, Y)
    inside = f[R < 30.0] / mu0
    assert abs(inside.mean() - 1.0) < 2e-3
    assert np.abs(inside - 1.0).max() < 5e-3
    # just outside the disk (further out, the aliasing of 180 views grows)
    out = np.abs(f[(R > 43.0) & (R < 46.0)])
    assert out.max() < 0.03 * mu0 and out.mean() < 0.005 * mu0


@pytest.mark.parametrize("geo", ["narrow", "wide"])
def test_fbp_offcentre_blob_through_system_operator(mo, geo):
    from oracle import oracle as O
    g = offset_fan() if geo == "narrow" else wide_fan()
    cx, cy = (-20.0, 12.0) if geo == "narrow" else (-30.0, 25.0)
    X, Y = _grid(g)
    img = 0.03 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 6.0 ** 2))
    f = mo.fbp(g, O.forward(g, img[None]))[0]
    assert np.linalg.norm(f - img) / np.linalg.norm(img) < 0.025
    assert f.max() == pytest.approx(img.max(), rel=0.01)
    w = np.where(f > 0.2 * f.max(), f, 0.0)
    assert abs((w * X).sum() / w.sum() - cx) < 0.3
    assert abs((w * Y).sum() / w.sum() - cy) < 0.3


def test_prior_and_metal_classes(mo):
    prm = dict(water=np.array([0.03, 0.025]), air_frac=0.5, bone_frac=1.5, metal_frac=5.0)
    rh = np.array([0.0, 0.2, 0.49, 0.51, 1.0, 1.49, 1.51, 3.0, 4.99, 5.01, 30.0])
    rl = np.array([6.0, 0.3, 0.45, 1.2, 0.8, 1.6, 1.4, 2.5, 0.1, 9.0, 40.0])
    mu_img = np.stack([rl * 0.03, rh * 0.025])
    M = mo.metal_image(mu_img, prm)                      # from the high-energy image only
    assert M.tolist() == [0] * 9 + [1, 1]
    pri = mo.prior(mu_img, M, prm)
    for j, (wj, r) in enumerate(zip(prm["water"], (rl, rh))):
        exp = np.where(r < 0.5, 0.0, np.where(r < 1.5, wj, r * wj))
        exp[M != 0] = wj
        assert np.allclose(pri[j], exp, rtol=1e-15, atol=0)


def _trace_mask(g, runs):
    m = np.zeros((g.n_views, g.n_cols), dtype=np.uint8)
    for v, a, b in runs:
        m[v, a:b] = 1
    return m.reshape(-1)


def test_nmar_fixed_point_and_linear_exactness(mo):
    g = Gw.fan2d(16, 1.0, 6, 40)
    rng = np.random.default_rng(91)
    R = g.n_rays
    runs = [(0, 10, 17), (1, 0, 5), (2, 33, 40), (3, 12, 13), (4, 3, 9), (4, 20, 31)]
    mask = _trace_mask(g, runs)
    eps = 0.01
    pp = rng.uniform(0.0, 3.0, (2, R))
    kappa = rng.uniform(0.5, 2.0, (2, g.n_views))
    p = np.repeat(kappa, g.n_cols, axis=1) * (pp + eps)
    out = mo.nmar(g, p, mask, pp, eps)
    assert np.allclose(out, p, rtol=1e-14, atol=0)
    # normalised data linear in the channel: exact across interior runs,
    # nearest value beyond the detector ends
    k = np.tile(np.arange(g.n_cols, dtype=float), g.n_views)
    lin = (0.3 + 0.01 * k) * (pp + eps)
    noisy = lin + rng.normal(0.0, 1.0, lin.shape) * mask          # garbage on the trace
    out = mo.nmar(g, noisy, mask, pp, eps)
    assert np.array_equal(out[:, mask == 0], noisy[:, mask == 0])
    mk = mask.reshape(g.n_views, g.n_cols)
    o = out.reshape(2, g.n_views, g.n_cols)
    L = lin.reshape(2, g.n_views, g.n_cols)
    den = (pp + eps).reshape(2, g.n_views, g.n_cols)
    for v, a, b in runs:
        if a > 0 and b < g.n_cols:
            assert np.allclose(o[:, v, a:b], L[:, v, a:b], rtol=1e-13)
        elif a == 0:
            assert np.allclose(o[:, v, a:b] / den[:, v, a:b], (0.3 + 0.01 * b), rtol=1e-13)
        else:
            assert np.allclose(o[:, v, a:b] / den[:, v, a:b], (0.3 + 0.01 * (a - 1)), rtol=1e-13)
    assert mk[5].sum() == 0 and np.array_equal(o[:, 5], noisy.reshape(o.shape)[:, 5])


def test_decompose_inverts_effective_mu(mo):
    from workloads.physics import basis_mu, spectra
    I0, mu = spectra(1e5), basis_mu()
    rng = np.random.default_rng(92)
    c = np.stack([rng.uniform(0, 1, 50), rng.uniform(0, 0.1, 50)])
    Mt = np.array([[(I0[j] * mu[i]).sum() / I0[j].sum() for i in range(2)] for j in range(2)])
    assert np.allclose(mo.effective_mu(I0, mu), Mt, rtol=1e-14)
    mu_img = np.stack([Mt[0, 0] * c[0] + Mt[0, 1] * c[1], Mt[1, 0] * c[0] + Mt[1, 1] * c[1]])
    assert np.allclose(mo.decompose(mu_img, I0, mu), c, rtol=1e-12, atol=1e-15)
    # one energy bin per spectrum: the 2x2 system of the attenuations themselves
    e1 = np.zeros_like(I0)
    e1[0, 30], e1[1, 90] = 1e5, 2e5
    A = np.array([[mu[0, 30], mu[1, 30]], [mu[0, 90], mu[1, 90]]])
    assert np.allclose(mo.decompose(A @ c, e1, mu), c, rtol=1e-12, atol=1e-15)


def test_mar_init_reduces_metal_artifact(mo):
    from workloads.configs import expected_counts
    from workloads.phantoms import MaterialPhantom, METALS
    from scipy.ndimage import distance_transform_edt
    inp = make_inputs("fan128")
    g = inp["geom"]
    ph = phantom_for("fan128")
    no_metal = MaterialPhantom([dataclasses.replace(o, material=o.parent) if o.material in METALS
                                else o for o in ph.objects])
    ref = mo.fbp(g, mo.line_integrals(expected_counts(g, no_metal, inp["I0"]), inp["I0"]))
    prm = mar_params(g, inp["I0"])
    res = mo.mar_init(g, inp["I0"], inp["mu"], inp["d"], prm)
    met = inp["metal"].reshape(g.ny, g.nx) != 0
    assert np.array_equal(res["M"] != 0, inp["metal"] != 0)     # the threshold finds the rod
    dm = distance_transform_edt(~met).ravel() * g.dx
    ring = (dm > 2) & (dm < 40) & (ref[1] > 0.5 * prm["water"][1])
    for j in range(2):
        e0 = np.sqrt(np.mean((res["mu0"][j][ring] - ref[j][ring]) ** 2))
        e1 = np.sqrt(np.mean((res["mu1"][j][ring] - ref[j][ring]) ** 2))
        assert e1 < 0.6 * e0, (j, e0, e1)
    # the trace is the projection of the thresholded metal image
    assert res["mask"].sum() > 0 and res["mask"].mean() < 0.05
