"""MAR initialisation on the GPU (Section 2.2, Fig. 1, Eq. 4) against the
oracle: the fan-beam FBP on narrow, wide and offset geometries, NMAR on
trace runs including the detector ends, and the whole initialisation on the
128 x 128 and 512 x 512 fan-beam workloads (metal image and trace compared
exactly where the threshold decision is not within rounding of the
threshold)."""
import numpy as np
import pytest
import torch

from workloads import make_inputs, mar_params
import workloads.geometry as Gw
from tests.test_oracle_mar import offset_fan, wide_fan, _trace_mask
from tests.errors import rel_l2, rel_max

pytestmark = pytest.mark.gpu
DEV = "cuda"
# The FBP backprojection places pixels on the detector and sums in FP64 in
# both precisions; FP32 plans round only the stored filtered sinogram and the
# image (2^-24 relative each).  The ramp-filtered terms partly cancel in the
# sum over views, which amplifies the first rounding relative to the image:
# 16 units of 2^-24 of the image maximum leave room for a cancellation ratio
# of about 8 (measured errors are below 1 unit).
TOL = {"mixed": 1e-6, "fp64": 1e-12}
# The whole initialisation in FP32 plans also takes FP32 line integrals, the
# FP32 projection of the prior, NMAR and the Eq. 4 decomposition; the
# threshold decisions are compared where the oracle's value is not within
# 1e-5 of the threshold.
TOL_INIT = {"mixed": 2e-5, "fp64": 1e-10}


@pytest.fixture(scope="module")
def mo():
    from oracle import mar_oracle
    return mar_oracle


def _plan(g, I0, mu, prec):
    from paper_2202_00116_amd.plan import Plan
    return Plan(g, I0, mu, prec)


def _spectra():
    from workloads.physics import basis_mu, spectra
    return spectra(1e5), basis_mu()


def _relmax(a, b):
    return float(np.abs(np.asarray(a, float) - b).max() / np.abs(b).max())


@pytest.mark.parametrize("geo", ["fan128", "offset", "wide", "fan512"])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_fbp_matches_oracle(mo, geo, prec):
    from workloads.configs import geometry_for
    g = {"offset": offset_fan, "wide": wide_fan}.get(geo, lambda: geometry_for(geo))()
    I0, mu = _spectra()
    plan = _plan(g, I0, mu, prec)
    rng = np.random.default_rng(95)
    # smooth sinogram of an object plus noise, both channels
    k = np.arange(g.n_cols)
    prof = np.maximum(0.0, 1.0 - ((k - g.n_cols / 2) / (0.4 * g.n_cols)) ** 2) * 6.0
    p = np.stack([np.tile(prof, g.n_views), np.tile(0.8 * prof, g.n_views)])
    p = p + 0.05 * rng.standard_normal(p.shape)
    pt = torch.tensor(p, dtype=plan.dtype, device=DEV)
    ref = mo.fbp(g, pt.cpu().numpy().astype(np.float64))
    out = plan.fbp(pt).cpu().numpy()
    e = _relmax(out, ref)
    print(f"{geo} {prec}: FBP max rel err {e:.3e}")
    assert e <= TOL[prec]
    one = plan.fbp(pt[:1].contiguous()).cpu().numpy()
    assert np.array_equal(one[0], out[0])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_nmar_matches_oracle(mo, prec):
    g = Gw.fan2d(16, 1.0, 6, 40)
    I0, mu = _spectra()
    plan = _plan(g, I0, mu, prec)
    rng = np.random.default_rng(96)
    runs = [(0, 10, 17), (1, 0, 5), (2, 33, 40), (3, 12, 13), (4, 3, 9), (4, 20, 31)]
    mask = _trace_mask(g, runs)
    p = rng.uniform(0.0, 8.0, (2, g.n_rays))
    pp = rng.uniform(0.0, 8.0, (2, g.n_rays))
    pt = torch.tensor(p, dtype=plan.dtype, device=DEV)
    ppt = torch.tensor(pp, dtype=plan.dtype, device=DEV)
    ref = mo.nmar(g, pt.cpu().numpy().astype(float), mask, ppt.cpu().numpy().astype(float), 0.01)
    out = plan.nmar(pt, torch.tensor(mask, device=DEV), ppt, 0.01).cpu().numpy()
    assert _relmax(out, ref) <= (1e-6 if prec == "mixed" else 1e-15)
    off = mask == 0
    assert np.array_equal(out[:, off], pt.cpu().numpy()[:, off])
    # a fully masked view is copied
    full = np.zeros_like(mask)
    full[:g.n_cols] = 1
    out = plan.nmar(pt, torch.tensor(full, device=DEV), ppt, 0.01)
    assert torch.equal(out, pt)


@pytest.mark.parametrize("name", ["fan128", "fan512"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mar_init_matches_oracle(mo, name, prec):
    inp = make_inputs(name)
    g = inp["geom"]
    prm = mar_params(g, inp["I0"])
    ref = mo.mar_init(g, inp["I0"], inp["mu"], inp["d"], prm)
    plan = _plan(g, inp["I0"], inp["mu"], prec)
    c, M, mask = plan.mar_init(torch.tensor(inp["d"], device=DEV), prm)
    c, M, mask = c.cpu().numpy(), M.cpu().numpy(), mask.cpu().numpy()
    # threshold decisions: equal wherever the FBP value is not within the
    # precision's rounding of the threshold
    thr = prm["metal_frac"] * prm["water"][1]
    margin = np.abs(ref["mu0"][1] - thr) / thr
    sure = margin > (1e-5 if prec == "mixed" else 1e-10)
    print(f"{name} {prec}: min metal-threshold margin {margin.min():.2e}, "
          f"{int((~sure).sum())} undecided voxels")
    assert np.array_equal(M[sure], ref["M"][sure])
    if np.array_equal(M, ref["M"]):
        assert np.array_equal(mask, ref["mask"])
    e = max(rel_l2(c, ref["c"]), rel_max(c, ref["c"]))
    print(f"{name} {prec}: c rel err (L2 and element-wise) {e:.3e}, metal voxels {int(M.sum())}, "
          f"trace rays {int(mask.sum())}")
    assert e <= TOL_INIT[prec]


def test_mar_init_rejects_helical_plan():
    from paper_2202_00116_amd._lib import DeamError
    inp = make_inputs("helical_small", with_data=False)
    plan = _plan(inp["geom"], inp["I0"], inp["mu"], "mixed")
    with pytest.raises(DeamError, match="UNSUPPORTED"):
        plan.fbp(torch.zeros((1, plan.R), dtype=torch.float32, device=DEV))
    with pytest.raises(DeamError, match="UNSUPPORTED"):
        plan.mar_init(torch.zeros((2, plan.R), dtype=torch.float32, device=DEV),
                      mar_params(inp["geom"], inp["I0"]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
def test_deam_from_mar_initialisation(mo, prec, tol):
    """The 128 x 128 workload as its configuration states it: the MAR
    initialisation supplies c^0 and the metal trace, then 20 DEAM iterations;
    against the oracle doing the same from its own initialisation."""
    from oracle import oracle as O
    inp = make_inputs("fan128")
    g = inp["geom"]
    prm = mar_params(g, inp["I0"])
    ref0 = mo.mar_init(g, inp["I0"], inp["mu"], inp["d"], prm)
    ref, href = O.iterate(g, inp["I0"], inp["mu"], inp["d"], ref0["mask"], inp["Z"], ref0["c"], 20)
    plan = _plan(g, inp["I0"], inp["mu"], prec)
    d = torch.tensor(inp["d"], device=DEV)
    c, M, mask = plan.mar_init(d, prm)
    h = torch.zeros(20, dtype=torch.float64, device=DEV)
    plan.iterate(c, d, mask, inp["Z"], 20, h)
    e = max(rel_l2(c.cpu().numpy(), ref), rel_max(c.cpu().numpy(), ref))
    eh = float(np.abs(h.cpu().numpy() - href).max() / abs(href[0]))
    print(f"fan128 {prec}: DEAM from the MAR image, 20 it.: image rel {e:.3e}, objective rel {eh:.3e}")
    assert e <= tol and eh <= tol
    assert np.all(np.diff(href) < 0)


def test_fbp_at_the_channel_limit(mo):
    """4096 channels: the filter's row and kernel fill 64 KiB of LDS; one
    more channel is refused."""
    from paper_2202_00116_amd._lib import DeamError
    I0, mu = _spectra()
    g = Gw.fan2d(32, 1.0, 6, 4096)
    plan = _plan(g, I0, mu, "fp64")
    rng = np.random.default_rng(104)
    p = torch.tensor(rng.uniform(0, 2, (1, g.n_rays)), device=DEV)
    ref = mo.fbp(g, p.cpu().numpy())
    out = plan.fbp(p).cpu().numpy()
    # each filtered value sums ~2048 FP64 terms of both signs in another order
    # than the oracle: n_cols * eps (~5e-13) times the cancellation of a noise
    # sinogram
    assert _relmax(out, ref) <= 1e-11
    g2 = Gw.fan2d(32, 1.0, 6, 4097)
    plan2 = _plan(g2, I0, mu, "mixed")
    with pytest.raises(DeamError, match="UNSUPPORTED"):
        plan2.fbp(torch.zeros((1, plan2.R), dtype=torch.float32, device=DEV))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mar_init_without_metal(mo, prec):
    """A scan with no metal and some photon-starved rays: the metal image and
    the trace are empty, NMAR leaves the data alone, and c is Eq. 4 of the
    first FBP; against the oracle."""
    import dataclasses
    from workloads.configs import expected_counts, phantom_for
    from workloads.phantoms import MaterialPhantom, METALS
    inp = make_inputs("fan128", with_data=False)
    g = inp["geom"]
    ph = phantom_for("fan128")
    ph = MaterialPhantom([dataclasses.replace(o, material=o.parent) if o.material in METALS else o
                          for o in ph.objects])
    d = np.random.default_rng(106).poisson(expected_counts(g, ph, inp["I0"])).astype(np.float32)
    # a few starved rays, counted as one photon: sparse enough that their
    # streaks stay below the metal threshold (3.9 x water at the peak)
    d[:, ::4999] = 0.0
    prm = mar_params(g, inp["I0"])
    ref = mo.mar_init(g, inp["I0"], inp["mu"], d, prm)
    assert ref["M"].sum() == 0 and ref["mask"].sum() == 0
    plan = _plan(g, inp["I0"], inp["mu"], prec)
    c, M, mask = plan.mar_init(torch.tensor(d, device=DEV), prm)
    assert int(M.sum()) == 0 and int(mask.sum()) == 0
    e = max(rel_l2(c.cpu().numpy(), ref["c"]), rel_max(c.cpu().numpy(), ref["c"]))
    assert e <= TOL_INIT[prec], e
    assert np.allclose(mo.decompose(ref["mu0"], inp["I0"], inp["mu"]), ref["c"], rtol=1e-12, atol=1e-14)
