"""Pins of the oracle's penalised DEAM (Section 2.3, Eqs. 6-7):

* the potential of Eq. 7 in its convex "fair" reading: closed values, small-
  and large-argument behaviour, its derivative by central differences, and
  convexity;
* the penalty of Eq. 6 on images where it has a closed form (a constant
  image, linear ramps along x in 2D and along z in 3D, anisotropic voxels):
  neighbour set, weights 1/distance, and the double count of each pair;
* the decoupled per-voxel c-step: lambda = 0 gives the DEAM update; in the
  quadratic limit of the potential (delta -> infinity) on a constant image it
  has a closed form through the Lambert W function; in general it minimises
  the per-voxel surrogate, checked by derivative-free minimisation of the
  surrogate's values;
* the penalised iteration: lambda = 0 gives the DEAM iteration, and the
  penalised objective (masked I-divergence + R) decreases at every iteration
  (majorise-minimise).
"""
import math

import numpy as np
import pytest

from workloads import make_inputs
from tests.test_oracle_geometry import small_fan, small_box3d

DELTA = 0.01


def test_fair_potential_closed_forms(orc):
    d = DELTA
    assert orc.fair(0.0, d) == 0.0
    assert orc.fair(d, d) == pytest.approx(d * d * (1.0 - math.log(2.0)), rel=1e-14)
    t = np.array([1e-7, 3e-4, 0.004, 0.01, 0.07, 2.0])
    assert np.array_equal(orc.fair(t, d), orc.fair(-t, d))
    # near zero: t^2/2 - |t|^3/(3 delta) + ..., the quadratic regime
    for x in (1e-6, 1e-5, 1e-4):
        assert abs(orc.fair(x, d) - 0.5 * x * x) <= x ** 3 / (3 * d) * 1.01 + 1e-12 * x * x
    # far from zero: delta |t| - delta^2 ln(|t|/delta) + O(delta^2), the linear regime
    big = 1e4 * d
    assert orc.fair(big, d) == pytest.approx(d * big - d * d * math.log(big / d), rel=1e-6)
    # derivative by central differences, at both regimes and across |t| = delta
    for x in (-0.3, -0.012, -1e-3, 2e-5, 0.009, 0.011, 0.5):
        h = 1e-7
        fd = (orc.fair(x + h, d) - orc.fair(x - h, d)) / (2 * h)
        assert orc.fair_d1(x, d) == pytest.approx(fd, rel=1e-6, abs=1e-12)
    # slope bounded by delta, approached for |t| >> delta
    assert orc.fair_d1(1e6 * d, d) == pytest.approx(d, rel=2e-6)
    # convex everywhere (the printed sign would be concave on |t| < delta)
    xs = np.linspace(-0.1, 0.1, 401)
    f = orc.fair(xs, d)
    assert np.all(f[:-2] - 2 * f[1:-1] + f[2:] > 0)


def _ramp_penalty_2d(nx, ny, dx, dy, a, lam, delta, fair):
    """c_i(x) = a_i * ix: x-neighbours and diagonal neighbours differ by a_i,
    y-neighbours by 0.  Ordered pairs: 2 (nx-1) ny along x, 4 (nx-1)(ny-1)
    diagonal."""
    s = 0.0
    for ai in a:
        s += (2 * (nx - 1) * ny / dx + 4 * (nx - 1) * (ny - 1) / math.hypot(dx, dy)) * fair(ai, delta)
    return lam * s


@pytest.mark.parametrize("dx,dy", [(1.0, 1.0), (0.7, 1.3)])
def test_penalty_ramp_2d_closed_form(orc, dx, dy):
    g = small_fan(nx=7, ny=5, dx=dx, dy=dy)
    V = g.n_voxels
    lam = 3.0
    assert orc.penalty(g, np.full((2, V), 0.37), lam, DELTA) == 0.0
    a = (0.004, -0.03)
    ix = np.arange(V) % g.nx
    c = np.stack([a[0] * ix, 1.0 + a[1] * ix]).astype(float)
    ref = _ramp_penalty_2d(g.nx, g.ny, dx, dy, a, lam, DELTA, lambda t, d: float(orc.fair(t, d)))
    assert orc.penalty(g, c, lam, DELTA) == pytest.approx(ref, rel=1e-12)
    # a ramp along y: swap the roles of the axes
    iy = np.arange(V) // g.nx
    c = np.stack([a[0] * iy, a[1] * iy]).astype(float)
    ref = _ramp_penalty_2d(g.ny, g.nx, dy, dx, a, lam, DELTA, lambda t, d: float(orc.fair(t, d)))
    assert orc.penalty(g, c, lam, DELTA) == pytest.approx(ref, rel=1e-12)


def test_penalty_ramp_3d_closed_form(orc):
    g = small_box3d()
    nx, ny, nz = g.nx, g.ny, g.nz
    V = g.n_voxels
    a = (0.02, 0.005)
    iz = np.arange(V) // (nx * ny)
    c = np.stack([a[0] * iz, a[1] * iz]).astype(float)
    # every neighbour one slice up or down differs by a_i: per offset (ox, oy),
    # (nx-|ox|)(ny-|oy|)(nz-1) voxels have it, in both z directions
    s = 0.0
    for ox in (-1, 0, 1):
        for oy in (-1, 0, 1):
            w = 1.0 / math.sqrt((ox * g.dx) ** 2 + (oy * g.dy) ** 2 + g.dz ** 2)
            s += 2 * (nx - abs(ox)) * (ny - abs(oy)) * (nz - 1) * w
    # ordered pairs (x, x~) with a z step: check the count of the sum above
    n_ordered = sum(2 * (nx - abs(ox)) * (ny - abs(oy)) * (nz - 1)
                    for ox in (-1, 0, 1) for oy in (-1, 0, 1))
    assert n_ordered == 2 * (nz - 1) * (3 * nx - 2) * (3 * ny - 2)
    ref = s * sum(float(orc.fair(ai, DELTA)) for ai in a)
    assert orc.penalty(g, c, 1.0, DELTA) == pytest.approx(ref, rel=1e-12)


def _random_b(rng, V, frac_skip=0.1):
    b = rng.uniform(5e4, 2e5, (4, V))
    b[0, rng.uniform(size=V) < frac_skip] = 0.0     # voxels the update leaves alone
    b[3, rng.uniform(size=V) < frac_skip] = -1.0
    return b


@pytest.mark.parametrize("geo", [small_fan, small_box3d])
def test_update_pen_lambda_zero_is_deam_update(orc, geo):
    g = geo()
    rng = np.random.default_rng(71)
    V = g.n_voxels
    b = _random_b(rng, V)
    c = np.stack([rng.uniform(0.0, 1.0, V), rng.uniform(0.0, 0.1, V)])
    Z = np.array([8.57, 75.97])
    ref = orc.update(b, Z, c)
    out = orc.update_pen(g, b, Z, 0.0, DELTA, c)
    assert np.abs(out - ref).max() <= 1e-15 + 1e-13 * np.abs(ref).max()
    skip = ~((b[:2] > 0) & (b[2:] > 0))
    assert np.array_equal(out[skip], c[skip])


def _weight_sums(g):
    """sum over N_x of 1/distance, by shifting an indicator of the grid."""
    ones = np.ones((g.nz, g.ny, g.nx))
    P = np.pad(ones, 1)
    W = np.zeros_like(ones)
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                if (ox, oy, oz) == (0, 0, 0):
                    continue
                dist = math.sqrt((ox * g.dx) ** 2 + (oy * g.dy) ** 2 + (oz * g.dz) ** 2)
                W += P[1 + oz:1 + oz + g.nz, 1 + oy:1 + oy + g.ny, 1 + ox:1 + ox + g.nx] / dist
    return W.reshape(-1)


@pytest.mark.parametrize("geo", [small_fan, small_box3d])
def test_update_pen_quadratic_limit_lambert_w(orc, geo):
    """Constant c^k and delta -> infinity (phi(t) -> t^2/2): the step D = c - c^k
    solves b~ - b^ exp(-Z D) + 4 lambda W D = 0 with W = sum of the weights,
    i.e. D = u/Z - b~/a with a = 4 lambda W and u = W0((b^ Z / a) exp(Z b~ / a))."""
    lambertw = pytest.importorskip("scipy.special").lambertw
    g = geo()
    rng = np.random.default_rng(72)
    V = g.n_voxels
    b = rng.uniform(5e4, 2e5, (4, V))
    Z = np.array([8.57, 75.97])
    c0 = np.array([0.6, 0.03])
    c = np.repeat(c0[:, None], V, axis=1)
    W = _weight_sums(g)
    for lam in (3e4, 4e5):
        out = orc.update_pen(g, b, Z, lam, 1e9, c)
        for i in range(2):
            a = 4.0 * lam * W
            u = lambertw(b[2 + i] * Z[i] / a * np.exp(Z[i] * b[i] / a)).real
            D = u / Z[i] - b[i] / a
            got = out[i] - c0[i]
            assert np.abs(got - D).max() <= 1e-8 * np.abs(D).max() + 1e-14
            # the penalty pulls the step towards zero compared with the DEAM step
            Du = -np.log(b[i] / b[2 + i]) / Z[i]
            assert np.all(np.abs(got) <= np.abs(Du) + 1e-15)


def _voxel_surrogate(g, x, i, b, Z, lam, delta, c, fair):
    """The per-voxel c-step objective as a function of the new value, with the
    neighbour set and weights taken from the definition (offsets in {-1,0,1}^3
    inside the grid, 1 / physical distance)."""
    nx, ny, nz = g.nx, g.ny, g.nz
    ix, iy, iz = x % nx, (x // nx) % ny, x // (nx * ny)
    ck = c[i, x]
    terms = []
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                if (ox, oy, oz) == (0, 0, 0):
                    continue
                jx, jy, jz = ix + ox, iy + oy, iz + oz
                if not (0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz):
                    continue
                w = 1.0 / math.sqrt((ox * g.dx) ** 2 + (oy * g.dy) ** 2 + (oz * g.dz) ** 2)
                terms.append((w, c[i, (jz * ny + jy) * nx + jx]))
    bt, bh = b[i, x], b[2 + i, x]

    def f(v):
        s = bt * v + bh / Z[i] * math.exp(-Z[i] * (v - ck))
        return s + lam * sum(w * fair(2 * v - ck - cn, delta) for w, cn in terms)
    return f


@pytest.mark.parametrize("geo", [small_fan, small_box3d])
@pytest.mark.parametrize("lam,delta", [(2e4, 0.01), (5e5, 0.002)])
def test_update_pen_minimises_voxel_surrogate(orc, geo, lam, delta):
    minimize_scalar = pytest.importorskip("scipy.optimize").minimize_scalar
    g = geo()
    rng = np.random.default_rng(73)
    V = g.n_voxels
    b = rng.uniform(5e4, 2e5, (4, V))
    c = np.stack([rng.uniform(0.2, 1.0, V), rng.uniform(0.0, 0.1, V)])
    Z = np.array([8.57, 75.97])
    out = orc.update_pen(g, b, Z, lam, delta, c)
    fair = lambda t, d: float(orc.fair(t, d))
    moved = 0
    for x in rng.choice(V, 24, replace=False):
        for i in range(2):
            f = _voxel_surrogate(g, x, i, b, Z, lam, delta, c, fair)
            v = out[i, x]
            res = minimize_scalar(f, bounds=(v - 0.5, v + 0.5), method="bounded",
                                  options={"xatol": 1e-13, "maxiter": 2000})
            assert abs(res.x - v) <= 2e-6, (x, i, res.x, v)
            for h in (1e-5, 1e-4):
                assert f(v) <= min(f(v - h), f(v + h))
            Du = -math.log(b[i, x] / b[2 + i, x]) / Z[i]
            moved += abs((v - c[i, x]) - Du) > 1e-4 * abs(Du)
    assert moved > 10      # the penalty changes the step


def test_iterate_pen_lambda_zero_matches_iterate(orc):
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    args = (g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"])
    c1, h1 = orc.iterate(*args, inp["c0"], 3)
    c2, h2 = orc.iterate_pen(*args, 0.0, DELTA, inp["c0"], 3)
    assert np.abs(c2 - c1).max() <= 1e-12 * np.abs(c1).max()
    assert np.allclose(h2, h1, rtol=1e-13)


@pytest.mark.parametrize("lam,delta", [(2e5, 0.005), (2e6, 0.02)])
def test_penalised_objective_decreases(orc, lam, delta):
    inp = make_inputs("fan64")
    g = inp["geom"]
    mask = orc.metal_trace(g, inp["metal"], inp["t"])[0]
    args = (g, inp["I0"], inp["mu"], inp["d"], mask, inp["Z"])
    n = 6
    c, hist = orc.iterate_pen(*args, lam, delta, inp["c0"], n)
    final = orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, c) + orc.penalty(g, c, lam, delta)
    seq = np.append(hist, final)
    print(lam, delta, seq)
    assert np.all(np.diff(seq) < 0)
    # the history is the masked I-divergence plus R at each iterate
    assert hist[0] == pytest.approx(orc.objective(g, inp["I0"], inp["mu"], inp["d"], mask, inp["c0"])
                                    + orc.penalty(g, inp["c0"], lam, delta), rel=1e-12)
    # and the penalty lowers the roughness of the result compared with DEAM
    cu, _ = orc.iterate(*args, inp["c0"], n)
    assert orc.penalty(g, c, 1.0, delta) < orc.penalty(g, cu, 1.0, delta)
