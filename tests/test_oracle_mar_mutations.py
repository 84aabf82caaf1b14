"""The MAR-initialisation pins catch plausible mistakes: each case plants one
mistake in a copy of oracle/mar_oracle.py (on the CPU), loads it as a module
and requires that at least one pin of tests/test_oracle_mar.py fails on it."""
import importlib.util
import os
import sys
import tempfile

import numpy as np
import pytest

import tests.test_oracle_mar as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "mar_oracle.py")

MUTATIONS = {
    "ramp_odd_sign": ("g[odd] = -1.0 / (2.0 * math.pi ** 2", "g[odd] = 1.0 / (2.0 * math.pi ** 2"),
    "ramp_centre": ("g[m == 0] = 1.0 / (8.0 * dgamma * dgamma)", "g[m == 0] = 1.0 / (4.0 * dgamma * dgamma)"),
    "ramp_parallel_kernel": ("np.sin(m[odd] * dgamma) ** 2)", "(m[odd] * dgamma * 0.9) ** 2)"),
    "no_cosine_weight": ("w = g.sid * np.cos(channel_angles(g))", "w = g.sid * np.ones(g.n_cols)"),
    "distance_weight": ("out[c] += val / L2", "out[c] += val / np.sqrt(L2) / g.sid"),
    "gamma_sign": ("gam = np.arctan2(ux * vy - uy * vx,", "gam = np.arctan2(uy * vx - ux * vy,"),
    "channel_offset_sign": ("kc = 0.5 * (g.n_cols - 1) + g.col_offset", "kc = 0.5 * (g.n_cols - 1) - g.col_offset"),
    "start_angle": ("beta = g.beta0 + 2.0 * math.pi * v / g.views_per_rot",
                    "beta = 2.0 * math.pi * v / g.views_per_rot"),
    "interp_fraction": ("(1.0 - fr) * q[i0] + fr * q[i1]", "fr * q[i0] + (1.0 - fr) * q[i1]"),
    "view_weight": ("return (2.0 * math.pi / g.n_views) * out", "return (math.pi / g.n_views) * out"),
    "nmar_no_denormalise": ("np.interp(k[bad], k[~bad], pn[~bad]) * den[bad]", "np.interp(k[bad], k[~bad], pn[~bad])"),
    "nmar_unnormalised": ("pn = p[c, v] / den", "pn = p[c, v] / (eps + 1.0)"),
    "prior_bone_flattened": ('np.where(m < prm["bone_frac"] * wj, wj, m)', 'np.where(m < prm["bone_frac"] * wj, wj, wj)'),
    "prior_metal_kept": ("out[j][np.asarray(M) != 0] = wj", "pass"),
    "decompose_transposed": ("np.linalg.solve(effective_mu(I0, mu),", "np.linalg.solve(effective_mu(I0, mu).T,"),
    "line_integral_floor": ("np.maximum(d, 1.0)", "np.maximum(d, 1e-3)"),
    "metal_from_low_energy": ("(np.asarray(mu_img)[1] >=", "(np.asarray(mu_img)[0] >="),
}

PINS = [
    P.test_line_integrals,
    lambda m: P.test_fbp_centred_disk_closed_form(m, "narrow"),
    lambda m: P.test_fbp_centred_disk_closed_form(m, "wide"),
    lambda m: P.test_fbp_offcentre_blob_through_system_operator(m, "narrow"),
    lambda m: P.test_fbp_offcentre_blob_through_system_operator(m, "wide"),
    P.test_prior_and_metal_classes,
    P.test_nmar_fixed_point_and_linear_exactness,
    P.test_decompose_inverts_effective_mu,
    P.test_mar_init_reduces_metal_artifact,
]


def _load(src, name):
    d = tempfile.mkdtemp(prefix="mar_mut_")
    path = os.path.join(d, name + ".py")
    open(path, "w").write(src.replace("from . import oracle as O", "from oracle import oracle as O"))
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_pins_pass_on_the_real_oracle():
    mod = _load(open(SRC).read(), "mar_real")
    for pin in PINS:
        pin(mod)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mar_pins_catch_mutation(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    mod = _load(src.replace(old, new), "mar_mut_" + name)
    caught = None
    for i, pin in enumerate(PINS):
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, ValueError, FloatingPointError, IndexError):
            caught = i
            break
    assert caught is not None, f"no pin caught the mutation {name}"
