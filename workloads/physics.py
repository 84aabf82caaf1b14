"""Energy grid, attenuation stand-in and source spectra for the synthetic scans.

The forward model (Section 2.3, Eq. 8) needs mu_i(E) of the two basis
materials (polystyrene and a 23% CaCl2 solution, Figure 5 caption) and the
spectra I0_j(E) of the low and high tube voltages (90 and 140 kVp, Section
3.1).  The tabulated attenuation data that a scanner calibration would use is
not available here, so a parametric stand-in is used: a Compton term that
follows the Klein-Nishina total cross-section and a photoelectric term that
scales as Z^3/E^3, both scaled by the electron density relative to water.
Between 20 and 140 keV no K-edge of the listed elements occurs (all lie below
10 keV), so the smooth form has the right shape.  Only the scans are
synthetic; no part of the reconstruction method lives here.
"""
from __future__ import annotations

import numpy as np

# 1-keV bins from 20 to 140 keV, point values at the bin centre.
ENERGY_KEV = np.arange(20.0, 141.0, 1.0)

# Water at 60 keV: 0.0206 /mm, split 90 % Compton / 10 % photoelectric.
_MU_WATER_60 = 0.0206
_A_COMPTON = 0.9 * _MU_WATER_60
_A_PHOTO = 0.1 * _MU_WATER_60

# (electron density relative to water, effective Z)
MATERIALS = {
    "air": (0.0, 7.6),
    "water": (1.00, 7.4),
    "fat": (0.95, 6.4),
    "cortical_bone": (1.78, 12.5),
    "trabecular_bone": (1.10, 9.5),
    "bone": (1.45, 11.5),
    "polystyrene": (1.02, 5.7),
    "cacl2_23": (1.17, 13.5),
    "titanium": (3.73, 22.0),
    "steel": (6.60, 26.0),
    "aluminium": (2.34, 13.0),
}

BASIS = ("polystyrene", "cacl2_23")


def klein_nishina(e_kev):
    """Klein-Nishina total cross-section per electron, up to the constant 2*pi*r_e^2."""
    k = np.asarray(e_kev, dtype=np.float64) / 510.99895
    l12 = np.log1p(2.0 * k)
    return ((1.0 + k) / k**2 * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l12 / k)
            + l12 / (2.0 * k) - (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2)


def mu(material: str, e_kev=ENERGY_KEV):
    """Linear attenuation coefficient (1/mm) of a material on the energy grid."""
    rho, z = MATERIALS[material]
    e = np.asarray(e_kev, dtype=np.float64)
    compton = _A_COMPTON * klein_nishina(e) / klein_nishina(60.0)
    photo = _A_PHOTO * (z / 7.4) ** 3 * (60.0 / e) ** 3
    return rho * (compton + photo)


def basis_mu(e_kev=ENERGY_KEV):
    """mu_i(E) of the two basis components, shape (2, n_energy)."""
    return np.stack([mu(m, e_kev) for m in BASIS])


def spectrum(kvp: float, i0: float, e_kev=ENERGY_KEV, filt_al_mm=2.5):
    """Photon-number spectrum: Kramers' law behind an aluminium filter,
    zero at and above the tube voltage, normalised to i0 photons per ray."""
    e = np.asarray(e_kev, dtype=np.float64)
    s = np.maximum(kvp - e, 0.0) / e * np.exp(-mu("aluminium", e) * filt_al_mm)
    return i0 * s / s.sum()


def spectra(i0: float, kvps=(90.0, 140.0), e_kev=ENERGY_KEV):
    """I0_j(E) for the low and high spectra, shape (2, n_energy)."""
    return np.stack([spectrum(k, i0, e_kev) for k in kvps])


def material_in_basis(material, I0, e_kev=ENERGY_KEV):
    """Basis fractions (c1, c2) whose attenuation best matches a material, in
    the least-squares sense over the energies where either spectrum is
    non-zero, weighted by the summed spectra (air: zero)."""
    if material == "air":
        return np.zeros(2)
    mb = basis_mu(e_kev)
    w = I0.sum(axis=0)
    keep = w > 0
    sw = np.sqrt(w[keep] / w[keep].sum())
    a = (mb[:, keep] * sw).T
    b = mu(material, e_kev)[keep] * sw
    sol, *_ = np.linalg.lstsq(a, b, rcond=None)
    return sol


def water_in_basis(I0, e_kev=ENERGY_KEV):
    """material_in_basis for water."""
    return material_in_basis("water", I0, e_kev)
