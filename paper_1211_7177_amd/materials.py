"""Permittivity models of the metals the paper simulates, and unit conversions.

* Gold (Sec. 3.2): a Drude model eps = 9.6 - w_p^2 / (w^2 + i w_t w) with
  w_p = 1.37e16 rad/s and w_t = 1.068e14 rad/s.
* Silver (eq. 4.1): a Drude term plus two Lorentz poles,
  eps = eps_inf - w_D^2 / (w^2 + i w g_D) + sum_L de_L w_L^2 / (w_L^2 - 2 i w d_L - w^2),
  with the fit of McMahon et al. (2009).  Two of the printed rates lost their
  powers of ten (g_D and w_1 are printed as 12.6126 and 8.25718e5); they are taken
  as 1.26126e14 and 8.25718e15 rad/s, the scale of every other rate in the fit.

Times run as e^{-i w t}, so a lossy metal has Im eps > 0.  The solver works in a
length unit of the caller's choosing: k0 = 2 pi / lambda in that unit.
"""

import numpy as np

C0 = 299_792_458.0                          # m/s

GOLD = dict(eps_inf=9.6, w_p=1.37e16, w_t=1.068e14)
SILVER = dict(eps_inf=1.17152, w_D=1.39604e16, g_D=1.26126e14,
              poles=((2.23994, 8.25718e15, 1.95614e14), (0.222651, 3.05707e15, 8.52675e14)))


def angular_frequency(wavelength_m):
    """w = 2 pi c / lambda in rad/s (vacuum wavelength in metres)."""
    return 2.0 * np.pi * C0 / np.asarray(wavelength_m, dtype=np.float64)


def gold_drude(wavelength_m):
    """Relative permittivity of gold at the vacuum wavelength (metres)."""
    w = angular_frequency(wavelength_m)
    p = GOLD
    return p["eps_inf"] - p["w_p"] ** 2 / (w * w + 1j * p["w_t"] * w)


def silver_drude_lorentz(wavelength_m):
    """Relative permittivity of silver at the vacuum wavelength (metres)."""
    w = angular_frequency(wavelength_m)
    p = SILVER
    eps = p["eps_inf"] - p["w_D"] ** 2 / (w * w + 1j * w * p["g_D"])
    for de, wl, dl in p["poles"]:
        eps = eps + de * wl * wl / (wl * wl - 2j * w * dl - w * w)
    return eps


def wavenumber(wavelength_m, length_unit_m):
    """Vacuum wavenumber k0 in inverse length units (mesh coordinates in units of length_unit_m)."""
    return 2.0 * np.pi * length_unit_m / np.asarray(wavelength_m, dtype=np.float64)


def force_newtons(force, intensity_w_m2, length_unit_m):
    """Convert a force computed for a unit-amplitude plane wave (eps0 = mu0 = 1,
    irradiance 1/2, lengths in units of length_unit_m) to newtons for a wave of
    the given irradiance: F = F_unit * eps0 |E0|^2 L^2 with eps0 |E0|^2 = 2 I / c."""
    return np.asarray(force) * (2.0 * intensity_w_m2 / C0) * length_unit_m ** 2
