"""Pins of the metals' dielectric functions (CPU only)."""

import numpy as np

from oracle import materials as om
from oracle import mie

LAM = np.linspace(250e-9, 1000e-9, 301)


def _peak_nm(eps_fn, radius=15e-9, lam=np.linspace(300e-9, 700e-9, 401)):
    q = [mie.efficiencies(2 * np.pi * radius / l, np.sqrt(complex(e)))[0] for l, e in zip(lam, eps_fn(om.omega(lam)))]
    return lam[int(np.argmax(q))] * 1e9


def test_silver_sphere_resonance_near_355_nm():
    """A silver sphere of radius 15 nm has its dipole resonance near 355 nm
    (Sec. 4.2, Fig. 13).  With the printed rates taken literally (g_D = 12.6126,
    w_1 = 8.25718e5 rad/s) the extinction has no peak inside 300-700 nm."""
    assert 345.0 <= _peak_nm(om.eps_silver) <= 365.0

    def literal(w):
        w = np.asarray(w, dtype=np.complex128)
        return (1.17152 - (1.39604e16) ** 2 / (w ** 2 + 1j * w * 12.6126)
                + 2.23994 * (8.25718e5) ** 2 / ((8.25718e5) ** 2 - 2j * w * 1.95614e14 - w ** 2)
                + 0.222651 * (3.05707e15) ** 2 / ((3.05707e15) ** 2 - 2j * w * 8.52675e14 - w ** 2))
    assert _peak_nm(literal) <= 301.0


def test_passive_and_metallic_in_the_visible():
    """e^{-i w t} convention: Im eps > 0 (loss) at every wavelength; Re eps < 0 from
    450 nm on for both metals (plasmonic); eps tends to eps_inf as w grows and its
    imaginary part diverges as w -> 0 (a conductor)."""
    for f, einf in ((om.eps_gold, 9.6), (om.eps_silver, 1.17152)):
        e = f(om.omega(LAM))
        assert np.all(e.imag > 0.0)
        assert np.all(e.real[LAM >= 450e-9] < 0.0)
        assert abs(f(1e22) - einf) < 1e-8
        assert f(1e8).imag > 1e6


def test_package_models_equal_the_oracle():
    from paper_1211_7177_amd import materials as pm
    w = om.omega(LAM)
    assert np.max(np.abs(pm.gold_drude(LAM) - om.eps_gold(w)) / np.abs(om.eps_gold(w))) < 1e-13
    assert np.max(np.abs(pm.silver_drude_lorentz(LAM) - om.eps_silver(w)) / np.abs(om.eps_silver(w))) < 1e-13
    assert abs(pm.wavenumber(500e-9, 100e-9) - 2 * np.pi / 5.0) < 1e-15
    # force of one unit-amplitude wave (irradiance 1/2) on C_pr = 2: F = I C_pr / c
    ref = 1e9 * 2 * 1e-14 / 2.99792458e8
    assert abs(pm.force_newtons(1.0, 1e9, 1e-7) - ref) <= 1e-14 * ref
