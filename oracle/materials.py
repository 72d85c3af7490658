"""Dielectric functions of the paper's metals, as functions of the angular
frequency (test infrastructure; FP64).

Gold follows the Drude form of Sec. 3.2; silver the Drude + two-Lorentz form of
eq. 4.1.  The silver fit prints g_D = 12.6126 and w_1 = 8.25718e5; both are read
as having lost their exponents (1.26126e14 and 8.25718e15 rad/s), and the pin of
this reading is the resonance of a small silver sphere that the paper reports
near 355 nm (Fig. 13)."""

import numpy as np

SPEED_OF_LIGHT = 2.99792458e8


def omega(lam):
    return 2.0 * np.pi * SPEED_OF_LIGHT / np.asarray(lam, dtype=np.float64)


def eps_gold(w):
    w = np.asarray(w, dtype=np.complex128)
    return 9.6 - (1.37e16) ** 2 / (w ** 2 + 1j * 1.068e14 * w)


def eps_silver(w):
    w = np.asarray(w, dtype=np.complex128)
    drude = (1.39604e16) ** 2 / (w ** 2 + 1j * w * 1.26126e14)
    lor1 = 2.23994 * (8.25718e15) ** 2 / ((8.25718e15) ** 2 - 2j * w * 1.95614e14 - w ** 2)
    lor2 = 0.222651 * (3.05707e15) ** 2 / ((3.05707e15) ** 2 - 2j * w * 8.52675e14 - w ** 2)
    return 1.17152 - drude + lor1 + lor2
