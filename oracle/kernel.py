"""Scalar Helmholtz Green's function and its source gradient (test infrastructure).

g(s', s) = exp(i k R) / (4 pi R), R = |s' - s|                     (eq. 2.4)
grad' g  = (i k R - 1) exp(i k R) (s' - s) / (4 pi R^3)             (gradient
            taken at the source point s', as stated after eq. 2.5)

The wavenumber of a medium with relative permittivity eps and permeability mu
is k = k0 sqrt(eps mu) with the principal square root, so that Im k >= 0 under
the exp(-i omega t) time convention (Sec. 2.1, text after eq. 2.1).

Only `tests/`, the smoke check and the CPU-baseline leg of the benchmark use
this package; the GPU library never does.
"""

import numpy as np


def wavenumber(k0: float, eps: complex, mu: complex = 1.0) -> complex:
    """k = k0 sqrt(eps mu), principal branch (Im k >= 0)."""
    return complex(k0) * np.sqrt(complex(eps) * complex(mu))


def green(k: complex, src: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    """g(src, tgt) for broadcastable arrays of 3-vectors."""
    d = np.asarray(src, dtype=np.float64) - np.asarray(tgt, dtype=np.float64)
    R = np.sqrt(np.sum(d * d, axis=-1))
    return np.exp(1j * k * R) / (4.0 * np.pi * R)


def green_grad_src(k: complex, src: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    """Gradient of g with respect to the source point, shape (..., 3)."""
    d = np.asarray(src, dtype=np.float64) - np.asarray(tgt, dtype=np.float64)
    R = np.sqrt(np.sum(d * d, axis=-1))
    f = (1j * k * R - 1.0) * np.exp(1j * k * R) / (4.0 * np.pi * R ** 3)
    return f[..., None] * d
