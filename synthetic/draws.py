"""Seeded random draws: complex densities and plane-wave directions/polarisations.

Seeds follow one rule, `12117177 + 100*cfg + purpose`, with purpose
0 = a-densities, 1 = b-densities, 2 = wave directions, 3 = polarisations,
4 = sampled rows.  NumPy's PCG64 generator is used throughout.
"""

import numpy as np

SEED_BASE = 12117177
PURPOSE = {"a": 0, "b": 1, "dirs": 2, "pols": 3, "rows": 4}


def seed_for(cfg: int, purpose) -> int:
    if isinstance(purpose, str):
        purpose = PURPOSE[purpose]
    return SEED_BASE + 100 * int(cfg) + int(purpose)


def complex_normal(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """CN(0,1) draws: (N(0,1) + i N(0,1)) / sqrt(2) per entry."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) / np.sqrt(2.0)).astype(dtype)


def plane_waves(nrhs: int, seed_dirs: int, seed_pols: int):
    """Directions uniform on the unit sphere (normalised Gaussian triples) and
    polarisations p = cos(psi) e_theta + sin(psi) e_phi with psi ~ U[0, 2pi).

    Returns (dirs f64[nrhs,3], pols f64[nrhs,3]); each polarisation is a real
    unit vector orthogonal to its direction.
    """
    rd = np.random.Generator(np.random.PCG64(seed_dirs))
    d = rd.standard_normal((nrhs, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rp = np.random.Generator(np.random.PCG64(seed_pols))
    psi = rp.uniform(0.0, 2.0 * np.pi, nrhs)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    e_theta = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], 1)
    e_phi = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], 1)
    p = np.cos(psi)[:, None] * e_theta + np.sin(psi)[:, None] * e_phi
    return d, p
