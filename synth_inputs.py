"""Seeded synthetic inputs shared by the oracle tests and the GPU tests.

This module holds no arithmetic of the method: it only draws random numbers
and random group elements through numpy's generators and library
factorizations, so that both sides of a parity test can start from the same
field.  (Hot starts are not drawn here: each side draws them from its own
Philox implementation.)
"""
from __future__ import annotations

import numpy as np


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-random SU(3) matrices as complex128 [n,3,3] (QR of a complex
    Gaussian matrix with the phases of R's diagonal removed, then the
    determinant phase divided out)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def random_field(dims, seed: int) -> np.ndarray:
    """Haar-random link field in the host exchange layout
    float64 [V,4,3,3,2] (site n0 fastest, direction, row-major, re/im)."""
    V = int(np.prod(dims))
    m = random_su3(V * 4, seed).reshape(V, 4, 3, 3)
    return np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1))


def near_identity_field(dims, seed: int, eps: float) -> np.ndarray:
    """Links exp(i eps H) with H a random traceless hermitian matrix per link
    (a smooth, weak-field start), float64 [V,4,3,3,2]."""
    from scipy.linalg import expm
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((V * 4, 3, 3)) + 1j * rng.standard_normal((V * 4, 3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, 1, 2)))
    h -= np.eye(3)[None] * (np.trace(h, axis1=1, axis2=2) / 3.0)[:, None, None]
    m = np.stack([expm(1j * eps * x) for x in h]).reshape(V, 4, 3, 3)
    return np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1))


def batch_betas(n: int, seed: int, lo: float = 5.9, hi: float = 6.2) -> np.ndarray:
    """Per-lattice couplings drawn uniformly in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return lo + (hi - lo) * rng.random(n)
