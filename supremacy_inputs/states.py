"""Seeded random state vectors and Haar-random unitaries (inputs only)."""
from __future__ import annotations

import numpy as np


def random_state(n: int, seed: int, normalize: bool = True) -> np.ndarray:
    """Complex Gaussian vector of 2^n amplitudes (complex128), optionally
    scaled to unit norm."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    if normalize:
        v /= np.sqrt(np.vdot(v, v).real)
    return v.astype(np.complex128)


def haar_unitary(k: int, seed: int) -> np.ndarray:
    """Haar-distributed U(2^k): QR of a complex Ginibre matrix with the phases
    of R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    d = 2 ** k
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return np.ascontiguousarray(q * ph[None, :])
