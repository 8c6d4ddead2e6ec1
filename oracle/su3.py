"""FP64 SU(3) matrix utilities for the oracle (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def dag(a):
    """Hermitian conjugate over the last two axes."""
    return np.conj(np.swapaxes(a, -1, -2))


def trace(a):
    return np.trace(a, axis1=-2, axis2=-1)


def reunitarize(m):
    """Project a near-SU(3) matrix onto SU(3) by row Gram-Schmidt.

    r1 <- r1/|r1|; r2 <- r2 - (r1^dagger r2) r1; r2 <- r2/|r2|;
    r3 <- conj(r1 x r2). The third row is fixed by unitarity and det = 1,
    which is also what makes the two-row (12-real) link storage of the
    paper's Section 2.2 possible.
    """
    r1 = m[..., 0, :]
    r2 = m[..., 1, :]
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=-1, keepdims=True))
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=-1, keepdims=True) * r1
    r2 = r2 / np.sqrt(np.sum(np.abs(r2) ** 2, axis=-1, keepdims=True))
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=-2)


def third_row(m):
    """Row 3 of an SU(3) matrix rebuilt from rows 1 and 2 (Section 2.2)."""
    return np.conj(np.cross(m[..., 0, :], m[..., 1, :]))


def expm_antihermitian(a):
    """exp(A) for anti-Hermitian A, through the eigen-decomposition of -iA."""
    w, v = np.linalg.eigh(-1j * a)
    return (v * np.exp(1j * w)[..., None, :]) @ dag(v)


def unitarity_error(u):
    eye = np.eye(3)
    return float(np.max(np.abs(u @ dag(u) - eye)))


def det_error(u):
    return float(np.max(np.abs(np.linalg.det(u) - 1.0)))
