"""Tolerances of the FP64 parity tests that depend on the size of the compared quantity.

theta = (1/(3V)) sum_x |Delta(x)|^2 over the 9V entries of Delta. Two correct FP64 evaluations of the
same iteration (the oracle's full matrix products, the library's two-row products with the third row
rebuilt from unitarity) round each entry of Delta differently by delta ~ 1e-15 (eight O(1) link terms
per entry, unit roundoff 1.1e-16). Uncorrelated over the 9V entries, that moves theta by about
2 delta sqrt(3 theta) / sqrt(9V); near convergence (theta ~ 1e-15, entries ~ 1e-8) this, not a fixed
relative bound, sets the scale. The bound is ten times it plus 1e-10 relative for the large thetas of
the early updates.
"""
import numpy as np

DELTA_ENTRY = 1e-15


def theta_bound(theta, vol):
    theta = np.asarray(theta, dtype=np.float64)
    return 1e-10 * theta + 10.0 * 2.0 * DELTA_ENTRY * np.sqrt(3.0 * theta) / np.sqrt(9.0 * vol)
