"""FP64 CPU oracle for Landau gauge fixing by Fourier-accelerated steepest descent.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The HIP library never
calls it, links it or shares code with it; the product fails loudly when its
HIP extension is missing instead of falling back here.

The oracle is plain NumPy in float64/complex128. It follows the steps of the
method in the paper's order (Section 1: Landau gauge by steepest descent with
Fourier acceleration, after Davies et al. 1988; Section 2.2: the filter acts on
every element of Delta(x) separately, and links may be stored as their first
two rows). The paper does not print the formulas; the readings taken where it
is silent are stated per function and collected in the design notes.

Conventions: links are complex128 arrays of shape (Nt, Nz, Ny, Nx, 4, 3, 3),
``dims = (Nx, Ny, Nz, Nt)``, direction mu is array axis ``3 - mu``, all
boundaries are periodic.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force and library routines. ``mlp`` functions
are pinned by central finite differences.
"""
from . import su3, landau, observables  # noqa: F401
