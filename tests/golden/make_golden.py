"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Only the oracle (and the seeded input generator) is called here; the HIP
library is never loaded. Run from the repository root:

    python tests/golden/make_golden.py

fa_landau_12x6x4x8_seed11.txt: one seeded synthetic configuration (near-identity
links of plaquette ~0.59 under a Haar-random gauge transformation) fixed to Landau
gauge by Fourier-accelerated steepest descent (Sec. 2: the divergence Delta, the
quality theta = sum Tr Delta Delta^dag / (3V), the functional F = sum Re Tr U / (12V),
the p^2max / p^2 filter, alpha = 0.08). It records the input's plaquette and
functional, theta and F after each of the first ten updates, and the number of
updates to theta < 1e-14 with the final theta and F.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import landau, observables  # noqa: E402
from paper_1208_1186_amd import synth  # noqa: E402

FA_DIMS = (12, 6, 4, 8)
FA_SEED = 11
FA_ALPHA = 0.08
FA_TOL = 1e-14
FA_STEPS = 10


def fa_fixture():
    u = synth.make_config(FA_DIMS, FA_SEED)
    lines = [
        "# Landau gauge by Fourier-accelerated steepest descent (Sec. 2), FP64 oracle.",
        f"# input: synth.make_config({FA_DIMS}, {FA_SEED}) (dims are Nx, Ny, Nz, Nt), alpha = {FA_ALPHA}",
        "# written by tests/golden/make_golden.py",
        f"input_plaquette {observables.plaquette(u):.17e}",
        f"input_F {landau.functional(u):.17e}",
        "# update  theta  F   (update 0 is the input)",
    ]
    ref = u
    lines.append(f"{0} {landau.theta(ref):.17e} {landau.functional(ref):.17e}")
    for k in range(1, FA_STEPS + 1):
        ref, *_ = landau.fa_step(ref, FA_ALPHA)
        lines.append(f"{k} {landau.theta(ref):.17e} {landau.functional(ref):.17e}")
    _, info = landau.fix(u, FA_TOL, 100000, FA_ALPHA)
    assert info["converged"]
    lines.append(f"tol {FA_TOL:.1e}")
    lines.append(f"iters_to_tol {info['iters']}")
    lines.append(f"final_theta {info['theta']:.17e}")
    lines.append(f"final_F {info['F']:.17e}")
    return "\n".join(lines) + "\n"


def main():
    path = os.path.join(HERE, f"fa_landau_{'x'.join(map(str, FA_DIMS))}_seed{FA_SEED}.txt")
    with open(path, "w") as fh:
        fh.write(fa_fixture())
    print("wrote", path)


if __name__ == "__main__":
    main()
