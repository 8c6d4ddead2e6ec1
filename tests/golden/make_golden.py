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

fa_landau_32x32x32x32_seed0.txt: the 32^4 headline input (seed 0, plaquette ~0.59,
Haar-random gauge transformation; Sec. 3 fixes 32^4 configurations in double
precision) driven to theta < 1e-15: theta and F before every update, the update
count, and the plaquette and functional of the oracle's final field.

fa_landau_48x48x48x8_seed0_p060.txt: the 48^3 x 8 input of the mixed-precision
workload (seed 0, plaquette ~0.60) driven to theta < 1e-15: the update count,
final theta and F, and the plaquettes of input and result.

The two large fixtures take a few minutes of host time; pass --small to write
only the 12x6x4x8 one.
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


HEADLINE_DIMS = (32, 32, 32, 32)
MIXED_DIMS = (48, 48, 48, 8)
BIG_TOL = 1e-15


def full_trajectory_fixture(dims, seed, eps, eps_name, history=True):
    """The oracle's whole solve to theta < BIG_TOL: every (theta_k, F_k) if history, the update count, the
    final theta and F, and the plaquettes of the input and of the oracle's result."""
    u = synth.make_config(dims, seed, eps)
    out, info = landau.fix(u, BIG_TOL, 100000, FA_ALPHA)
    assert info["converged"]
    lines = [
        "# Landau gauge by Fourier-accelerated steepest descent (Sec. 2), FP64 oracle, solved to theta < tol.",
        f"# input: synth.make_config({dims}, {seed}) (dims are Nx, Ny, Nz, Nt), alpha = {FA_ALPHA}",
        f"# eps {eps_name} = {eps}",
        "# written by tests/golden/make_golden.py",
        f"input_plaquette {observables.plaquette(u):.17e}",
        f"input_F {landau.functional(u):.17e}",
    ]
    if history:
        lines.append("# update  theta  F   (theta_k, F_k measured before update k + 1; update 0 is the input)")
        for k, (th, f) in enumerate(info["history"]):
            lines.append(f"{k} {th:.17e} {f:.17e}")
    lines += [
        f"tol {BIG_TOL:.1e}",
        f"iters_to_tol {info['iters']}",
        f"final_theta {info['theta']:.17e}",
        f"final_F {info['F']:.17e}",
        f"final_plaquette {observables.plaquette(out):.17e}",
    ]
    return "\n".join(lines) + "\n"


def write(name, text):
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        fh.write(text)
    print("wrote", path, flush=True)


def main():
    write(f"fa_landau_{'x'.join(map(str, FA_DIMS))}_seed{FA_SEED}.txt", fa_fixture())
    if "--small" in sys.argv:
        return
    write("fa_landau_32x32x32x32_seed0.txt",
          full_trajectory_fixture(HEADLINE_DIMS, 0, synth.EPS_P059, "EPS_P059"))
    write("fa_landau_48x48x48x8_seed0_p060.txt",
          full_trajectory_fixture(MIXED_DIMS, 0, synth.EPS_P060, "EPS_P060", history=False))


if __name__ == "__main__":
    main()
