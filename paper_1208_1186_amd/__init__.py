"""MI355X-native Landau gauge fixing (Fourier-accelerated steepest descent).

``paper_1208_1186_amd.gf`` binds the HIP library ``libgf.so`` (C ABI in
``include/gf.h``); ``paper_1208_1186_amd.synth`` generates seeded synthetic
configurations. Importing the package loads nothing; the binding loads the
library on first use and raises if it has not been built.
"""
