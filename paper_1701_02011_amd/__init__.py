"""MI355X-native hot path of DSRG-MRPT3 (arXiv:1701.02011).

The computation lives in libdsrg.so (HIP kernels for gfx950 behind a C ABI, see
include/dsrg.h).  ``paper_1701_02011_amd._lib`` is its thin Python binding and
``paper_1701_02011_amd.synth`` draws seeded synthetic inputs.  Importing the package
loads nothing; the binding loads the library on first use and raises if it is missing.
"""
__version__ = "0.1.0"
