"""Fast Selective Extrapolation (FaSE) on AMD Instinct MI355X (gfx950).

The compute path is the C-ABI shared library ``libsefase.so`` built from
``csrc/`` (hand-written HIP).  ``paper_2204_14194_amd.binding`` marshals
arguments into it; ``paper_2204_14194_amd.synth`` produces seeded inputs.
Importing the package loads nothing: the library is opened on first use of
the binding and raises if it is missing.
"""
__version__ = "0.1.0"
