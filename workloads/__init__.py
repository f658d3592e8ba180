"""Seeded synthetic inputs for the chi0 build.

This package only draws and prepares inputs: real-space wavefunctions on the
FFT grid, band energies, G-sphere Miller indices and complex frequencies.  It
holds none of the chi0 arithmetic (no pair products, transforms, energy
factors or contractions), so that the CPU oracle and the device path can both
consume the same bytes without sharing any of the method's code.
"""
from .gen import (  # noqa: F401
    Problem,
    gsphere,
    gsphere_shifted,
    orthonormal_bands,
    band_energies,
    frequencies,
    make_problem,
    make_config,
    make_batched_config,
    CONFIG_SHAPES,
)
