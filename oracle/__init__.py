"""Plain FP64 CPU oracle for the chi0 build.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under ``oracle/``: only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the device
library (no kernels, tables, constants or pre/post-processing); both sides
only consume the seeded inputs from ``workloads``.

Parity status of each function is stated in its docstring; every function
here is pinned by the ``-m "not gpu"`` tests against closed forms,
identities, brute force or library special cases (the paper prints no
numerical values for this path).
"""
from .chi0_oracle import (  # noqa: F401
    grid_phase,
    pair_density,
    mtxel,
    mtxel_direct,
    energy_factor,
    energy_factor_dE,
    chi0,
    chi0_entries,
    chi0_backward,
    pseudobands,
    static_subspace_basis,
    chi0_subspace,
    coulomb,
    epsilon_inverse,
    gpp_inner,
    gpp_sigma_offdiag,
)
