"""MI355X (gfx950) solver for the hybrid lattice-Boltzmann colour-gradient /
finite-difference method for two-phase flow with soluble surfactants
(Ba, Liu, Li, Yang; arXiv 2311.15242).

The compute path is the HIP library ``liblbfd.so`` (C ABI in include/lbfd.h);
``lbfd.Solver`` marshals arguments and lets PyTorch own device memory and
streams.
"""
from .lbfd import FIELDS, PRECISION, LbfdError, Solver, load, workspace_bytes  # noqa: F401
