"""Seeded synthetic crystals for the dual-k-mesh TDA-BSE hot path.

This package is the only code shared between the FP64 CPU oracle and the
HIP path.  It produces *inputs* only: a tight-binding band structure (the
stand-in for the DFT/GW front end), random LRI coefficients, a bare
Coulomb matrix, a screened interaction W(R) on a Wigner-Seitz R set,
velocity matrix elements and random exciton blocks.  It holds none of the
BSE method's arithmetic (no Fourier interpolation of W, no pair
densities, no Hamiltonian, no Lanczos).
"""
from .crystal import (CONFIGS, SEED_BASE, Problem, make_problem, ws_rset,
                      dense_kmesh, random_block, polarisations)

__all__ = ["CONFIGS", "SEED_BASE", "Problem", "make_problem", "ws_rset",
           "dense_kmesh", "random_block", "polarisations"]
