"""Seeded synthetic inputs shared by the CPU oracle and the GPU tests.

This package only draws random numbers and lays out geometry. It holds none
of the method's arithmetic (no Hamiltonian, no Coulomb matrix, no density
matrix, no integrator coefficients): the oracle and the HIP library each
build those themselves from the raw parameters returned here.
"""
from .systems import (CONFIGS, System, make_system, lattice_system,
                      packed_system, serving_stream, with_overlap)

__all__ = ["CONFIGS", "System", "make_system", "lattice_system",
           "packed_system", "serving_stream", "with_overlap"]
