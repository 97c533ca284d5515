"""CPU oracle of the DG Helmholtz pressure solve -- test infrastructure only.

Plain FP64 reference implementations (C via ctypes, numpy for the solvers and
the network) that the tests, the smoke check and the CPU-baseline leg of the
benchmark compare the HIP library against.  Nothing in the product library
imports, links or calls anything here.
"""
from .core import (OR_ALL, OR_CELL, OR_FACE, Problem, build, gauss_legendre,
                   gauss_lobatto, lagrange)
from . import solvers, mlp

__all__ = ["OR_ALL", "OR_CELL", "OR_FACE", "Problem", "build",
           "gauss_legendre", "gauss_lobatto", "lagrange", "solvers", "mlp"]
