"""Seeded synthetic inputs for the SU(2) two-site H.psi path.

This subpackage is the only code shared by the oracle and the library
tests: it draws integrals, builds reduced block operators (exactly, from
the Fock space of small blocks, or at random with the right selection
rules for large blocks) and random starting vectors.  It contains no part
of the H.psi contraction itself.
"""
from .integrals import make_integrals, middle_bond
from .problem import Problem, BlockData, exact_problem, random_problem

__all__ = ["make_integrals", "middle_bond", "Problem", "BlockData",
           "exact_problem", "random_problem"]
