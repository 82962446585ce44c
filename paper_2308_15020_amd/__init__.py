"""MI355X (gfx950) hot path of gradient-driven continuous local search for
hybrid SAT: the Walsh-expansion objective of OR / XOR / at-least-t
constraints and its gradient for a batch of restarts, evaluated through
elementary symmetric polynomials at roots of unity, behind the C ABI of
``libffsat.so`` (include/ffsat.h)."""
from ._lib import FFSatError, FLAG_DEBUG_CHECKS, FLAG_FORCE_DFT, FLAG_UNIT_CIRCLE, MAX_CONSTRAINT_LEN, lib  # noqa: F401
from .api import Plan, Problem, coefficients, unit_circle_coefficients, walsh_coefficients  # noqa: F401

__all__ = ["Problem", "Plan", "FFSatError", "coefficients", "walsh_coefficients", "unit_circle_coefficients",
           "lib", "FLAG_FORCE_DFT", "FLAG_DEBUG_CHECKS", "FLAG_UNIT_CIRCLE", "MAX_CONSTRAINT_LEN"]
