"""MI355X-native joint piston-gap Reynolds solver (HIP, gfx950, FP64).

Implements the hot path of the multi-working-condition joint analysis framework of
arXiv 2511.06824: assembly of the 9 working conditions, ASSOR-preconditioned CG on the
joint block-diagonal system with a synchronized stopping test, boundary/cavitation
treatment, force/moment integration and the finite-difference double Jacobian.  The
numerical work lives in ``lib/libgapsolve.so`` (built from ``csrc/``); ``gapsolve`` is its
ctypes binding and ``solver.JointGapSolver`` a torch-facing convenience wrapper.
"""

from . import gapsolve  # noqa: F401

__all__ = ["gapsolve"]
