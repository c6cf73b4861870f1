"""MI355X-native (gfx950, HIP) hot path of a weakly-compressible SPH solver
with the dummy-particle wall treatment of Rezavand, Zhang & Hu (arXiv
2110.02621): cell-list build, density reinitialisation, wall pressure,
Riemann continuity and momentum sweeps, kick-drift-kick integration.

Importing the package loads nothing; ``paper_2110_02621_amd.solver`` loads
the compiled C-ABI library and raises if it is missing.
"""
__all__ = ["scenes", "solver"]
