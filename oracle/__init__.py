"""CPU FP64 oracle of the coupled level-set lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use it; the product path never does.
"""
from .oracle import Oracle, TangentOracle, lattice, feq, refill_weights, heaviside, geometry, \
    advect_rate, advect, reinit, extend, build, LIB_PATH, cumulants_points, moments_from_cumulants, \
    cumulant_collide, RefineOracle, refill, TwoPhaseRefineOracle  # noqa: F401
