"""FP64 CPU oracle of the double-MRT lattice Boltzmann step.

Test infrastructure only: the tests, the package smoke check and the
benchmark's CPU-baseline leg are its only users.
"""
