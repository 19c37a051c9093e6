"""CPU oracle of the coupled D2Q9/D2Q5 porous-media MRT lattice Boltzmann step.

Test infrastructure only: imported by ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark, never by the product path.
"""
