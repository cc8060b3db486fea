"""MI355X-native electrofreezing phase-field lattice Boltzmann hot path (arXiv:2410.06657).

Importing the package loads nothing; ``paper_2410_06657_amd.lbm`` is the binding of the
HIP library and ``paper_2410_06657_amd.inputs`` the seeded case generator.
"""
