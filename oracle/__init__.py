"""FP64 CPU oracle for the relativistic lattice-Boltzmann (RLB) step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or executes it, and
this package imports nothing from the product path.

Every function follows the dissertation "Turbulence in Two-Dimensional
Relativistic Hydrodynamic Systems with a Lattice Boltzmann Model" (Watson,
2022, arXiv:2205.04658) and cites the chapter, section, equation or appendix
it restates.  The oracle is written for clarity, not speed: plain NumPy in
float64, full 26 populations, full 4x4 energy-momentum tensor, no fusion.

Modules
-------
velocity_set  the spherical momentum set and the angular polynomials
rlb           streaming, moments, Landau matching, equilibrium, collision,
              driving term, bounce-back, the full step and its diagnostics
forcing       counter-based random numbers and the k-shell stirring field
geometry      obstacle masks (channel walls, discs)
diagnostics   energy spectrum and enstrophy
linear        the linearised single-mode update matrix used by the pins
"""
