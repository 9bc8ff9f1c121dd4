"""CPU FP64 oracle of the TDSLDA time step (test infrastructure only).

Imported by the test suite, the smoke check of the entry module and the benchmark's CPU
baseline; never by the library.
"""
from .lise_oracle import (wavenumbers, dft_matrix, dft3, k_squared, kinetic,
                          densities, external_potential, potentials, apply_h,
                          hamiltonian_of, rhs, taylor_propagate, series_step,
                          abm_update, Evolver, observables, gram, lattice_K,
                          effective_coupling, quasiparticle_energies, apply_h_shifted,
                          derivative_matrix, gradient, current_density, kick,
                          ABM_P, ABM_C, ABM_M, ABM_Y)
