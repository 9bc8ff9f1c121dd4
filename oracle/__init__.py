"""CPU FP64 oracle of the TDSLDA time step (test infrastructure only).

Imported by the test suite, the graft smoke check and the benchmark's CPU
baseline; never by the library.
"""
from .lise_oracle import (wavenumbers, dft_matrix, dft3, k_squared, kinetic,
                          densities, external_potential, potentials, apply_h,
                          hamiltonian_of, rhs, taylor_propagate, series_step,
                          abm_update, Evolver, observables, gram,
                          ABM_P, ABM_C, ABM_M, ABM_Y)
