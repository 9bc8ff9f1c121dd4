"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package builds initial states only; it contains none of the time-step
arithmetic (Hamiltonian, densities, integrator).
"""
from .configs import (Lattice, Functional, Workload, FP64, FP32, FP32_MFMA,
                      config1, config2, config3, config4, config5_systems,
                      uniform_bcs, k_order, k_of, plane_waves, bcs_uv,
                      noise_factors, phase_noise, signed_index)
from . import rng
