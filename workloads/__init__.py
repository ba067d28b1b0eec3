"""Seeded synthetic inputs shared by the oracle and the device library.

This package only *draws* inputs: atom positions, couplings, the Gaussian-well
local potential sampled on the FFT grid, and starting blocks.  It contains none
of the eigensolver's arithmetic (no sphere, no Hamiltonian, no FFT), so the
oracle and the HIP path can both consume it without sharing method code.
"""
from .gen import (Workload, make_workload, well_potential, WORKLOADS,
                  start_block, make_kpoint_workloads, KPTS_4X4X4_IRREDUCIBLE, make_request,
                  overlap_coefficients)

__all__ = ["Workload", "make_workload", "well_potential", "WORKLOADS",
           "start_block", "make_kpoint_workloads", "KPTS_4X4X4_IRREDUCIBLE", "make_request",
           "overlap_coefficients"]
