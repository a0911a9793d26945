"""Seeded synthetic workloads for the lAIR solver.

This package only builds input matrices and right-hand sides (finite
difference and discontinuous Galerkin discretisations of advection,
diffusion and reaction).  It holds none of the solver's arithmetic, so both
the CPU oracle and the GPU library may consume it.

Every generator returns a plain dict of NumPy arrays:
  ``rowptr`` int32[n+1], ``col`` int32[nnz] (sorted per row, unique, diagonal
  present), ``val`` float64[nnz], ``rhs`` float64[n] (or [n, nrhs]) and
  scalar metadata.
"""
from .fd import (upwind_transport_2d, adr_2d, adr_batch, reaction_field_2d,
                 implicit_euler_adr_3d, chain_1d, random_ff_digraph,
                 workload_c1, workload_c3, workload_c4, workload_c5)
from .dg import (dense_blocks, upwind_dg_p2, diffusion_reaction_dg_p2, workload_c2,
                 workload_dg_curved, workload_dgu)

__all__ = [
    "upwind_transport_2d", "adr_2d", "adr_batch", "reaction_field_2d",
    "implicit_euler_adr_3d", "chain_1d", "random_ff_digraph",
    "workload_c1", "workload_c2", "workload_c3", "workload_c4", "workload_c5",
    "upwind_dg_p2", "dense_blocks", "workload_dg_curved", "diffusion_reaction_dg_p2",
    "workload_dgu",
]
