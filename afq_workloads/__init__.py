"""Seeded synthetic workloads for the ph-AFQMC walker step.

This module only draws inputs: the one-body matrix h, the Cholesky vectors
L_g, the closed-shell trial determinant and the auxiliary fields.  It holds
none of the walker-step arithmetic (force bias, propagation, weights,
energies), so both the GPU library's tests and the CPU oracle may use it.

The paper's molecular workloads (HEAT set, water clusters, N2) need basis
sets and integrals that are not available; these generators stand in for
them with the same tensor shapes and structure: a symmetric real h, a
symmetric real L_g for every Cholesky index g (so that
<pq|rs> = sum_g L_{g,pr} L_{g,qs} is positive semidefinite, Sec. II.A),
and an orthonormal real trial with N doubly occupied orbitals.
"""
from .generate import (  # noqa: F401
    C4,
    CONFIGS,
    Hamiltonian,
    UnevenBatch,
    WorkloadConfig,
    comb_uniform,
    fields,
    hamiltonian,
    make_system,
    make_uneven_batch,
    rhf_trial,
    spin_orbital_system,
    uneven_batch_sizes,
)
