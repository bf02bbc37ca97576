"""Brute-force second quantisation for tiny systems (test-only helper).

Jordan-Wigner creation / annihilation matrices for 2M spin orbitals
(mode index sigma * M + p), Slater determinants built by applying creation
operators to the vacuum, and the many-body Hamiltonian of Eq. (mbham)
built term by term from its definition.  Shares nothing with the oracle.
"""
import functools

import numpy as np
import scipy.sparse as sp


@functools.lru_cache(maxsize=None)
def annihilators(n_modes: int):
    """Sparse a_m, m = 0..n_modes-1, acting on the 2^n_modes Fock space.

    Basis state index = sum_m occ_m 2^m; sign = (-1)^(occupied modes < m)."""
    dim = 1 << n_modes
    ops = []
    states = np.arange(dim)
    for m in range(n_modes):
        occ = (states >> m) & 1
        src = states[occ == 1]
        dst = src ^ (1 << m)
        below = np.array([bin(s & ((1 << m) - 1)).count("1") for s in src])
        sign = np.where(below % 2 == 0, 1.0, -1.0)
        ops.append(sp.csr_matrix((sign, (dst, src)), shape=(dim, dim)))
    return ops


def one_body(mat, M):
    """sum_sigma sum_pq mat_pq a^dag_{p sigma} a_{q sigma} (sparse)."""
    a = annihilators(2 * M)
    out = None
    for s in range(2):
        for p in range(M):
            for q in range(M):
                if mat[p, q] == 0:
                    continue
                t = mat[p, q] * (a[s * M + p].T @ a[s * M + q])
                out = t if out is None else out + t
    dim = 1 << (2 * M)
    return out if out is not None else sp.csr_matrix((dim, dim))


def hamiltonian(h, L, e_core=0.0):
    """e_core + sum h_pq a^dag_p a_q + 1/2 sum V_pqrs a^dag_p a^dag_q a_s a_r,
    V_pqrs = <pq|rs> = sum_g L_g,pr L_g,qs, spin summed (sigma on p,r; tau on q,s)."""
    M = h.shape[0]
    a = annihilators(2 * M)
    V = np.einsum("gpr,gqs->pqrs", L, L)
    dim = 1 << (2 * M)
    H = one_body(h, M) + e_core * sp.identity(dim, format="csr")
    for s1 in range(2):
        for s2 in range(2):
            for p in range(M):
                for q in range(M):
                    apq = a[s1 * M + p].T @ a[s2 * M + q].T
                    for r in range(M):
                        for s in range(M):
                            v = V[p, q, r, s]
                            if v == 0:
                                continue
                            H = H + 0.5 * v * (apq @ (a[s2 * M + s] @ a[s1 * M + r]))
    return H.tocsr()


def determinant(phi_up, phi_dn=None):
    """Fock vector of prod_j c^dag_j(up) prod_j c^dag_j(dn) |0>, with
    c^dag_j(sigma) = sum_p phi_pj a^dag_{p sigma}; both spins share phi by default."""
    if phi_dn is None:
        phi_dn = phi_up
    M = phi_up.shape[0]
    a = annihilators(2 * M)
    v = np.zeros(1 << (2 * M), dtype=complex)
    v[0] = 1.0
    for s, phi in ((1, phi_dn), (0, phi_up)):
        for j in reversed(range(phi.shape[1])):
            c = sum(phi[p, j] * a[s * M + p].T for p in range(M))
            v = c @ v
    return v
