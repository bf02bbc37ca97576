"""Generators for h, L_g, the RHF trial and the auxiliary fields.

Recipe (stated once here, used everywhere):

* h: diagonal ~ U(-2, 0); each upper off-diagonal entry ~ N(0, sigma_h^2),
  mirrored.  L_g = A_g + A_g^T with every entry of A_g ~ N(0, sigma_A^2).
  One ``numpy.random.default_rng(seed)`` stream, drawn in the order
  (h diagonal, h upper triangle row by row, A_0 .. A_{G-1}).
* Trial: closed-shell mean field in the Cholesky representation,
  F[C] = h + J - K with J = 2 sum_g L_g tr(L_g D), K = sum_g L_g D L_g,
  D = C C^T; ten Roothaan iterations from the core-Hamiltonian guess with
  Fock-matrix damping 0.5; the trial is the lowest N eigenvectors of the
  last Fock matrix, each column's sign fixed so that its largest-magnitude
  entry is positive.
* Fields: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key
  (seed, system id).  Block index b = (step * W + w) * ceil(G / 4) + g // 4;
  numpy's ``Philox(counter=b)`` emits the block of counter value b + 1.
  Each 64-bit word x gives u = ((x >> 11) + 1) * 2^-53 in (0, 1]; the pairs
  (u0, u1) and (u2, u3) of a block give, by the Box-Muller transform,
  fields g, g+1 and g+2, g+3 of that walker.
* Population-control uniforms: the same generator under the key
  (seed, system id + 2^32), counter = step; u = (x >> 11) 2^-53 in [0, 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    M: int                 # orbitals
    N: int                 # electrons per spin (closed shell)
    G: int                 # Cholesky vectors
    W: int                 # walkers
    tau: float
    k: int                 # Krylov dimension / Taylor order
    steps: int
    reorth_every: int
    sigma_h: float
    sigma_A: float
    seed: int = 0


def _cfg(name, M, N, G, W, tau, k, steps, reorth, scaled, seed=0):
    s = 1.0 / math.sqrt(M) if scaled else 1.0
    return WorkloadConfig(name, M, N, G, W, tau, k, steps, reorth,
                          0.1 * s, 0.05 * s, seed)


# The five workload shapes.  The first finishes in the oracle within seconds;
# the third is the production shape the throughput metric is quoted on.
CONFIGS = {
    "c1": _cfg("c1", 24, 5, 96, 16, 0.01, 6, 20, 1, scaled=False),
    "c2": _cfg("c2", 120, 20, 600, 256, 0.05, 8, 50, 1, scaled=True),
    "c3": _cfg("c3", 300, 50, 1500, 512, 0.05, 10, 100, 5, scaled=True),
    "c5": _cfg("c5", 200, 40, 1000, 256, 0.05, 8, 30, 1, scaled=True),
}
# Time steps of the extrapolation sweep at the production shape.
C3_TAUS = (0.02, 0.05, 0.1)


@dataclasses.dataclass
class Hamiltonian:
    h: np.ndarray          # (M, M) float64, symmetric
    L: np.ndarray          # (G, M, M) float64, symmetric in the last two axes
    e_core: float = 0.0


def hamiltonian(M: int, G: int, sigma_h: float, sigma_A: float, seed=0,
                e_core: float = 0.0) -> Hamiltonian:
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    h[np.diag_indices(M)] = rng.uniform(-2.0, 0.0, size=M)
    iu = np.triu_indices(M, 1)
    h[iu] = rng.normal(0.0, sigma_h, size=iu[0].size)
    h = np.triu(h) + np.triu(h, 1).T
    L = np.empty((G, M, M))
    for g in range(G):
        a = rng.normal(0.0, sigma_A, size=(M, M))
        L[g] = a + a.T
    return Hamiltonian(h, L, e_core)


def rhf_trial(h: np.ndarray, L: np.ndarray, N: int, n_iter: int = 10,
              damping: float = 0.5) -> np.ndarray:
    """Closed-shell mean-field trial orbitals (M, N), orthonormal columns.

    A fixed number of Roothaan iterations with Fock-matrix damping from the
    core-Hamiltonian guess: C_k = lowest N eigenvectors of F_{k-1},
    F_k = damping F_{k-1} + (1 - damping) F[C_k], F[C] = h + J - K.  The
    random Cholesky vectors of these workloads have no stable aufbau RHF
    solution (neither damping nor DIIS converges), so the recipe fixes the
    iteration count instead of a tolerance; the walker step only needs an
    orthonormal determinant."""
    M = h.shape[0]
    G = L.shape[0]
    Lf = L.reshape(G, M * M)

    def occupied(F):
        _, v = np.linalg.eigh(F)
        C = v[:, :N].copy()
        idx = np.argmax(np.abs(C), axis=0)
        C *= np.sign(C[idx, np.arange(N)])
        return C

    def fock(C):
        D = C @ C.T
        J = 2.0 * (Lf.T @ (Lf @ D.reshape(-1))).reshape(M, M)
        LC = np.matmul(L, C)                       # (G, M, N)
        K = np.einsum("gpi,gqi->pq", LC, LC, optimize=True)
        return h + J - K

    F = h
    for _ in range(n_iter):
        F = damping * F + (1.0 - damping) * fock(occupied(F))
    return occupied(F)


def spin_orbital_system(h: np.ndarray, L: np.ndarray, psi_a: np.ndarray,
                        psi_b: np.ndarray):
    """The same Hamiltonian in the basis of 2M spin orbitals (alpha block,
    then beta): h and every L_g repeated on the diagonal, and the occupied
    spin orbitals of an open-shell determinant, Psi = diag(Psi_a, Psi_b)
    (M x N_a and M x N_b blocks; 2M x (N_a + N_b)).  Input layout only."""
    M, G = h.shape[0], L.shape[0]
    Na, Nb = psi_a.shape[1], psi_b.shape[1]
    h2 = np.zeros((2 * M, 2 * M))
    h2[:M, :M] = h
    h2[M:, M:] = h
    L2 = np.zeros((G, 2 * M, 2 * M))
    L2[:, :M, :M] = L
    L2[:, M:, M:] = L
    psi = np.zeros((2 * M, Na + Nb))
    psi[:M, :Na] = psi_a
    psi[M:, Na:] = psi_b
    return h2, L2, psi


def fields(seed: int, sys_id: int, step: int, n_walkers: int,
           n_chol: int) -> np.ndarray:
    """Auxiliary fields x[w, g] ~ N(0, 1) of one step, shape (W, G)."""
    nb = (n_chol + 3) // 4
    start = step * n_walkers * nb
    bitgen = np.random.Philox(key=np.array([seed, sys_id], dtype=np.uint64),
                              counter=start)
    raw = bitgen.random_raw(4 * n_walkers * nb).reshape(n_walkers, nb, 4)
    u = ((raw >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0**-53
    r = np.sqrt(-2.0 * np.log(u[..., 0::2]))       # from u0, u2
    th = 2.0 * np.pi * u[..., 1::2]                # from u1, u3
    z = np.empty((n_walkers, nb, 4))
    z[..., 0::2] = r * np.cos(th)
    z[..., 1::2] = r * np.sin(th)
    return z.reshape(n_walkers, 4 * nb)[:, :n_chol].copy()


def comb_uniform(seed: int, sys_id: int, step: int) -> float:
    """The uniform number u in [0, 1) of a population-control step: word 0
    of the Philox4x64-10 block of counter value step + 1 (numpy's counter
    convention, as for the fields) under the key (seed, sys_id + 2^32), a key
    the fields never use; u = (x >> 11) 2^-53."""
    bitgen = np.random.Philox(key=np.array([seed, sys_id + (1 << 32)], dtype=np.uint64),
                              counter=step)
    x = bitgen.random_raw(4)[0]
    return float(int(x) >> 11) * 2.0**-53


def make_system(cfg: WorkloadConfig, trial_iters: int = 10):
    """(Hamiltonian, trial) for a named configuration."""
    ham = hamiltonian(cfg.M, cfg.G, cfg.sigma_h, cfg.sigma_A, cfg.seed)
    psi = rhf_trial(ham.h, ham.L, cfg.N, n_iter=trial_iters)
    return ham, psi


@dataclasses.dataclass(frozen=True)
class UnevenBatch:
    """Many systems of uneven size propagated together: M ~ U{m_lo..m_hi},
    N = M // 6, G = 5 M, the same walker count, time step and Krylov
    dimension for all; system i uses seed i, scaled sigmas (1 / sqrt(M))
    and a trial from `trial_iters` Roothaan iterations."""
    name: str
    n_sys: int
    W: int
    tau: float
    k: int
    steps: int
    reorth_every: int
    m_lo: int = 40
    m_hi: int = 400
    seed: int = 0
    trial_iters: int = 3

    def configs(self):
        return [_cfg(f"{self.name}[{i}]", M, N, G, self.W, self.tau, self.k, self.steps,
                     self.reorth_every, scaled=True, seed=i)
                for i, (M, N, G) in enumerate(
                    uneven_batch_sizes(self.n_sys, self.m_lo, self.m_hi, self.seed))]


C4 = UnevenBatch("c4", n_sys=48, W=64, tau=0.05, k=8, steps=20, reorth_every=1)


def make_uneven_batch(batch: UnevenBatch, only=None):
    """[(config, Hamiltonian, trial)] of the batch (or of the listed systems)."""
    out = []
    for i, cfg in enumerate(batch.configs()):
        if only is not None and i not in only:
            continue
        ham, psi = make_system(cfg, trial_iters=batch.trial_iters)
        out.append((cfg, ham, psi))
    return out


def uneven_batch_sizes(n_sys: int = 48, m_lo: int = 40, m_hi: int = 400,
                       seed: int = 0):
    """Orbital counts of the uneven multi-system batch: M ~ U{m_lo..m_hi},
    N = M // 6, G = 5 M."""
    rng = np.random.default_rng(seed)
    Ms = rng.integers(m_lo, m_hi + 1, size=n_sys)
    return [(int(M), int(M) // 6, 5 * int(M)) for M in Ms]
