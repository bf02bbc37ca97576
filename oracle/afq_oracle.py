"""FP64 CPU oracle of the phaseless AFQMC walker step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
calls it and shares no code with it.

Source: Sukurma, Schlipf, Humer, Taheridehkordi, Kresse, "Towards Large-Scale
AFQMC Calculations: Large Time Step Auxiliary-Field Quantum Monte Carlo"
(arXiv 2403.02542).  Every function below cites the section / equation it
follows.  The oracle works in float64 / complex128 throughout, loops over
walkers one at a time and uses numpy / scipy routines (matmul, slogdet,
solve, qr, eigh, expm) as single steps.

Conventions (closed shell, restricted): a walker is one complex M x N
orbital matrix Phi shared by both spins, so <Psi_T|Phi> = det(Psi_T^T Phi)^2.
Readings of the paper where it is silent or ambiguous are marked "Reading:".

Parity pins: every public function is pinned by a test in tests/ against a
brute-force Fock-space computation, a closed form, a textbook routine or an
invariant (see the test module docstrings): the weighted estimator of `run`
by Fock-space ratios and energies of distinct walkers, the phase convention
of `reorthonormalise` by Gram-Schmidt on inputs whose raw LAPACK factor has
negative diagonal entries.  The phaseless bias of a whole trajectory has no
exact value to pin against (parity of trajectories is checked step by step).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg

EXP_KRYLOV = 0
EXP_TAYLOR = 1
# EXP_BLOCK_KRYLOV = 2 (defined with block_krylov below)

# Reading (Sec. IV.C): Arnoldi stops early ("happy breakdown") when the new
# residual is negligible against the vector it was orthogonalised from.
KRYLOV_BREAKDOWN_REL = 1e-12


# --------------------------------------------------------------------------
# Setup: Sec. II.A (Eq. mbham, hstrafo, heffTOT, force_shift) and Sec. III.B
# --------------------------------------------------------------------------

def mean_field_shift(L: np.ndarray, psi_t: np.ndarray, spin: int = 2) -> np.ndarray:
    """Lbar_g = <Psi_T|L_g|Psi_T> / <Psi_T|Psi_T>  (Eq. force_shift).

    For a restricted closed-shell determinant with orthonormal orbitals both
    spins contribute tr(Psi_T^T L_g Psi_T) (spin = 2); a determinant of spin
    orbitals (spin = 1, open shell) counts each orbital once."""
    G = L.shape[0]
    out = np.empty(G)
    for g in range(G):
        out[g] = spin * np.trace(psi_t.T @ L[g] @ psi_t)
    return out


def effective_one_body(h: np.ndarray, L: np.ndarray, lbar: np.ndarray) -> np.ndarray:
    """One-body matrix that accompanies the HS-transformed two-body term.

    Reading (Eq. mbham with V = sum_g L L, Eq. hstrafo): writing the
    two-body part as (1/2) sum_g Lhat_g^2 moves -(1/2) sum_g L_g L_g into the
    one-body part; subtracting the mean field, (1/2) sum (Lhat - Lbar)^2,
    adds + sum_g Lbar_g L_g to it (and a constant, see `energy_constant`)."""
    H1 = h.copy()
    for g in range(L.shape[0]):
        H1 -= 0.5 * (L[g] @ L[g])
        H1 += lbar[g] * L[g]
    return H1


def energy_constant(e_core: float, lbar: np.ndarray) -> float:
    """Constant of the mean-field-shifted Hamiltonian: e_core - (1/2) sum Lbar^2."""
    return float(e_core - 0.5 * np.dot(lbar, lbar))


def half_step_propagator(H1: np.ndarray, tau: float) -> np.ndarray:
    """exp(-tau H1 / 2), computed exactly by diagonalisation (Sec. III.A-B)."""
    e, v = np.linalg.eigh(H1)
    return (v * np.exp(-0.5 * tau * e)) @ v.T


@dataclasses.dataclass
class Prepared:
    """Everything derived from (h, L, e_core, Psi_T, tau) once per run."""
    h: np.ndarray
    L: np.ndarray
    e_core: float
    psi_t: np.ndarray
    tau: float
    lbar: np.ndarray
    H1: np.ndarray
    B: np.ndarray
    e_const: float
    h_half: np.ndarray        # Psi_T^T h          (N, M)
    L_half: np.ndarray        # Psi_T^T L_g        (G, N, M)
    e0: float                 # fixed trial energy (Reading: E0 = E_L(Psi_T))
    spin: int = 2             # 2: closed shell, one spin block; 1: spin orbitals

    @property
    def M(self):
        return self.h.shape[0]

    @property
    def N(self):
        return self.psi_t.shape[1]

    @property
    def G(self):
        return self.L.shape[0]


def prepare(h, L, e_core, psi_t, tau, e0=None, spin=2) -> Prepared:
    """spin = 2: restricted closed shell (h, L spatial, Psi_T the doubly
    occupied orbitals).  spin = 1: open shell in a spin-orbital basis (h, L
    block-diagonal over the two spins, Psi_T the occupied spin orbitals, see
    afq_workloads.spin_orbital_system); every closed-shell factor 2 becomes 1
    and the exchange term keeps its 1/2."""
    if spin not in (1, 2):
        raise ValueError("spin must be 1 or 2")
    lbar = mean_field_shift(L, psi_t, spin)
    H1 = effective_one_body(h, L, lbar)
    B = half_step_propagator(H1, tau)
    h_half = psi_t.T @ h
    L_half = np.stack([psi_t.T @ L[g] for g in range(L.shape[0])])
    p = Prepared(h, L, float(e_core), psi_t, float(tau), lbar, H1, B,
                 energy_constant(e_core, lbar), h_half, L_half, 0.0, spin)
    if e0 is None:
        e0 = local_energy(p, psi_t.astype(complex), psi_t.astype(complex)).real
    p.e0 = float(e0)
    return p


# --------------------------------------------------------------------------
# Mixed Green's function, overlap (Eq. force_shift, hyben, eloc)
# --------------------------------------------------------------------------

def overlap(psi_t: np.ndarray, phi: np.ndarray):
    """log det(Psi_T^T Phi) (one spin) and Theta = Phi (Psi_T^T Phi)^-1.

    Returns (logdet, theta); logdet is complex with Im in (-pi, pi]."""
    O = psi_t.T @ phi
    sign, logabs = np.linalg.slogdet(O)
    if sign == 0 or not np.isfinite(logabs):
        return complex(-np.inf), None
    theta = np.linalg.solve(O.T, phi.T).T
    return complex(logabs + np.log(sign)), theta


# --------------------------------------------------------------------------
# Force bias and the one-body operator (Eq. heffTOT, force_shift; Sec. V.C)
# --------------------------------------------------------------------------

def coulomb_vector(p: Prepared, theta: np.ndarray) -> np.ndarray:
    """ell_g = <Psi_T|Lhat_g|Phi>/<Psi_T|Phi> = 2 tr(Psi_T^T L_g Theta)
    (closed shell; tr(...) for spin orbitals)."""
    G = p.G
    ell = np.empty(G, dtype=complex)
    for g in range(G):
        ell[g] = p.spin * np.trace(p.L_half[g] @ theta)
    return ell


def force_bias(p: Prepared, ell: np.ndarray):
    """f_g = -i sqrt(tau) (<Lhat_g>_mixed - Lbar_g)   (Eq. force_shift),
    then the cap of Sec. V.C: components with |f_g| >= 1 are set to zero.

    Returns (f, fbar)."""
    f = -1j * math.sqrt(p.tau) * (ell - p.lbar)
    fbar = np.where(np.abs(f) < 1.0, f, 0.0 + 0.0j)
    return f, fbar


def interaction_operator(p: Prepared, x: np.ndarray, fbar: np.ndarray):
    """A = -tau H_int (Eq. heffTOT) as an orbital matrix, plus its scalar.

    Reading: the mean-field term Lbar_g is a c-number, so
        -tau H_int = i sqrt(tau) sum_g c_g L_g  -  i sqrt(tau) sum_g c_g Lbar_g,
    with c = x - fbar.  The matrix part acts on the orbitals; the scalar
    s_mf = -i sqrt(tau) c . Lbar multiplies the determinant once.
    Also returns log I = sum_g x_g fbar_g - (1/2) fbar_g fbar_g (importance
    sampling factor after Eq. hyben; the square is complex, as printed)."""
    c = x - fbar
    st = math.sqrt(p.tau)
    A = np.zeros((p.M, p.M), dtype=complex)
    for g in range(p.G):
        A += c[g] * p.L[g]
    A *= 1j * st
    s_mf = -1j * st * np.dot(c, p.lbar)
    log_i = np.dot(x, fbar) - 0.5 * np.dot(fbar, fbar)
    return A, complex(s_mf), complex(log_i)


# --------------------------------------------------------------------------
# Exponential of the one-body operator on the orbitals (Sec. IV)
# --------------------------------------------------------------------------

def taylor(A: np.ndarray, phi: np.ndarray, k: int) -> np.ndarray:
    """taylor_k{A, Psi} = sum_{n=0..k} A^n Psi / n!   (Eq. taylor)."""
    term = phi.copy()
    out = phi.copy()
    for n in range(1, k + 1):
        term = (A @ term) / n
        out = out + term
    return out


def arnoldi(A: np.ndarray, psi: np.ndarray, k: int):
    """Orthonormal Krylov basis and projected operator (Eq. krylovsub, projham).

    k applications of A; modified Gram-Schmidt.  Returns (basis (M, j),
    Hessenberg (j, j), beta = ||psi||) with j <= k: j < k after a happy
    breakdown (the residual vanishes against ||A b_j||)."""
    M = psi.shape[0]
    beta = np.linalg.norm(psi)
    V = np.zeros((k, M), dtype=complex)      # basis vectors as rows (contiguous)
    Hk = np.zeros((k, k), dtype=complex)
    if beta == 0.0:
        return V[:0].T, Hk[:0, :0], 0.0
    V[0] = psi / beta
    for j in range(k):
        w = A @ V[j]
        wnorm = np.linalg.norm(w)
        for i in range(j + 1):
            Hk[i, j] = np.vdot(V[i], w)
            w = w - Hk[i, j] * V[i]
        if j + 1 == k:
            break
        hn = np.linalg.norm(w)
        if hn <= KRYLOV_BREAKDOWN_REL * wnorm or hn == 0.0:
            return V[:j + 1].T, Hk[:j + 1, :j + 1], beta
        Hk[j + 1, j] = hn
        V[j + 1] = w / hn
    return V.T, Hk, beta


def krylov_vector(A: np.ndarray, psi: np.ndarray, k: int) -> np.ndarray:
    """krylov_k{A, psi} = B_k exp(A_k) e_1 ||psi||   (Eq. krylov)."""
    Bk, Hk, beta = arnoldi(A, psi, k)
    if beta == 0.0:
        return np.zeros_like(psi)
    y = scipy.linalg.expm(Hk)[:, 0]
    return beta * (Bk @ y)


def krylov(A: np.ndarray, phi: np.ndarray, k: int) -> np.ndarray:
    """Non-blocked Krylov: every orbital (column) gets its own subspace."""
    out = np.empty_like(phi)
    for j in range(phi.shape[1]):
        out[:, j] = krylov_vector(A, phi[:, j], k)
    return out


def block_arnoldi(A: np.ndarray, phi: np.ndarray, k: int):
    """Block Krylov basis of span{Psi, A Psi, ..., A^(k-1) Psi} and the
    projected operator (Eq. bkrylovsub, Sec. IV.D).

    Psi = B_1 R (QR); then for j = 1..k: W = A B_j, block modified
    Gram-Schmidt against B_1..B_j gives H_ij = B_i^dag W, and (for j < k) the
    QR of the residual W = B_{j+1} H_{j+1,j}.  Returns (B_k (M, kN),
    A_k (kN, kN) block upper Hessenberg, R (N, N)).  k applications of A."""
    M, N = phi.shape
    Q, R = np.linalg.qr(phi)
    blocks = [Q]
    H = np.zeros((k * N, k * N), dtype=complex)
    for j in range(k):
        W = A @ blocks[j]
        for i in range(j + 1):
            Hij = blocks[i].conj().T @ W
            H[i * N:(i + 1) * N, j * N:(j + 1) * N] = Hij
            W = W - blocks[i] @ Hij
        if j + 1 == k:
            break
        Qn, Rn = np.linalg.qr(W)
        H[(j + 1) * N:(j + 2) * N, j * N:(j + 1) * N] = Rn
        blocks.append(Qn)
    return np.hstack(blocks), H, R


def block_krylov(A: np.ndarray, phi: np.ndarray, k: int) -> np.ndarray:
    """bkrylov_k{A, Psi} = B_k exp(A_k) E_N R   (Eq. bkrylov)."""
    Bk, Hk, R = block_arnoldi(A, phi, k)
    N = phi.shape[1]
    ENR = np.zeros((Hk.shape[0], N), dtype=complex)
    ENR[:N, :] = R
    return Bk @ (scipy.linalg.expm(Hk) @ ENR)


EXP_BLOCK_KRYLOV = 2
EXP_CHEBYSHEV = 3
# The reference of the exponential comparisons (Sec. IV.E): the dense
# exp(A) (scipy's expm), k unused.
EXP_EXACT = -1


def chebyshev_coefficient(n: int) -> float:
    """c_0 = J_0(i), c_n = 2 i^n J_n(-i) for n > 0 (Sec. IV.B), evaluated as
    printed with the Bessel function of complex argument; the imaginary
    part vanishes (to rounding) and is dropped."""
    import scipy.special
    c = scipy.special.jv(0, 1j) if n == 0 else 2.0 * (1j ** n) * scipy.special.jv(n, -1j)
    assert abs(c.imag) <= 1e-15 * max(1.0, abs(c.real))
    return float(c.real)


def chebyshev(A: np.ndarray, phi: np.ndarray, k: int) -> np.ndarray:
    """cheb_k{A, Psi} = sum_{n=0..k} c_n T_n(A) Psi with T_0 = 1, T_1 = x,
    T_n = 2 x T_{n-1} - T_{n-2} (Eq. chebpoly).  Reading: the expansion is
    applied to A as it stands (the paper gives no spectral shift or scaling)."""
    t_prev = phi.copy()
    out = chebyshev_coefficient(0) * t_prev
    if k == 0:
        return out
    t_cur = A @ phi
    out = out + chebyshev_coefficient(1) * t_cur
    for n in range(2, k + 1):
        t_next = 2.0 * (A @ t_cur) - t_prev
        out = out + chebyshev_coefficient(n) * t_next
        t_prev, t_cur = t_cur, t_next
    return out


def exponential(A, phi, method: int, k: int):
    if method == EXP_KRYLOV:
        return krylov(A, phi, k)
    if method == EXP_TAYLOR:
        return taylor(A, phi, k)
    if method == EXP_BLOCK_KRYLOV:
        return block_krylov(A, phi, k)
    if method == EXP_CHEBYSHEV:
        return chebyshev(A, phi, k)
    if method == EXP_EXACT:
        return scipy.linalg.expm(A) @ phi
    raise ValueError(f"unknown exponential method {method}")


# --------------------------------------------------------------------------
# Local energy (Eq. eloc) and its capping (Eq. enwin)
# --------------------------------------------------------------------------

def local_energy(p: Prepared, phi: np.ndarray, theta: np.ndarray) -> complex:
    """E_L = <Psi_T|H|Phi> / <Psi_T|Phi>   (Eq. eloc), Cholesky form.

    With Theta = Phi (Psi_T^T Phi)^-1 and T_g = Psi_T^T L_g Theta (N x N),
    Wick's theorem for a closed-shell pair of determinants gives
        E_L = e_core + 2 tr(Psi_T^T h Theta)
              + (1/2) sum_g (2 tr T_g)^2 - sum_g tr(T_g T_g),
    and for a pair of spin-orbital determinants (p.spin = 1)
        E_L = e_core + tr(Psi_T^T h Theta)
              + (1/2) sum_g (tr T_g)^2 - (1/2) sum_g tr(T_g T_g)."""
    s = p.spin
    e1 = s * np.trace(p.h_half @ theta)
    ej = 0.0 + 0.0j
    ek = 0.0 + 0.0j
    for g in range(p.G):
        T = p.L_half[g] @ theta
        tr = np.trace(T)
        ej += 0.5 * (s * tr) ** 2
        ek += np.sum(T * T.T)
    return complex(p.e_core + e1 + ej - 0.5 * s * ek)


def energy_window(n_electrons: int, tau: float) -> float:
    """Delta E = (1/2) sqrt(N_e / tau) + sqrt(N_e tau)   (Eq. enwin)."""
    return 0.5 * math.sqrt(n_electrons / tau) + math.sqrt(n_electrons * tau)


def capped_energy(e_loc: complex, e0: float, n_electrons: int, tau: float) -> float:
    """Eq. enwin applied to Re E_L (Reading: E_L is complex; the cap and the
    estimator use its real part; N_e counts both spins)."""
    d = energy_window(n_electrons, tau)
    return float(min(max(e_loc.real, e0 - d), e0 + d))


# --------------------------------------------------------------------------
# Weight update (Eq. wupdate, hyben, phaseless, theta; Sec. V.B, V.D)
# --------------------------------------------------------------------------

def hybrid_energy(p: Prepared, log_ratio: complex, log_i: complex) -> complex:
    """E_H = -(1/tau) log(<Psi_T|Psi_k+1>/<Psi_T|Psi_k> I) + e_const  (Eq. hyben).

    log_ratio already holds the mean-field scalar s_mf; e_const is the
    constant of the shifted Hamiltonian, which multiplies every walker by
    exp(-tau e_const)."""
    return -(log_ratio + log_i) / p.tau + p.e_const


def phaseless_factor(p: Prepared, e_h: complex, dtheta: float) -> float:
    """exp(-tau (Re E_H - E0)) max(0, cos dtheta)   (Eq. phaseless), with the
    reweighting cap of Sec. V.B: a factor of 10 or more becomes 0 (Reading:
    the cap applies to the magnitude, before the cosine)."""
    return phaseless_parts(p, e_h, dtheta)[0]


def phaseless_parts(p: Prepared, e_h: complex, dtheta: float):
    """(factor, rule): the factor of `phaseless_factor` and which rule, if
    any, made it zero: "reweight_cap" (Sec. V.B) or "phase" (cos dtheta <= 0,
    Eq. phaseless); "" otherwise."""
    arg = -p.tau * (e_h.real - p.e0)
    m = math.exp(arg) if arg < 700.0 else math.inf
    rule = ""
    if not m < 10.0:
        m = 0.0
        rule = "reweight_cap"
    c = math.cos(dtheta)
    if c <= 0.0 and rule == "":
        rule = "phase"
    return m * max(0.0, c), rule


# --------------------------------------------------------------------------
# Reorthonormalisation (Sec. IV.D: orbitals must be re-orthogonalised)
# --------------------------------------------------------------------------

def reorthonormalise(phi: np.ndarray):
    """Phi = Q R with real positive diag(R); returns (Q, sum_i log R_ii)."""
    Q, R = np.linalg.qr(phi)
    d = np.diag(R)
    ph = d / np.abs(d)
    Q = Q * ph[None, :]
    return Q, float(np.sum(np.log(np.abs(d))))


# --------------------------------------------------------------------------
# One walker step (Split-2 propagator, Sec. III.B) and a run driver
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Walker:
    phi: np.ndarray           # (M, N) complex
    logdet: complex           # log det(Psi_T^T Phi), one spin
    theta: np.ndarray         # (M, N) complex
    weight: float = 1.0
    alive: bool = True


@dataclasses.dataclass
class StepInfo:
    e_loc: complex
    e_capped: float
    e_hybrid: complex
    dtheta: float
    log_i: complex
    n_capped_f: int
    f: np.ndarray
    zeroed_by: str = ""       # rule that set a nonzero weight to 0 this step


def init_walker(p: Prepared, phi0=None) -> Walker:
    """Psi_0 = Psi_I with W_0 e^{i theta_0} = <Psi_T|Psi_I> (Sec. II.A);
    with Psi_I = Psi_T the weight is 1 and the stored log-overlap 0."""
    phi = (p.psi_t if phi0 is None else phi0).astype(complex)
    logdet, theta = overlap(p.psi_t, phi)
    return Walker(phi, logdet, theta, 1.0, theta is not None)


PROP_SPLIT2, PROP_SPLIT1, PROP_TAYLOR, PROP_CN = 0, 1, 2, 3


def full_step_propagator(H1: np.ndarray, tau: float) -> np.ndarray:
    """exp(-tau H1), exactly by diagonalisation (Split-1, Sec. III.A)."""
    e, v = np.linalg.eigh(H1)
    return (v * np.exp(-tau * e)) @ v.T


def propagate_orbitals(p: Prepared, phi: np.ndarray, A: np.ndarray, method: int, k: int,
                       prop: int = PROP_SPLIT2) -> np.ndarray:
    """The orbital update of one step with A = -tau H_int^w (Sec. III):
      Split-2 (Sec. III.B): exp(-tau H1/2) exp(A) exp(-tau H1/2) Phi,
      Split-1 (Sec. III.A): exp(-tau H1) exp(A) Phi (the interaction acts
        first: it is the right factor of the split product),
      Taylor propagator (Sec. III.C): exp(A - tau H1) Phi, the refactorised
        exp(-tau H_eff^w), with the exponential method of the step,
      Crank-Nicolson (Sec. III.D): (1 + tau H_eff / 2)^-1 (1 - tau H_eff / 2)
        Phi = (I - A_T / 2)^-1 (I + A_T / 2) Phi with A_T = A - tau H1, by a
        dense solve (no exponential).
    H1 is the effective one-body matrix of `effective_one_body`."""
    if prop == PROP_SPLIT2:
        return p.B @ exponential(A, p.B @ phi, method, k)
    if prop == PROP_SPLIT1:
        return full_step_propagator(p.H1, p.tau) @ exponential(A, phi, method, k)
    if prop == PROP_TAYLOR:
        return exponential(A - p.tau * p.H1, phi, method, k)
    if prop == PROP_CN:
        At = A - p.tau * p.H1
        eye = np.eye(p.M)
        return np.linalg.solve(eye - 0.5 * At, phi + 0.5 * (At @ phi))
    raise ValueError(f"unknown propagator {prop}")


FB_START, FB_HALF = 0, 1


def walker_step(p: Prepared, wk: Walker, x: np.ndarray, method: int, k: int,
                reorth: bool, prop: int = PROP_SPLIT2, fb_at: int = FB_START):
    """One step of one walker (Split-2 unless `prop` says otherwise):
    returns (new walker, StepInfo).

    Order: force bias at the start-of-step Green's function (Reading: the
    paper does not say where f is evaluated; fb_at = FB_HALF evaluates it at
    Phi' = exp(-tau H1/2) Phi after the first Split-2 half-step instead, the
    alternative placement), operator, the orbital update of
    `propagate_orbitals`, overlap and weight, optional reorthonormalisation,
    local energy of the new determinant.  Any f is a change of variables of
    the field integral, so both placements sample the same propagator."""
    if not wk.alive:
        e = local_energy(p, wk.phi, wk.theta)
        return wk, StepInfo(e, capped_energy(e, p.e0, p.spin * p.N, p.tau),
                            0j, 0.0, 0j, 0, np.zeros(p.G, complex))
    if fb_at == FB_HALF:
        if prop != PROP_SPLIT2:
            raise ValueError("the half-step force bias belongs to the Split-2 propagator")
        _, theta_half = overlap(p.psi_t, p.B @ wk.phi)
        ell = (coulomb_vector(p, theta_half) if theta_half is not None
               else np.full(p.G, complex(np.nan)))
    else:
        ell = coulomb_vector(p, wk.theta)
    f, fbar = force_bias(p, ell)
    A, s_mf, log_i = interaction_operator(p, x, fbar)
    phi = propagate_orbitals(p, wk.phi, A, method, k, prop)
    logdet, theta = overlap(p.psi_t, phi)
    if theta is None or not np.all(np.isfinite(theta)) or not np.isfinite(logdet):
        dead = Walker(wk.phi, wk.logdet, wk.theta, 0.0, False)
        e = local_energy(p, dead.phi, dead.theta)
        return dead, StepInfo(e, capped_energy(e, p.e0, p.spin * p.N, p.tau), 0j,
                              0.0, log_i, int(np.sum(fbar == 0)), f,
                              "frozen" if wk.weight != 0.0 else "")
    # <Psi_T|Phi> = det(Psi_T^T Phi)^spin (both spins share the determinant
    # in the closed-shell form)
    log_ratio = p.spin * (logdet - wk.logdet) + s_mf
    e_h = hybrid_energy(p, log_ratio, log_i)
    dtheta = float(log_ratio.imag)
    factor, rule = phaseless_parts(p, e_h, dtheta)
    weight = wk.weight * factor
    if wk.weight == 0.0:
        rule = ""
    if reorth:
        phi, logr = reorthonormalise(phi)
        logdet = logdet - logr
        _, theta = overlap(p.psi_t, phi)
    e = local_energy(p, phi, theta)
    n_capped = int(np.sum(np.abs(f) >= 1.0))
    return (Walker(phi, logdet, theta, weight, True),
            StepInfo(e, capped_energy(e, p.e0, p.spin * p.N, p.tau), e_h, dtheta,
                     log_i, n_capped, f, rule))


def reorth_due(step: int, every: int) -> bool:
    """Reorthonormalise at the end of global step t when (t + 1) % every == 0."""
    return every > 0 and (step + 1) % every == 0


def run(p: Prepared, walkers, fields_of_step, n_steps: int, method: int,
        k: int, reorth_every: int, step0: int = 0, e0_state: E0State = None,
        pop_every: int = 0, comb_u=None, prop: int = PROP_SPLIT2, fb_at: int = FB_START):
    """Propagate a list of walkers; fields_of_step(t) -> (W, G) array.

    Returns (walkers, history) where history[s] holds per-walker arrays of
    e_loc, weight, e_capped and the estimator (sum_w W E_L, sum_w W)
    (Sec. II.A, weighted energy of step k).  With e0_state, p.e0 follows
    `update_e0` after every step; with pop_every > 0 the population is
    comb-resampled after the estimator of every pop_every-th global step,
    comb_u(t) giving the step's uniform number (history[s]["comb"] holds
    the source indices)."""
    hist = []
    for s in range(n_steps):
        t = step0 + s
        x = fields_of_step(t)
        infos = []
        new = []
        for w, wk in enumerate(walkers):
            nw, info = walker_step(p, wk, x[w], method, k, reorth_due(t, reorth_every), prop,
                                   fb_at)
            new.append(nw)
            infos.append(info)
        walkers = new
        wts = np.array([wk.weight for wk in walkers])
        ec = np.array([i.e_capped for i in infos])
        hist.append({
            "e_loc": np.array([i.e_loc for i in infos]),
            "e_capped": ec,
            "weight": wts,
            "e_hybrid": np.array([i.e_hybrid for i in infos]),
            "dtheta": np.array([i.dtheta for i in infos]),
            "n_capped_f": np.array([i.n_capped_f for i in infos]),
            "f": np.array([i.f for i in infos]),
            "zeroed_by": [i.zeroed_by for i in infos],
            "estimator": (float(np.sum(wts * ec)), float(np.sum(wts))),
            "e0": p.e0,
            "comb": None,
        })
        if e0_state is not None:
            p.e0 = update_e0(e0_state, hist[-1]["estimator"])
        if pop_control_due(t, pop_every):
            src = comb_resample(wts, comb_u(t))
            if src is not None:
                walkers = [dataclasses.replace(walkers[i], weight=1.0) for i in src]
                hist[-1]["comb"] = src
    return walkers, hist


# --------------------------------------------------------------------------
# E0 as the running best estimate (Sec. II.A, Eq. imag_prop)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class E0State:
    """Reading: E0 of Eq. (imag_prop) is "the best estimate of the ground-
    state energy".  With updates on, E0 for the next step is the mean of the
    weighted per-step estimates E_k = sum W Ebar / sum W (Sec. II.A) over the
    last `window` steps that had weight; a step with sum W = 0 leaves E0 as
    it is.  e0 holds the current value."""
    e0: float
    window: int = 10
    recent: list = dataclasses.field(default_factory=list)


def update_e0(state: E0State, estimator) -> float:
    """Feed one step's (sum W Ebar, sum W); returns the E0 of the next step."""
    num, den = estimator
    if den > 0.0 and math.isfinite(num / den):
        state.recent.append(num / den)
        if len(state.recent) > state.window:
            state.recent.pop(0)
        total = 0.0
        for e in state.recent:
            total += e
        state.e0 = total / len(state.recent)
    return state.e0


# --------------------------------------------------------------------------
# Population control (not described in the paper)
# --------------------------------------------------------------------------

def comb_resample(weights: np.ndarray, u: float):
    """Systematic ("comb") resampling of a walker population by weight.

    Reading: the paper gives no population-control scheme; this is the
    standard comb.  With T = sum_w W_w and the running sums
    C_i = W_0 + ... + W_i (both added left to right), slot j of the new
    population copies walker i(j) = min{i : C_i > (j + u) T / n}, for one
    uniform u in [0, 1) per step.  Every copy gets weight 1 (the estimator
    is a ratio, so the scale of the weights drops out).  Returns the list of
    source indices, or None when T = 0 (an extinct population is left as
    it is)."""
    n = len(weights)
    total = 0.0
    csum = np.empty(n)
    for i in range(n):
        total += float(weights[i])
        csum[i] = total
    if not total > 0.0:
        return None
    src = []
    i = 0
    for j in range(n):
        z = (j + u) * total / n
        while i < n - 1 and not csum[i] > z:
            i += 1
        src.append(i)
    return src


def pop_control_due(step: int, every: int) -> bool:
    """Population control after global step t when (t + 1) % every == 0."""
    return every > 0 and (step + 1) % every == 0


# --------------------------------------------------------------------------
# Adjoint of the local energy and of the Coulomb vector (Eq. eloc)
# --------------------------------------------------------------------------

def local_energy_gradient(p: Prepared, theta: np.ndarray):
    """d Re E_L / d h and d Re E_L / d L_g at a fixed walker (and fixed Psi_T),
    closed shell (p.spin = 2).

    From E_L = e_core + 2 tr(Psi_T^T h Theta) + (1/2) sum_g ell_g^2
    - sum_g tr(T_g T_g):
        dE/dh_pq   = 2 (Psi_T Theta^T)_pq
        dE/dL_g,pq = ell_g 2 (Psi_T Theta^T)_pq - 2 (Psi_T T_g^T Theta^T)_pq
    Gradients are with respect to unconstrained matrix entries; real parts."""
    if p.spin != 2:
        raise ValueError("the gradients are written for the closed-shell form")
    P = p.psi_t @ theta.T                       # (M, M) complex
    gh = 2.0 * P.real
    gL = np.empty_like(p.L)
    for g in range(p.G):
        T = p.L_half[g] @ theta
        ell = 2.0 * np.trace(T)
        gL[g] = (ell * 2.0 * P - 2.0 * (p.psi_t @ (T.T @ theta.T))).real
    return gh, gL


def coulomb_vector_gradient(p: Prepared, theta: np.ndarray, d_ell: np.ndarray):
    """d/dL_g of sum_g Re(d_ell_g^* ... ) -- the adjoint of ell_g = 2 tr(Psi_T^T
    L_g Theta) with respect to the real entries of L_g, contracted with a
    real upstream gradient on Re ell and Im ell packed as complex d_ell:
        grad L_g = Re(d_ell_g) 2 Re(Psi_T Theta^T) + Im(d_ell_g) 2 Im(Psi_T Theta^T)."""
    if p.spin != 2:
        raise ValueError("the gradients are written for the closed-shell form")
    P = 2.0 * (p.psi_t @ theta.T)
    return (d_ell.real[:, None, None] * P.real[None]
            + d_ell.imag[:, None, None] * P.imag[None])
