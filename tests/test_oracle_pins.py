"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the oracle function(s) it pins and the source of truth:
brute-force second quantisation (tests/fock.py), a textbook closed form, a
library routine (scipy.linalg.expm / numpy eigh), an exact special case, or
an invariant.  A plausible slip in the oracle (a dropped factor of 2, a sign
of i, a transposed T_g, a missing mean-field constant, a wrong cap) fails at
least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import fock
from oracle import afq_oracle as O


def _rand_system(M, G, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(M, M)) * 0.5
    h = h + h.T
    A = rng.normal(size=(G, M, M)) * scale
    L = A + A.transpose(0, 2, 1)
    return h, L


def _trial(M, N, seed):
    rng = np.random.default_rng(seed + 100)
    q, _ = np.linalg.qr(rng.normal(size=(M, N)))
    return q


def _rand_walker(M, N, seed):
    rng = np.random.default_rng(seed + 200)
    return rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))


# ---------------------------------------------------------------- P-1 / P-2

def test_p1_trial_energy_three_ways():
    """local_energy(Psi_T) == textbook RHF energy == Fock-space <H>."""
    M, N, G = 4, 2, 3
    h, L = _rand_system(M, G, 0)
    psi = _trial(M, N, 0)
    p = O.prepare(h, L, 0.7, psi, 0.05)
    e_chol = p.e0
    hm = psi.T @ h @ psi
    Lm = np.einsum("pi,gpq,qj->gij", psi, L, psi)
    eri = np.einsum("gij,gkl->ijkl", Lm, Lm)          # (ij|kl)
    e_text = 0.7 + 2 * np.trace(hm)
    e_text += sum(2 * eri[i, i, j, j] - eri[i, j, j, i] for i in range(N) for j in range(N))
    H = fock.hamiltonian(h, L, 0.7)
    v = fock.determinant(psi.astype(complex))
    e_fock = np.vdot(v, H @ v).real / np.vdot(v, v).real
    assert abs(e_chol - e_text) < 1e-12
    assert abs(e_chol - e_fock) < 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_p2_mixed_estimators_bruteforce(seed):
    """local_energy, coulomb_vector and overlap for arbitrary complex Phi
    against <Psi_T|O|Phi>/<Psi_T|Phi> in the 256-dim Fock space."""
    M, N, G = 4, 2, 3
    h, L = _rand_system(M, G, seed)
    psi = _trial(M, N, seed)
    phi = _rand_walker(M, N, seed)
    p = O.prepare(h, L, -0.4, psi, 0.05)
    logdet, theta = O.overlap(psi, phi)
    t = fock.determinant(psi.astype(complex))
    v = fock.determinant(phi)
    ov = np.vdot(t, v)
    assert abs(np.exp(2 * logdet) - ov) < 1e-12 * abs(ov)
    H = fock.hamiltonian(h, L, -0.4)
    e_ref = np.vdot(t, H @ v) / ov
    e = O.local_energy(p, phi, theta)
    assert abs(e - e_ref) < 1e-11 * max(1.0, abs(e_ref))
    ell = O.coulomb_vector(p, theta)
    for g in range(G):
        ref = np.vdot(t, fock.one_body(L[g], M) @ v) / ov
        assert abs(ell[g] - ref) < 1e-12 * max(1.0, abs(ref))


def test_p1_lbar_is_trial_expectation():
    M, N, G = 4, 2, 3
    _, L = _rand_system(M, G, 5)
    psi = _trial(M, N, 5)
    lbar = O.mean_field_shift(L, psi)
    t = fock.determinant(psi.astype(complex))
    for g in range(G):
        ref = np.vdot(t, fock.one_body(L[g], M) @ t).real / np.vdot(t, t).real
        assert abs(lbar[g] - ref) < 1e-12


# ---------------------------------------------------------------- P-3 / P-5

def test_p3_thouless_exponentials():
    """exp(Ahat)|Phi> == |exp(A) Phi>; krylov with k = M and high-order
    Taylor both reproduce it (Eq. krylov, taylor)."""
    M, N = 4, 2
    rng = np.random.default_rng(7)
    A = (rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))) * 0.3
    phi = _rand_walker(M, N, 7)
    Ahat = fock.one_body(A, M).toarray()
    ref = scipy.linalg.expm(Ahat) @ fock.determinant(phi)
    for out in (O.krylov(A, phi, M), O.taylor(A, phi, 40)):
        got = fock.determinant(out)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k", [2, 4, 6, 8])
def test_p5_exponential_error_bounds(k):
    """Against exp(A) by eigendecomposition; error within the a-priori bounds:
    Taylor ||A||^(k+1) e^||A|| / (k+1)!, Krylov 2 rho^k e^rho / k!
    (Saad 1992), rho = ||A||_2."""
    M, N = 24, 5
    rng = np.random.default_rng(k)
    S = rng.normal(size=(M, M))
    S = (S + S.T) / math.sqrt(4 * M)
    A = 1j * 0.6 * S + 0.05 * np.eye(M)       # the shape of -tau H_int
    w, v = np.linalg.eig(A)
    expA = (v * np.exp(w)) @ np.linalg.inv(v)
    phi = _rand_walker(M, N, k)
    ref = expA @ phi
    rho = np.linalg.norm(A, 2)
    for j in range(N):
        nrm = np.linalg.norm(phi[:, j])
        et = np.linalg.norm(O.taylor(A, phi[:, [j]], k)[:, 0] - ref[:, j])
        ek = np.linalg.norm(O.krylov_vector(A, phi[:, j], k) - ref[:, j])
        assert et <= nrm * rho ** (k + 1) * math.exp(rho) / math.factorial(k + 1) * 1.0001 + 1e-13
        assert ek <= nrm * 2 * rho ** k * math.exp(rho) / math.factorial(k) * 1.0001 + 1e-13
    full = O.krylov(A, phi, M)
    assert np.abs(full - ref).max() < 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- P-7

def test_p7_krylov_invariances():
    M = 16
    rng = np.random.default_rng(11)
    S = rng.normal(size=(M, M))
    S = S + S.T
    A = 0.2j * S
    psi = rng.normal(size=M) + 1j * rng.normal(size=M)
    k = 6
    Bk, Hk, beta = O.arnoldi(A, psi, k)
    assert np.abs(Bk.conj().T @ Bk - np.eye(k)).max() < 1e-13
    assert abs(beta - np.linalg.norm(psi)) < 1e-13
    # Arnoldi relation: B_k^dag A B_k == H_k (Eq. projham), upper Hessenberg
    assert np.abs(Bk.conj().T @ A @ Bk - Hk).max() < 1e-12
    assert np.abs(np.tril(Hk, -2)).max() == 0.0
    # norm preserved for skew-Hermitian A
    out = O.krylov_vector(A, psi, k)
    assert abs(np.linalg.norm(out) - np.linalg.norm(psi)) < 1e-12
    # shift: krylov(A + cI) = e^c krylov(A)
    c = 0.3 - 0.2j
    out2 = O.krylov_vector(A + c * np.eye(M), psi, k)
    assert np.abs(out2 - np.exp(c) * out).max() < 1e-12 * np.abs(out).max()


def test_p7_krylov_breakdown_eigenvector():
    """An eigenvector spans an invariant subspace: Arnoldi stops at j = 1 and
    the result is exact."""
    M = 10
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(M, M)))
    d = rng.normal(size=M)
    A = 0.3j * (Q * d) @ Q.T
    Bk, Hk, _ = O.arnoldi(A, Q[:, 2].astype(complex), 6)
    assert Bk.shape[1] == 1
    out = O.krylov_vector(A, Q[:, 2].astype(complex), 6)
    assert np.abs(out - np.exp(0.3j * d[2]) * Q[:, 2]).max() < 1e-14


# ---------------------------------------------------------------- P-4 / R-1

def test_r1_shifted_hamiltonian_identity():
    """H == e_const + H1_eff(hat) + 1/2 sum_g (Lhat_g - Lbar_g)^2 as Fock
    operators (pins effective_one_body, energy_constant, mean_field_shift)."""
    M, N, G = 4, 2, 2
    h, L = _rand_system(M, G, 21)
    psi = _trial(M, N, 21)
    p = O.prepare(h, L, 0.25, psi, 0.1)
    dim = 1 << (2 * M)
    H = fock.hamiltonian(h, L, 0.25).toarray()
    rhs = p.e_const * np.eye(dim) + fock.one_body(p.H1, M).toarray()
    for g in range(G):
        X = fock.one_body(L[g], M).toarray() - p.lbar[g] * np.eye(dim)
        rhs += 0.5 * X @ X
    assert np.abs(H - rhs).max() < 1e-12


def test_p4_operator_complex_symmetric():
    """interaction_operator: with symmetric L_g and complex shifts the
    operator is complex symmetric, A = A^T (not Hermitian), so its upper
    triangle mirrored is A itself, exactly -- the property the GPU's operator
    build relies on when it forms only the blocks on or above the diagonal."""
    M, N, G = 7, 3, 5
    h, L = _rand_system(M, G, seed=3)
    p = O.prepare(h, L, 0.0, _trial(M, N, 3), tau=0.05)
    rng = np.random.default_rng(9)
    x = rng.normal(size=G)
    fbar = 0.3 * (rng.normal(size=G) + 1j * rng.normal(size=G))
    A, _, _ = O.interaction_operator(p, x, fbar)
    assert np.array_equal(A, A.T)
    assert not np.allclose(A, A.conj().T)
    assert np.array_equal(np.triu(A) + np.triu(A, 1).T, A)


@pytest.mark.parametrize("method", [O.EXP_KRYLOV, O.EXP_TAYLOR])
def test_p4_importance_sampled_step_expectation(method):
    """With one Cholesky vector the HS transform is exact.  The Gauss-Hermite
    average over x of exp(-tau (E_H(x) - E0)) |Phi'(x)> / <Psi_T|Phi'(x)>
    must equal the split propagator exp(-tau(e_const - E0))
    exp(-tau H1/2) exp(-tau/2 (Lhat - Lbar)^2) exp(-tau H1/2) |Phi>/<Psi_T|Phi>.
    This pins the sign and scale of A, s_mf, the importance factor I (with a
    nonzero complex force bias), e_const and the spin factor of the ratio."""
    M, N, G = 4, 2, 1
    h, L = _rand_system(M, G, 31, scale=0.5)
    psi = _trial(M, N, 31)
    tau = 0.3
    p = O.prepare(h, L, 0.1, psi, tau)
    phi = psi + 0.3 * _rand_walker(M, N, 31)
    wk = O.init_walker(p, phi)
    ell = O.coulomb_vector(p, wk.theta)
    f, fbar = O.force_bias(p, ell)
    assert np.all(fbar == f) and abs(f[0]) > 0.05
    xs, ws = np.polynomial.hermite_e.hermegauss(90)
    ws = ws / math.sqrt(2 * math.pi)
    t = fock.determinant(psi.astype(complex))
    acc = np.zeros(1 << (2 * M), dtype=complex)
    k = M if method == O.EXP_KRYLOV else 60
    for x, wq in zip(xs, ws):
        A, s_mf, log_i = O.interaction_operator(p, np.array([x]), fbar)
        new = p.B @ O.exponential(A, p.B @ wk.phi, method, k)
        logdet, _ = O.overlap(psi, new)
        log_ratio = 2 * (logdet - wk.logdet) + s_mf
        e_h = O.hybrid_energy(p, log_ratio, log_i)
        v = fock.determinant(new)
        acc += wq * np.exp(-tau * (e_h - p.e0)) * v / np.vdot(t, v)
    dim = 1 << (2 * M)
    Bh = scipy.linalg.expm(-0.5 * tau * fock.one_body(p.H1, M).toarray())
    X = fock.one_body(L[0], M).toarray() - p.lbar[0] * np.eye(dim)
    U = math.exp(-tau * (p.e_const - p.e0)) * Bh @ scipy.linalg.expm(-0.5 * tau * X @ X) @ Bh
    v0 = fock.determinant(wk.phi)
    ref = U @ v0 / np.vdot(t, v0)
    assert np.abs(acc - ref).max() < 1e-9 * np.abs(ref).max()


# ---------------------------------------------------------------- P-6 / P-9

def _diagonal_system(M, N, G, seed):
    """h and every L_g diagonal in one random orthogonal basis; Psi_T = the N
    lowest orbitals of that basis."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(M, M)))
    eh = np.sort(rng.uniform(-2, 0, size=M))
    dl = rng.normal(size=(G, M)) * 0.2
    h = (Q * eh) @ Q.T
    L = np.stack([(Q * dl[g]) @ Q.T for g in range(G)])
    return h, L, Q[:, :N].copy()


@pytest.mark.parametrize("method", [O.EXP_KRYLOV, O.EXP_TAYLOR])
def test_p6_commuting_hamiltonian_exact(method):
    """All L_g commute with h and each other (E_HS = 0, Sec. III.A): for any
    fields f == 0, dtheta == 0, E_H == E_HF, W == 1 and E_L == E_HF."""
    M, N, G = 8, 3, 5
    h, L, psi = _diagonal_system(M, N, G, 4)
    tau = 0.2
    p = O.prepare(h, L, 0.3, psi, tau)
    rng = np.random.default_rng(9)
    wks = [O.init_walker(p) for _ in range(3)]
    k = 6 if method == O.EXP_KRYLOV else 40
    wks, hist = O.run(p, wks, lambda t: rng.normal(size=(3, G)), 5, method, k, 1)
    for hs in hist:
        assert np.abs(hs["f"]).max() < 1e-13
        assert np.abs(hs["dtheta"]).max() < 1e-12
        assert np.abs(hs["e_hybrid"] - p.e0).max() < 1e-11
        assert np.abs(hs["weight"] - 1.0).max() < 1e-11
        assert np.abs(hs["e_loc"] - p.e0).max() < 1e-11


# ---------------------------------------------------------------- P-8

def test_p8_right_multiplication_invariance():
    """Theta, E_L and overlap ratios are unchanged by Phi -> Phi R; the
    log-overlap shifts by log det R; Taylor commutes with Phi -> Phi R."""
    M, N, G = 10, 3, 6
    h, L = _rand_system(M, G, 41, scale=0.1)
    psi = _trial(M, N, 41)
    p = O.prepare(h, L, 0.0, psi, 0.05)
    phi = psi + 0.2 * _rand_walker(M, N, 41)
    rng = np.random.default_rng(2)
    R = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    l1, t1 = O.overlap(psi, phi)
    l2, t2 = O.overlap(psi, phi @ R)
    assert np.abs(t1 - t2).max() < 1e-12
    d = np.exp(l2 - l1) - np.linalg.det(R)
    assert abs(d) < 1e-12 * abs(np.linalg.det(R))
    assert abs(O.local_energy(p, phi, t1) - O.local_energy(p, phi @ R, t2)) < 1e-12
    A = 0.3j * h
    assert np.abs(O.taylor(A, phi @ R, 6) - O.taylor(A, phi, 6) @ R).max() < 1e-12
    Q, logr = O.reorthonormalise(phi)
    assert np.abs(Q.conj().T @ Q - np.eye(N)).max() < 1e-13
    lq, tq = O.overlap(psi, Q)
    assert abs((l1 - logr) - lq) < 1e-12 and np.abs(tq - t1).max() < 1e-12
    Rq = Q.conj().T @ phi
    assert np.all(np.abs(np.diag(Rq).imag) < 1e-13) and np.all(np.diag(Rq).real > 0)


def _gram_schmidt(phi):
    """Textbook classical Gram-Schmidt with reorthogonalisation: the unique
    Q with Q^H Q = I and Q^H phi upper triangular with a real positive
    diagonal (written out column by column, independent of LAPACK)."""
    M, N = phi.shape
    Q = np.zeros((M, N), dtype=complex)
    for j in range(N):
        v = phi[:, j].astype(complex)
        for _ in range(2):
            for i in range(j):
                v = v - np.vdot(Q[:, i], v) * Q[:, i]
        Q[:, j] = v / np.linalg.norm(v)
    return Q


def test_p8_qr_phase_convention_against_gram_schmidt():
    """reorthonormalise returns the unique Q whose R = Q^H Phi has a real
    positive diagonal (Gram-Schmidt), and sum log R_jj = 1/2 log det(Phi^H Phi).
    The inputs include -Phi and column-scaled copies, so that LAPACK's own
    factor has negative (or, for the phases, different) diagonal entries in
    at least one case and the phase fix is exercised."""
    M, N = 9, 4
    phi = _trial(M, N, 77) + 0.4 * _rand_walker(M, N, 77)
    rng = np.random.default_rng(5)
    ph = np.exp(1j * rng.uniform(-math.pi, math.pi, size=N))
    cases = [phi, -phi, phi * ph[None, :], phi * np.array([1, -1, 1, -1])[None, :]]
    raw_negative = 0
    for X in cases:
        _, Rraw = np.linalg.qr(X)
        raw_negative += int(np.any(np.diag(Rraw).real < 0))
        Q, logr = O.reorthonormalise(X)
        assert np.abs(Q - _gram_schmidt(X)).max() < 1e-12
        R = Q.conj().T @ X
        assert np.abs(np.tril(R, -1)).max() < 1e-12
        assert np.all(np.abs(np.diag(R).imag) < 1e-13) and np.all(np.diag(R).real > 0)
        _, ld = np.linalg.slogdet(X.conj().T @ X)
        assert abs(logr - 0.5 * ld) < 1e-12
    assert raw_negative >= 2   # the pin is not vacuous


def test_r12_reorthonormalisation_schedule():
    """Reading of the schedule: QR after global step t when (t + 1) % r == 0.
    With r = 3 the orbitals are orthonormal after steps t = 2 and 5 only."""
    M, N, G = 8, 3, 4
    h, L = _rand_system(M, G, 13, scale=0.1)
    psi = _trial(M, N, 13)
    p = O.prepare(h, L, 0.0, psi, 0.1)
    wks = [O.init_walker(p)]
    rng = np.random.default_rng(1)
    xs = rng.normal(size=(6, 1, G))
    ortho = []
    for t in range(6):
        wks, _ = O.run(p, wks, lambda s: xs[s], 1, O.EXP_TAYLOR, 6, 3, step0=t)
        phi = wks[0].phi
        ortho.append(bool(np.abs(phi.conj().T @ phi - np.eye(N)).max() < 1e-12))
    assert ortho == [False, False, True, False, False, True]


def test_p14_weighted_estimator_bruteforce():
    """run's per-step estimator (sum_w W E_L, sum_w W) of Sec. II.A, pinned
    with L = 0 where every factor has a closed form in Fock space: the step
    is exp(-tau h) exactly, so W_w = |R_w| e^{tau (E0 - e_core)}
    max(0, cos arg R_w) with R_w = <Psi_T|e^{-tau H}|Phi_w>/<Psi_T|Phi_w>,
    and E_L^w = <Psi_T|H|Phi'_w>/<Psi_T|Phi'_w>, all by brute force for three
    walkers with distinct weights and energies, over two steps."""
    M, N = 4, 2
    h, _ = _rand_system(M, 1, 17)
    L = np.zeros((1, M, M))
    psi = _trial(M, N, 17)
    tau, e_core = 0.05, 0.3
    p = O.prepare(h, L, e_core, psi, tau)
    phis = [psi + s * _rand_walker(M, N, 17 + i) for i, s in enumerate((0.1, 0.25, 0.4))]
    wks = [O.init_walker(p, ph) for ph in phis]
    _, hist = O.run(p, wks, lambda t: np.zeros((3, 1)), 2, O.EXP_KRYLOV, 4, 0)
    H = fock.hamiltonian(h, L, e_core).toarray()
    U = scipy.linalg.expm(-tau * fock.one_body(h, M).toarray())
    t = fock.determinant(psi.astype(complex))
    e0 = (np.vdot(t, H @ t) / np.vdot(t, t)).real
    d = O.energy_window(2 * N, tau)
    W = np.ones(3)
    vs = [fock.determinant(ph) for ph in phis]
    for s in range(2):
        E = np.empty(3)
        for w in range(3):
            v1 = U @ vs[w]
            R = np.vdot(t, v1) / np.vdot(t, vs[w])
            m = abs(R) * math.exp(tau * (e0 - e_core))
            assert m < 10.0
            W[w] *= m * max(0.0, math.cos(np.angle(R)))
            E[w] = (np.vdot(t, H @ v1) / np.vdot(t, v1)).real
            assert abs(E[w] - e0) < d            # inside the energy window
            vs[w] = v1
        assert np.ptp(W) > 1e-3 and np.ptp(E) > 1e-3   # distinct walkers
        got = hist[s]["estimator"]
        assert abs(got[1] - W.sum()) < 1e-12 * W.sum()
        assert abs(got[0] - (W * E).sum()) < 1e-11 * abs((W * E).sum())
        assert np.abs(hist[s]["weight"] - W).max() < 1e-12


# ---------------------------------------------------------------- P-10 / P-11

def test_p10_small_tau_limit_no_interaction():
    """L = 0: E_H(tau) -> E_L at O(tau) (deterministic)."""
    M, N = 8, 3
    h, _ = _rand_system(M, 1, 51)
    L = np.zeros((1, M, M))
    psi = _trial(M, N, 51)
    phi = psi + 0.3 * _rand_walker(M, N, 51)
    errs = []
    for tau in (0.02, 0.01, 0.005):
        p = O.prepare(h, L, 0.0, psi, tau)
        wk = O.init_walker(p, phi)
        _, info = O.walker_step(p, wk, np.zeros(1), O.EXP_KRYLOV, 4, False)
        e_l = O.local_energy(p, wk.phi, wk.theta)
        errs.append(abs(info.e_hybrid - e_l))
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(2.0, rel=0.05)


def test_p10_small_tau_limit_expectation():
    """One Cholesky vector: the Gauss-Hermite average of E_H over the fields
    tends to E_L of the start walker, with an O(tau) bias."""
    M, N = 6, 2
    h, L = _rand_system(M, 1, 61, scale=0.3)
    psi = _trial(M, N, 61)
    phi = psi + 0.2 * _rand_walker(M, N, 61)
    xs, ws = np.polynomial.hermite_e.hermegauss(60)
    ws = ws / math.sqrt(2 * math.pi)
    errs = []
    for tau in (0.004, 0.002, 0.001):
        p = O.prepare(h, L, 0.0, psi, tau)
        wk = O.init_walker(p, phi)
        e_l = O.local_energy(p, wk.phi, wk.theta)
        avg = 0.0
        for x, wq in zip(xs, ws):
            _, info = O.walker_step(p, wk, np.array([x]), O.EXP_KRYLOV, M, False)
            avg += wq * info.e_hybrid
        errs.append(abs(avg - e_l))
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(2.0, rel=0.15)


def test_p11_no_interaction_projects_to_ground_state():
    """L = 0: imaginary-time projection from a random walker converges to
    2 x (sum of the N lowest eigenvalues of h) (numpy eigh)."""
    M, N = 8, 3
    h, _ = _rand_system(M, 1, 71)
    L = np.zeros((1, M, M))
    psi = _trial(M, N, 71)
    p = O.prepare(h, L, 0.0, psi, 0.5)
    wk = O.init_walker(p, psi + 0.5 * _rand_walker(M, N, 71))
    wks, hist = O.run(p, [wk], lambda t: np.zeros((1, 1)), 150, O.EXP_KRYLOV, 4, 1)
    e_ref = 2.0 * np.sort(np.linalg.eigvalsh(h))[:N].sum()
    assert abs(hist[-1]["e_loc"][0] - e_ref) < 1e-9


# ---------------------------------------------------------------- P-12

def test_p12_force_bias_cap():
    p = O.Prepared(*[None] * 4, 0.25, np.array([0.0, 0.0, 0.0]), *[None] * 5, 0.0)
    ell = np.array([1.9j, 2.0 + 0.0j, 2.1j])     # |f| = 0.5 |ell|
    f, fbar = O.force_bias(p, ell)
    assert np.allclose(f, -0.5j * ell)
    assert fbar[0] == f[0] and fbar[1] == 0 and fbar[2] == 0   # |f| == 1 is capped


def test_p12_reweight_and_phase_caps():
    p = O.Prepared(*[None] * 4, 0.1, *[None] * 6, 0.0)
    assert O.phaseless_factor(p, -10.0 + 0j, 0.0) == pytest.approx(math.e)
    assert O.phaseless_factor(p, -23.1 + 0j, 0.0) == 0.0        # e^2.31 > 10
    assert O.phaseless_factor(p, -22.9 + 0j, 0.0) > 9.0
    assert O.phaseless_factor(p, 0j, math.pi / 2 + 1e-3) == 0.0
    assert O.phaseless_factor(p, 5.0 + 3.0j, 0.5) == pytest.approx(math.exp(-0.5) * math.cos(0.5))


def test_p12_energy_window():
    d = O.energy_window(10, 0.1)
    assert d == pytest.approx(0.5 * 10.0 + 1.0)
    assert O.capped_energy(-1.0 + 5j, -2.0, 10, 0.1) == -1.0
    assert O.capped_energy(-20.0 + 0j, -2.0, 10, 0.1) == -2.0 - d
    assert O.capped_energy(20.0 + 0j, -2.0, 10, 0.1) == -2.0 + d


def test_p12_singular_overlap_freezes_walker():
    M, N, G = 6, 2, 3
    h, L = _rand_system(M, G, 81, scale=0.1)
    psi = _trial(M, N, 81)
    p = O.prepare(h, L, 0.0, psi, 0.05)
    wk = O.init_walker(p)
    # a field so large that the exponential overflows: the walker freezes
    x = np.full(G, 1e200)
    with np.errstate(all="ignore"):
        new, info = O.walker_step(p, wk, x, O.EXP_TAYLOR, 6, False)
    assert not new.alive and new.weight == 0.0
    assert np.array_equal(new.phi, wk.phi)


# ---------------------------------------------------------------- P-15

def test_p15_gradient_against_finite_differences():
    M, N, G = 6, 2, 3
    h, L = _rand_system(M, G, 91, scale=0.2)
    psi = _trial(M, N, 91)
    phi = psi + 0.3 * _rand_walker(M, N, 91)
    p = O.prepare(h, L, 0.0, psi, 0.05)
    _, theta = O.overlap(psi, phi)
    gh, gL = O.local_energy_gradient(p, theta)

    def energy(hh, LL):
        q = O.prepare(hh, LL, 0.0, psi, 0.05, e0=0.0)
        return O.local_energy(q, phi, theta).real

    eps = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(8):
        a, b = rng.integers(0, M, size=2)
        dh = np.zeros((M, M)); dh[a, b] = eps
        fd = (energy(h + dh, L) - energy(h - dh, L)) / (2 * eps)
        assert fd == pytest.approx(gh[a, b], abs=1e-7)
        g = rng.integers(0, G)
        dL = np.zeros((G, M, M)); dL[g, a, b] = eps
        fd = (energy(h, L + dL) - energy(h, L - dL)) / (2 * eps)
        assert fd == pytest.approx(gL[g, a, b], abs=1e-7)


def test_p15_gradient_equals_density_matrices():
    """dE/dh = spin-summed mixed 1-RDM <a+_p a_q>; dE/dL_g,ab =
    sum_qs Gamma_{a q b s} L_g,qs with the mixed 2-RDM
    Gamma_pqrs = sum_{st} <a+_{p s} a+_{q t} a_{s t} a_{r s}>  (Fock space)."""
    M, N, G = 4, 2, 2
    h, L = _rand_system(M, G, 95, scale=0.3)
    psi = _trial(M, N, 95)
    phi = _rand_walker(M, N, 95)
    p = O.prepare(h, L, 0.0, psi, 0.05)
    _, theta = O.overlap(psi, phi)
    gh, gL = O.local_energy_gradient(p, theta)
    a = fock.annihilators(2 * M)
    t = fock.determinant(psi.astype(complex))
    v = fock.determinant(phi)
    ov = np.vdot(t, v)
    rdm1 = np.zeros((M, M), dtype=complex)
    for s in range(2):
        for pp in range(M):
            for q in range(M):
                rdm1[pp, q] += np.vdot(t, a[s * M + pp].T @ (a[s * M + q] @ v)) / ov
    assert np.abs(gh - rdm1.real).max() < 1e-12
    gam = np.zeros((M, M, M, M), dtype=complex)
    for s1 in range(2):
        for s2 in range(2):
            for pp in range(M):
                for q in range(M):
                    for r in range(M):
                        for s in range(M):
                            op = a[s1 * M + pp].T @ (a[s2 * M + q].T @ (a[s2 * M + s] @ (a[s1 * M + r] @ v)))
                            gam[pp, q, r, s] += np.vdot(t, op) / ov
    for g in range(G):
        ref = np.einsum("aqbs,qs->ab", gam, L[g]).real
        assert np.abs(gL[g] - ref).max() < 1e-11


def test_p15_coulomb_vector_gradient_fd():
    M, N, G = 5, 2, 3
    h, L = _rand_system(M, G, 97, scale=0.2)
    psi = _trial(M, N, 97)
    phi = psi + 0.3 * _rand_walker(M, N, 97)
    p = O.prepare(h, L, 0.0, psi, 0.05)
    _, theta = O.overlap(psi, phi)
    d_ell = np.array([0.3 - 0.7j, 1.1 + 0.2j, -0.4 + 0.5j])
    gL = O.coulomb_vector_gradient(p, theta, d_ell)

    def obj(LL):
        q = O.prepare(h, LL, 0.0, psi, 0.05, e0=0.0)
        ell = O.coulomb_vector(q, theta)
        return float(np.sum(d_ell.real * ell.real + d_ell.imag * ell.imag))

    eps = 1e-6
    for (g, a, b) in [(0, 1, 2), (2, 4, 0), (1, 3, 3)]:
        dL = np.zeros((G, M, M)); dL[g, a, b] = eps
        fd = (obj(L + dL) - obj(L - dL)) / (2 * eps)
        assert fd == pytest.approx(gL[g, a, b], abs=1e-8)


# ---------------------------------------------------------------- population layer

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_comb_resample_definition_and_unbiasedness(seed):
    """comb_resample: slot j copies the first walker whose running weight
    sum exceeds (j + u) T / n (numpy searchsorted on cumsum); each walker
    is copied floor or ceil of n W_i / T times; zero weights never; and
    over u the mean copy count is exactly n W_i / T (the comb is unbiased)."""
    rng = np.random.default_rng(seed)
    n = 12
    w = rng.exponential(size=n)
    w[[2, 7]] = 0.0
    T = w.sum()
    for u in (0.0, 0.37, 0.999):
        src = O.comb_resample(w, u)
        ref = np.searchsorted(np.cumsum(w), (np.arange(n) + u) * T / n, side="right")
        assert list(ref) == src
        cnt = np.bincount(src, minlength=n)
        assert cnt[2] == 0 and cnt[7] == 0
        assert np.all(cnt >= np.floor(n * w / T) - 1e-12) and np.all(cnt <= np.ceil(n * w / T) + 1e-12)
    us = (np.arange(4000) + 0.5) / 4000
    mean = np.mean([np.bincount(O.comb_resample(w, u), minlength=n) for u in us], axis=0)
    assert np.abs(mean - n * w / T).max() < 2e-3
    assert O.comb_resample(np.zeros(4), 0.5) is None


def test_e0_update_running_mean():
    """update_e0: E0 of the next step is the mean of the weighted step
    estimates over the last `window` steps with weight; sum W = 0 keeps E0."""
    st = O.E0State(-1.0, window=3)
    seq = [(-2.0, 1.0), (-9.0, 3.0), (0.0, 0.0), (-8.0, 2.0), (-10.0, 2.0)]
    got = [O.update_e0(st, e) for e in seq]
    assert got == [pytest.approx(-2.0), pytest.approx(-2.5), pytest.approx(-2.5),
                   pytest.approx((-2 - 3 - 4) / 3), pytest.approx((-3 - 4 - 5) / 3)]


def test_run_population_control_copies_walkers():
    """run with pop_every = 1: after each step the walkers are the comb's
    copies of the pre-control walkers, with weight 1; with e0_state, p.e0 of
    the next step is the running mean of the estimates."""
    M, N, G = 8, 3, 5
    h, L = _rand_system(M, G, 23, scale=0.15)
    psi = _trial(M, N, 23)
    p = O.prepare(h, L, 0.0, psi, 0.1)
    rng = np.random.default_rng(4)
    xs = rng.normal(size=(3, 6, G))
    wks = [O.init_walker(p) for _ in range(6)]
    st = O.E0State(p.e0, window=2)
    us = [0.3, 0.8, 0.1]
    pre, _ = O.run(p, wks, lambda t: xs[t], 1, O.EXP_KRYLOV, 4, 1)
    p2 = O.prepare(h, L, 0.0, psi, 0.1)
    post, hist = O.run(p2, wks, lambda t: xs[t], 1, O.EXP_KRYLOV, 4, 1, e0_state=st,
                       pop_every=1, comb_u=lambda t: us[t])
    src = hist[0]["comb"]
    assert src == O.comb_resample(np.array([wk.weight for wk in pre]), us[0])
    for j, i in enumerate(src):
        assert np.array_equal(post[j].phi, pre[i].phi) and post[j].weight == 1.0
    est = hist[0]["estimator"]
    assert p2.e0 == pytest.approx(est[0] / est[1])


# ---------------------------------------------------------------- block Krylov (Sec. IV.D)

def _block_case(M, N, seed, scale=0.35):
    rng = np.random.default_rng(seed)
    S = rng.normal(size=(M, M))
    S = (S + S.T) / math.sqrt(4 * M)
    A = 1j * scale * S + 0.05 * np.eye(M)          # complex symmetric, like -tau H_int
    phi = _trial(M, N, seed) + 0.3 * _rand_walker(M, N, seed)
    return A, phi


def test_block_krylov_full_space_is_exact():
    """kN = M: the block Krylov space is the whole space and
    bkrylov_k{A, Psi} = exp(A) Psi (scipy expm)."""
    for M, N, k in ((8, 2, 4), (12, 3, 4), (10, 5, 2)):
        A, phi = _block_case(M, N, M + N)
        got = O.block_krylov(A, phi, k)
        ref = scipy.linalg.expm(A) @ phi
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_block_krylov_right_equivariance():
    """The result is V exp(V^dag A V) V^dag Psi for an orthonormal basis V of
    the block Krylov space, so Psi -> Psi S (S invertible) gives exactly
    bkrylov(A, Psi) S -- unlike the per-orbital Krylov."""
    M, N, k = 20, 4, 3
    A, phi = _block_case(M, N, 5)
    rng = np.random.default_rng(6)
    S = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    a = O.block_krylov(A, phi @ S, k)
    b = O.block_krylov(A, phi, k) @ S
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    # the per-orbital Krylov is not equivariant (the schedule of QR matters)
    c = O.krylov(A, phi @ S, k)
    assert np.abs(c - O.krylov(A, phi, k) @ S).max() > 1e-6


def test_block_krylov_one_orbital_is_krylov():
    """N = 1: the block method is the per-orbital Krylov of Eq. (krylov)."""
    M = 16
    A, phi = _block_case(M, 1, 9)
    for k in (2, 4, 6):
        a = O.block_krylov(A, phi, k)[:, 0]
        b = O.krylov_vector(A, phi[:, 0], k)
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_block_arnoldi_relations():
    """B_k^dag B_k = I, A_k = B_k^dag A B_k (Eq. projham for blocks), A_k is
    block upper Hessenberg with upper-triangular subdiagonal blocks, and
    Psi = B_1 R."""
    M, N, k = 24, 3, 4
    A, phi = _block_case(M, N, 11)
    Bk, Hk, R = O.block_arnoldi(A, phi, k)
    assert Bk.shape == (M, k * N) and Hk.shape == (k * N, k * N)
    assert np.abs(Bk.conj().T @ Bk - np.eye(k * N)).max() < 1e-13
    assert np.abs(Bk.conj().T @ A @ Bk - Hk).max() < 1e-12
    for i in range(k):
        for j in range(k):
            blk = Hk[i * N:(i + 1) * N, j * N:(j + 1) * N]
            if i > j + 1:
                assert np.abs(blk).max() == 0.0
            if i == j + 1:
                assert np.abs(np.tril(blk, -1)).max() < 1e-14
    assert np.abs(Bk[:, :N] @ R - phi).max() < 1e-13


def test_block_krylov_thouless_and_error_decreases():
    """Fock space: exp(Ahat)|Phi> = |bkrylov(A, Phi)> when kN = M; for
    kN < M the error against exp(A) Phi falls with k and stays below the
    per-orbital Krylov error at the same k."""
    M, N = 4, 2
    A, phi = _block_case(M, N, 13, scale=0.6)
    ref = scipy.linalg.expm(fock.one_body(A, M).toarray()) @ fock.determinant(phi)
    got = fock.determinant(O.block_krylov(A, phi, 2))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    M, N = 40, 4
    A, phi = _block_case(M, N, 14, scale=0.6)
    exact = scipy.linalg.expm(A) @ phi
    errs = [np.abs(O.block_krylov(A, phi, k) - exact).max() for k in (1, 2, 3, 4)]
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(3))
    for k in (2, 3, 4):
        assert np.abs(O.block_krylov(A, phi, k) - exact).max() < \
            np.abs(O.krylov(A, phi, k) - exact).max()
