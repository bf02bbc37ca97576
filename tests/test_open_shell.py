"""Oracle pins of the open-shell (spin-orbital) form: determinants of spin
orbitals with the closed-shell factor 2 replaced by 1 (Eq. eloc, hyben,
force_shift written for general determinants).  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg

import afq_workloads as W
import fock
from oracle import afq_oracle as O


def _spatial(M, N, G, seed, scale=0.4):
    ham = W.hamiltonian(M, G, 0.1, scale / math.sqrt(M), seed, 0.0)
    return ham.h, ham.L, W.rhf_trial(ham.h, ham.L, N, n_iter=3)


def test_spin_orbital_embedding_of_a_closed_shell_system():
    """A closed-shell system written in spin orbitals (Psi_a = Psi_b) and run
    with spin = 1 gives the closed-shell (spin = 2) trajectory: the same
    E_L, E_H, weights and log-overlaps (the spin-orbital log-overlap is the
    sum over both spin blocks), and the walker stays diag(Phi, Phi)."""
    M, N, G = 10, 3, 14
    h, L, psi = _spatial(M, N, G, seed=5)
    h2, L2, psi2 = W.spin_orbital_system(h, L, psi, psi)
    tau = 0.05
    p = O.prepare(h, L, 0.2, psi, tau)
    p2 = O.prepare(h2, L2, 0.2, psi2, tau, spin=1)
    assert p2.e0 == pytest.approx(p.e0, abs=1e-12)
    assert np.allclose(p2.lbar, p.lbar, atol=1e-13)
    a, b = O.init_walker(p), O.init_walker(p2)
    rng = np.random.default_rng(3)
    for t in range(6):
        x = rng.standard_normal(G)
        a, ia = O.walker_step(p, a, x, O.EXP_KRYLOV, 6, t % 2 == 1)
        b, ib = O.walker_step(p2, b, x, O.EXP_KRYLOV, 6, t % 2 == 1)
        assert ib.e_loc == pytest.approx(ia.e_loc, rel=1e-10, abs=1e-10)
        # E_H agrees up to the 2 pi / tau ambiguity of its imaginary part (the
        # phase of a log-overlap is wrapped per determinant)
        assert ib.e_hybrid.real == pytest.approx(ia.e_hybrid.real, rel=1e-10, abs=1e-9)
        d = tau * (ib.e_hybrid.imag - ia.e_hybrid.imag)
        assert abs((d + math.pi) % (2 * math.pi) - math.pi) < 1e-9
        assert b.weight == pytest.approx(a.weight, rel=1e-10)
        assert abs(b.logdet.real - 2 * a.logdet.real) < 1e-10
        assert np.abs(b.phi - scipy.linalg.block_diag(a.phi, a.phi)).max() < 1e-12


def test_open_shell_local_energy_against_fock_space():
    """N_a = 2, N_b = 1 on M = 4: E_L = <Psi_T|H|Phi> / <Psi_T|Phi> and
    ell_g = <Psi_T|Lhat_g|Phi> / <Psi_T|Phi> in the 256-dimensional Fock
    space (Jordan-Wigner) for random complex walker blocks."""
    M, G = 4, 3
    rng = np.random.default_rng(11)
    h, L, _ = _spatial(M, 2, G, seed=11, scale=1.0)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    pa, pb = Q[:, :2], Q[:, 2:3]
    h2, L2, psi2 = W.spin_orbital_system(h, L, pa, pb)
    p = O.prepare(h2, L2, 0.3, psi2, 0.1, spin=1)
    H = fock.hamiltonian(h, L, 0.3)
    t = fock.determinant(pa.astype(complex), pb.astype(complex))
    for s in range(3):
        fa = pa + 0.4 * (rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2)))
        fb = pb + 0.4 * (rng.standard_normal((M, 1)) + 1j * rng.standard_normal((M, 1)))
        v = fock.determinant(fa, fb)
        phi = np.zeros((2 * M, 3), complex)
        phi[:M, :2] = fa
        phi[M:, 2:] = fb
        logdet, theta = O.overlap(psi2, phi)
        ov = np.vdot(t, v)
        assert np.exp(logdet) == pytest.approx(ov, rel=1e-10)
        e = O.local_energy(p, phi, theta)
        assert e == pytest.approx(np.vdot(t, H @ v) / ov, rel=1e-10)
        ell = O.coulomb_vector(p, theta)
        for g in range(G):
            Lg = fock.one_body(L[g], M)
            assert ell[g] == pytest.approx(np.vdot(t, Lg @ v) / ov, rel=1e-10)
    # the trial energy and the mean-field shift
    assert p.e0 == pytest.approx((np.vdot(t, H @ t) / np.vdot(t, t)).real, rel=1e-12)
    for g in range(G):
        lg = np.vdot(t, fock.one_body(L[g], M) @ t).real
        assert p.lbar[g] == pytest.approx(lg, abs=1e-12)


def test_open_shell_importance_sampled_step_expectation():
    """One Cholesky vector, N_a = 2, N_b = 1: the Gauss-Hermite average of
    the oracle's own step, exp(-tau (E_H(x) - E0)) |Phi'(x)> / <Psi_T|Phi'(x)>,
    equals the split propagator in Fock space (the open-shell overlap ratio,
    mean-field shift, I and e_const together)."""
    M, G = 4, 1
    rng = np.random.default_rng(31)
    h, L, _ = _spatial(M, 2, G, seed=31, scale=1.5)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    pa, pb = Q[:, :2], Q[:, 2:3]
    h2, L2, psi2 = W.spin_orbital_system(h, L, pa, pb)
    tau = 0.3
    p = O.prepare(h2, L2, 0.1, psi2, tau, spin=1)
    fa = pa + 0.3 * (rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2)))
    fb = pb + 0.3 * (rng.standard_normal((M, 1)) + 1j * rng.standard_normal((M, 1)))
    phi = np.zeros((2 * M, 3), complex)
    phi[:M, :2] = fa
    phi[M:, 2:] = fb
    wk = O.init_walker(p, phi)
    xs, ws = np.polynomial.hermite_e.hermegauss(90)
    ws = ws / math.sqrt(2 * math.pi)
    t = fock.determinant(pa.astype(complex), pb.astype(complex))
    acc = np.zeros(1 << (2 * M), dtype=complex)
    fvals = set()
    for x, wq in zip(xs, ws):
        new, info = O.walker_step(p, wk, np.array([x]), O.EXP_KRYLOV, 2 * M, False)
        fvals.add(complex(info.f[0]))
        v = fock.determinant(new.phi[:M, :2], new.phi[M:, 2:])
        acc += wq * np.exp(-tau * (info.e_hybrid - p.e0)) * v / np.vdot(t, v)
    assert len(fvals) == 1 and abs(fvals.pop()) > 0.05
    dim = 1 << (2 * M)
    H1 = p.H1[:M, :M]
    assert np.allclose(p.H1[M:, M:], H1) and np.all(p.H1[:M, M:] == 0)
    Bh = scipy.linalg.expm(-0.5 * tau * fock.one_body(H1, M).toarray())
    X = fock.one_body(L[0], M).toarray() - p.lbar[0] * np.eye(dim)
    U = math.exp(-tau * (p.e_const - p.e0)) * Bh @ scipy.linalg.expm(-0.5 * tau * X @ X) @ Bh
    v0 = fock.determinant(fa, fb)
    ref = U @ v0 / np.vdot(t, v0)
    assert np.abs(acc - ref).max() < 1e-9 * np.abs(ref).max()


def test_spin_factor_is_checked():
    h, L, psi = _spatial(6, 2, 4, seed=1)
    with pytest.raises(ValueError):
        O.prepare(h, L, 0.0, psi, 0.1, spin=3)
    p = O.prepare(h, L, 0.0, psi, 0.1, spin=1)
    with pytest.raises(ValueError):
        O.local_energy_gradient(p, psi.astype(complex))
