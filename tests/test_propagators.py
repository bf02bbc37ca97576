"""Oracle pins of the propagator variants (Sec. III): Split-1, Split-2, the
refactorised (Taylor) propagator and Crank-Nicolson, and of the size
consistency of the local energy (Sec. V.F) on a direct sum of two systems.
CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg

import afq_workloads as W
from oracle import afq_oracle as O

PROPS = (O.PROP_SPLIT2, O.PROP_SPLIT1, O.PROP_TAYLOR, O.PROP_CN)


def _system(M, N, G, seed, diag=False, scale=0.3):
    rng = np.random.default_rng(seed)
    if diag:
        h = np.diag(rng.uniform(-2.0, 0.0, M))
        L = np.stack([np.diag(rng.normal(0.0, scale, M)) for _ in range(G)])
        psi = np.eye(M)[:, :N]
    else:
        ham = W.hamiltonian(M, G, 0.1, scale / math.sqrt(M), seed, 0.0)
        h, L = ham.h, ham.L
        psi = W.rhf_trial(h, L, N, n_iter=3)
    return h, L, psi


def _exact(A, phi):
    return scipy.linalg.expm(A) @ phi


def test_no_interaction_all_propagators_apply_exp_minus_tau_h1():
    """L = 0: the interaction vanishes, and Split-1 and Split-2 both apply
    exp(-tau H1) exactly; the refactorised propagator with the block Krylov
    space equal to the orbital space (k N = M) does too."""
    M, N = 12, 3
    h, _, psi = _system(M, N, 4, seed=2)
    L = np.zeros((1, M, M))
    p = O.prepare(h, L, 0.0, psi, tau=0.1)
    rng = np.random.default_rng(0)
    phi = psi + 0.1 * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N)))
    A = np.zeros((M, M), complex)
    want = _exact(-p.tau * p.H1, phi)
    for prop, method, k in ((O.PROP_SPLIT2, O.EXP_TAYLOR, 1), (O.PROP_SPLIT1, O.EXP_TAYLOR, 1),
                            (O.PROP_TAYLOR, O.EXP_BLOCK_KRYLOV, M // N)):
        got = O.propagate_orbitals(p, phi, A, method, k, prop)
        assert np.abs(got - want).max() < 1e-12, prop


def test_commuting_operators_all_propagators_agree():
    """Diagonal h and L commute with each other: then exp(-tau H1 / 2)
    exp(A) exp(-tau H1 / 2) = exp(-tau H1) exp(A) = exp(A - tau H1), so the
    three propagators give the same orbitals (long Taylor series)."""
    M, N, G = 10, 3, 6
    h, L, psi = _system(M, N, G, seed=4, diag=True)
    p = O.prepare(h, L, 0.0, psi, tau=0.05)
    x = np.random.default_rng(1).standard_normal(G)
    ell = O.coulomb_vector(p, psi.astype(complex))
    _, fbar = O.force_bias(p, ell)
    A, _, _ = O.interaction_operator(p, x, fbar)
    phi = psi.astype(complex)
    outs = [O.propagate_orbitals(p, phi, A, O.EXP_TAYLOR, 40, prop) for prop in PROPS[:3]]
    want = _exact(A - p.tau * p.H1, phi)
    for o in outs:
        assert np.abs(o - want).max() < 1e-13


@pytest.mark.parametrize("prop,order", [(O.PROP_SPLIT1, 1.5), (O.PROP_SPLIT2, 2.0)])
def test_splitting_error_scaling(prop, order):
    """With A ~ sqrt(tau) (fields of unit size) and tau H1 ~ tau, the one-step
    difference to the refactorised exp(A - tau H1) is O(tau^1.5) for Split-1
    (first order: [tau H1, A] / 2) and O(tau^2) for Split-2 (symmetric:
    the leading term is [A, [A, tau H1]]): quartering tau divides it by
    ~8 and ~16."""
    M, N, G = 14, 3, 8
    h, L, psi = _system(M, N, G, seed=7, scale=1.0)
    x = np.random.default_rng(3).standard_normal(G)
    diffs = []
    for tau in (0.04, 0.01, 0.0025):
        p = O.prepare(h, L, 0.0, psi, tau=tau)
        fbar = np.zeros(G, complex)
        A, _, _ = O.interaction_operator(p, x, fbar)
        phi = psi.astype(complex)
        a = O.propagate_orbitals(p, phi, A, O.EXP_TAYLOR, 40, prop)
        b = O.propagate_orbitals(p, phi, A, O.EXP_TAYLOR, 40, O.PROP_TAYLOR)
        diffs.append(np.abs(a - b).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    print(prop, diffs, r1, r2)
    assert r2 == pytest.approx(4.0 ** order, rel=0.15)


def _direct_sum(a, b):
    """System A + B: block-diagonal h, the Cholesky vectors of A padded with
    zeros, then those of B; the trial is the block-diagonal union of the
    occupied orbitals; e_core adds."""
    (ha, La, pa), (hb, Lb, pb) = a, b
    Ma, Mb = ha.shape[0], hb.shape[0]
    h = scipy.linalg.block_diag(ha, hb)
    L = np.zeros((La.shape[0] + Lb.shape[0], Ma + Mb, Ma + Mb))
    L[:La.shape[0], :Ma, :Ma] = La
    L[La.shape[0]:, Ma:, Ma:] = Lb
    psi = scipy.linalg.block_diag(pa, pb)
    return h, L, psi


@pytest.mark.parametrize("prop", PROPS)
def test_size_consistency_of_one_walker(prop):
    """Sec. V.F on a synthetic pair: for the direct sum A + B with the
    fields (x_A, x_B), a walker stays the direct sum of the walkers of A and
    B (every propagator; the Krylov space of an orbital of A stays in A),
    log <Psi_T|Phi> and the local and hybrid energies add exactly (up to
    rounding) over steps with reorthonormalisation.  The phaseless factor
    cos(dtheta_A + dtheta_B) does not factorise, so weights are not
    compared."""
    a = _system(9, 2, 10, seed=21)
    b = _system(7, 3, 8, seed=22)
    h, L, psi = _direct_sum(a, b)
    tau = 0.05
    pa = O.prepare(a[0], a[1], 0.3, a[2], tau)
    pb = O.prepare(b[0], b[1], -0.1, b[2], tau)
    pab = O.prepare(h, L, 0.2, psi, tau)
    assert pab.e0 == pytest.approx(pa.e0 + pb.e0, abs=1e-12)
    wa, wb, wab = O.init_walker(pa), O.init_walker(pb), O.init_walker(pab)
    rng = np.random.default_rng(5)
    for t in range(6):
        xa, xb = rng.standard_normal(10), rng.standard_normal(8)
        wa, ia = O.walker_step(pa, wa, xa, O.EXP_KRYLOV, 6, t % 2 == 1, prop)
        wb, ib = O.walker_step(pb, wb, xb, O.EXP_KRYLOV, 6, t % 2 == 1, prop)
        wab, iab = O.walker_step(pab, wab, np.concatenate([xa, xb]), O.EXP_KRYLOV, 6,
                                 t % 2 == 1, prop)
        assert iab.e_loc == pytest.approx(ia.e_loc + ib.e_loc, abs=1e-11)
        assert iab.e_hybrid == pytest.approx(ia.e_hybrid + ib.e_hybrid, abs=1e-9)
        assert abs(wab.logdet.real - (wa.logdet.real + wb.logdet.real)) < 1e-11
        blk = scipy.linalg.block_diag(wa.phi, wb.phi)
        assert np.abs(wab.phi - blk).max() < 1e-12


def test_crank_nicolson_is_the_cayley_transform():
    """Without interaction (L = 0), CN multiplies each eigenvector of H1 by
    (1 - tau lambda / 2) / (1 + tau lambda / 2): checked against that
    spectral form (eigh), not against a solve."""
    M, N = 11, 3
    h, _, psi = _system(M, N, 4, seed=6)
    p = O.prepare(h, np.zeros((1, M, M)), 0.0, psi, tau=0.2)
    lam, v = np.linalg.eigh(p.H1)
    cay = (v * ((1.0 - 0.5 * p.tau * lam) / (1.0 + 0.5 * p.tau * lam))) @ v.T
    phi = psi.astype(complex) * (1.0 + 0.5j)
    got = O.propagate_orbitals(p, phi, np.zeros((M, M), complex), O.EXP_TAYLOR, 1, O.PROP_CN)
    assert np.abs(got - cay @ phi).max() < 1e-13


def test_crank_nicolson_error_scaling():
    """CN is the (1,1) Pade approximant of exp(A_T): its one-step error
    against exp(A_T) is A_T^3 / 12 + ..., O(tau^1.5) with A ~ sqrt(tau):
    quartering tau divides it by ~8."""
    M, N, G = 14, 3, 8
    h, L, psi = _system(M, N, G, seed=7, scale=1.0)
    x = np.random.default_rng(3).standard_normal(G)
    diffs = []
    for tau in (0.04, 0.01, 0.0025):
        p = O.prepare(h, L, 0.0, psi, tau=tau)
        A, _, _ = O.interaction_operator(p, x, np.zeros(G, complex))
        phi = psi.astype(complex)
        a = O.propagate_orbitals(p, phi, A, O.EXP_TAYLOR, 40, O.PROP_CN)
        b = O.propagate_orbitals(p, phi, A, O.EXP_TAYLOR, 40, O.PROP_TAYLOR)
        diffs.append(np.abs(a - b).max())
    print(diffs, diffs[0] / diffs[1], diffs[1] / diffs[2])
    assert diffs[1] / diffs[2] == pytest.approx(8.0, rel=0.15)


@pytest.mark.parametrize("fb_at", [O.FB_START, O.FB_HALF])
def test_force_bias_placement_is_a_change_of_variables(fb_at):
    """One Cholesky vector (the HS transform is exact): whether f is taken at
    the start of the step or at the half-step orbitals, the Gauss-Hermite
    average over x of exp(-tau (E_H(x) - E0)) |Phi'(x)> / <Psi_T|Phi'(x)>
    from the oracle's own step equals the split propagator in Fock space;
    the two placements differ in f (so in the samples), not in the average."""
    import fock
    M, N, G = 4, 2, 1
    rng = np.random.default_rng(31)
    A0 = rng.normal(size=(M, M)) * 0.5
    h = np.diag(rng.uniform(-2, 0, M)) + 0.05 * (A0 + A0.T)
    L = (lambda a: (a + a.T)[None])(rng.normal(size=(M, M)) * 0.5)
    psi, _ = np.linalg.qr(rng.normal(size=(M, N)))
    tau = 0.3
    p = O.prepare(h, L, 0.1, psi, tau)
    phi = psi + 0.3 * (rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N)))
    wk = O.init_walker(p, phi)
    xs, ws = np.polynomial.hermite_e.hermegauss(90)
    ws = ws / math.sqrt(2 * math.pi)
    t = fock.determinant(psi.astype(complex))
    acc = np.zeros(1 << (2 * M), dtype=complex)
    fs = set()
    for x, wq in zip(xs, ws):
        new, info = O.walker_step(p, wk, np.array([x]), O.EXP_KRYLOV, M, False,
                                  O.PROP_SPLIT2, fb_at)
        fs.add(complex(info.f[0]))
        v = fock.determinant(new.phi)
        acc += wq * np.exp(-tau * (info.e_hybrid - p.e0)) * v / np.vdot(t, v)
    assert len(fs) == 1 and abs(fs.pop()) > 0.05
    dim = 1 << (2 * M)
    Bh = scipy.linalg.expm(-0.5 * tau * fock.one_body(p.H1, M).toarray())
    X = fock.one_body(L[0], M).toarray() - p.lbar[0] * np.eye(dim)
    U = math.exp(-tau * (p.e_const - p.e0)) * Bh @ scipy.linalg.expm(-0.5 * tau * X @ X) @ Bh
    v0 = fock.determinant(wk.phi)
    ref = U @ v0 / np.vdot(t, v0)
    assert np.abs(acc - ref).max() < 1e-9 * np.abs(ref).max()


def test_force_bias_placements_differ():
    """The half-step force bias is not the start-of-step one (a walker away
    from the trial): the placement is a real option, not a no-op."""
    M, N, G = 10, 3, 12
    h, L, psi = _system(M, N, G, seed=8, scale=1.0)
    p = O.prepare(h, L, 0.0, psi, tau=0.1)
    rng = np.random.default_rng(2)
    phi = psi + 0.3 * (rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N)))
    wk = O.init_walker(p, phi)
    x = rng.normal(size=G)
    _, a = O.walker_step(p, wk, x, O.EXP_KRYLOV, 6, False, O.PROP_SPLIT2, O.FB_START)
    _, b = O.walker_step(p, wk, x, O.EXP_KRYLOV, 6, False, O.PROP_SPLIT2, O.FB_HALF)
    assert np.abs(a.f - b.f).max() > 1e-3
    with pytest.raises(ValueError):
        O.walker_step(p, wk, x, O.EXP_KRYLOV, 6, False, O.PROP_SPLIT1, O.FB_HALF)
