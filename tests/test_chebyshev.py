"""Oracle pins of the Chebyshev expansion of the exponential (Sec. IV.B,
Eq. chebpoly).  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.special

from oracle import afq_oracle as O


def test_coefficients_are_modified_bessel_values():
    """c_0 = J_0(i) and c_n = 2 i^n J_n(-i) as printed equal I_0(1) and
    2 I_n(1) (J_n(i z) = i^n I_n(z)): the coefficients of
    exp(x) = I_0(1) + 2 sum_n I_n(1) T_n(x)."""
    assert O.chebyshev_coefficient(0) == pytest.approx(scipy.special.iv(0, 1.0), rel=1e-15)
    for n in range(1, 18):
        assert O.chebyshev_coefficient(n) == pytest.approx(2.0 * scipy.special.iv(n, 1.0),
                                                           rel=1e-14)


@pytest.mark.parametrize("k", [2, 5, 9])
def test_scalar_error_bound_on_the_interval(k):
    """For x in [-1, 1], |T_n(x)| <= 1, so |cheb_k(x) - e^x| <= sum_{n>k} c_n."""
    tail = sum(O.chebyshev_coefficient(n) for n in range(k + 1, 40))
    for x in np.linspace(-1.0, 1.0, 41):
        got = O.chebyshev(np.array([[x]], dtype=complex), np.ones((1, 1), complex), k)[0, 0]
        assert abs(got - math.exp(x)) <= tail * (1 + 1e-12) + 1e-15


def test_matrix_series_equals_scalar_series_on_the_spectrum():
    """For a normal matrix A = V diag(mu) V^H the expansion acts on each
    eigenvector by the scalar polynomial p_k(mu) = sum c_n T_n(mu), with
    T_n(mu) = cosh(n arccosh mu) evaluated directly (no recurrence), and it
    tends to expm(A) as k grows."""
    rng = np.random.default_rng(2)
    M, N = 9, 3
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))
    mu = 0.4 * (rng.uniform(-1, 1, M) + 1j * rng.uniform(-1, 1, M))
    A = (Q * mu) @ Q.conj().T
    phi = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    for k in (1, 4, 8):
        p = sum(O.chebyshev_coefficient(n) * np.cosh(n * np.arccosh(mu.astype(complex)))
                for n in range(k + 1))
        want = (Q * p) @ (Q.conj().T @ phi)
        assert np.abs(O.chebyshev(A, phi, k) - want).max() < 1e-12
    exact = scipy.linalg.expm(A) @ phi
    errs = [np.abs(O.chebyshev(A, phi, k) - exact).max() for k in (2, 4, 8, 16)]
    assert errs[-1] < 1e-13 and all(a > b for a, b in zip(errs, errs[1:]))
