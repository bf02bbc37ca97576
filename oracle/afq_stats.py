"""FP64 CPU oracle of the estimator statistics of a ph-AFQMC run.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
calls it and shares no code with it.

Source: Sukurma et al., arXiv 2403.02542, Sec. II.A (time average, variance
and correlation length of the per-step estimates W_k, E_k, Eq. (variance))
and Sec. V.G / VI (time-step extrapolation, Eqs. (square_fit),
(pure_square_fit) and the linear form beside it; statistical error of an
extrapolated energy, Eq. (staterr)).  Plain numpy, loops written out.

Readings (the paper defines kappa but names no estimator for it):
  * The squared-energy average in sigma_E^2 uses the same weights W_k as the
    energy average, and N in Eq. (variance) counts the samples after the
    equilibration phase.
  * kappa is estimated from the unweighted series E_k in two published ways:
    the integrated autocorrelation time 1 + 2 sum_t rho(t) with the
    self-consistent window of Sokal (1997), M = the smallest M >= c kappa(M);
    and the blocking transformation of Flyvbjerg and Petersen (1989) with the
    optimal level of Lee, Needs, Drummond and Towler (2011), kappa = the
    ratio of the blocked to the unblocked variance of the mean.
  * The fits are least squares weighted by 1 / sigma_i^2 (unit weights when
    no sigma is given); the error of E0 is the square root of its diagonal
    entry in (A^T Sigma^-1 A)^-1.

Parity pins: tests/test_stats.py checks these against hand-computed values,
closed forms (AR(1): kappa = (1 + phi) / (1 - phi); independent samples:
kappa = 1), exact polynomial data and a Monte Carlo spread of fitted E0.
"""
from __future__ import annotations

import math

import numpy as np


def time_average(w, e, n_eq=0):
    """(E_bar, sigma_E^2, n) of Sec. II.A: the W_k-weighted time averages of
    E_k and E_k^2 over k > n_eq, and the number n of those samples."""
    num = den = num2 = 0.0
    n = 0
    for k in range(n_eq, len(e)):
        num += w[k] * e[k]
        num2 += w[k] * e[k] * e[k]
        den += w[k]
        n += 1
    if n == 0 or den == 0.0:
        return float("nan"), float("nan"), n
    mean = num / den
    return mean, num2 / den - mean * mean, n


def error_of_mean(sigma2_e, n, kappa):
    """sigma_E_bar = sqrt(sigma_E^2 kappa / N)   (Eq. variance)."""
    return math.sqrt(sigma2_e * kappa / n)


def autocorrelation(e, t):
    """rho(t) = C(t) / C(0), C(t) = (1 / (n - t)) sum_i (E_i - m)(E_{i+t} - m)."""
    n = len(e)
    m = sum(e) / n
    c0 = sum((x - m) ** 2 for x in e) / n
    ct = sum((e[i] - m) * (e[i + t] - m) for i in range(n - t)) / (n - t)
    return ct / c0


def autocorrelation_time(e, c=5.0):
    """(kappa, M): kappa(M) = 1 + 2 sum_{t=1}^{M} rho(t) with M the smallest
    window such that M >= c kappa(M) (Sokal); M stops at n - 1."""
    n = len(e)
    kappa = 1.0
    for m in range(1, n):
        kappa += 2.0 * autocorrelation(e, m)
        if m >= c * kappa:
            return kappa, m
    return kappa, n - 1


def blocking(e):
    """Blocking transformation: level l holds the means of blocks of 2^l
    samples (a trailing odd sample dropped at each halving).  Returns a list
    of (n_l, se_l, se_err_l) with se_l^2 = sum (x - x_bar)^2 / (n_l (n_l - 1))
    and se_err_l = se_l / sqrt(2 (n_l - 1)), for every level with n_l >= 2."""
    x = list(e)
    out = []
    while len(x) >= 2:
        n = len(x)
        m = sum(x) / n
        se = math.sqrt(sum((v - m) ** 2 for v in x) / (n * (n - 1)))
        out.append((n, se, se / math.sqrt(2.0 * (n - 1))))
        x = [(x[2 * i] + x[2 * i + 1]) / 2.0 for i in range(n // 2)]
    return out


def blocking_kappa(e):
    """(kappa, level): the optimal level is the smallest l with
    (2^l)^3 > 2 n_0 (se_l / se_0)^4 (Lee et al.); kappa = (se_l / se_0)^2.
    With no such level the last one is taken."""
    lv = blocking(e)
    n0, se0, _ = lv[0]
    best = len(lv) - 1
    for l, (_, se, _) in enumerate(lv):
        if (2.0 ** l) ** 3 > 2.0 * n0 * (se / se0) ** 4:
            best = l
            break
    return (lv[best][1] / se0) ** 2, best


FIT_QUADRATIC, FIT_PURE_SQUARE, FIT_LINEAR = 0, 1, 2


def tau_fit(tau, e, sigma=None, form=FIT_QUADRATIC):
    """Time-step extrapolation (Sec. V.G): E(tau) = E0 + alpha tau + beta tau^2
    (Eq. square_fit), E0 + beta tau^2 (Eq. pure_square_fit) or E0 + alpha tau.
    Returns ((E0, alpha, beta), err_E0), with the absent coefficient 0."""
    tau = np.asarray(tau, dtype=float)
    e = np.asarray(e, dtype=float)
    s = np.ones_like(tau) if sigma is None else np.asarray(sigma, dtype=float)
    cols = {FIT_QUADRATIC: [0, 1, 2], FIT_PURE_SQUARE: [0, 2], FIT_LINEAR: [0, 1]}[form]
    A = np.stack([tau ** p for p in cols], axis=1)
    wgt = 1.0 / s ** 2
    AtA = A.T @ (wgt[:, None] * A)
    Atb = A.T @ (wgt * e)
    cov = np.linalg.inv(AtA)
    x = cov @ Atb
    coef = [0.0, 0.0, 0.0]
    for j, p in enumerate(cols):
        coef[p] = float(x[j])
    return tuple(coef), math.sqrt(cov[0, 0])


def sigma_x(sigmas):
    """sigma_x = sqrt(sum_i sigma_i^2) / N_tau   (Eq. staterr)."""
    return math.sqrt(sum(s * s for s in sigmas)) / len(sigmas)
