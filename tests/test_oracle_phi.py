"""Pins of the oracle's phi-functions against definitions and closed forms.

Nothing here re-calls the oracle's own library routine as the reference:
the references are the Taylor definition (eq. seriesdef), scalar phi
functions on eigenvalues in closed form (sine / Fourier bases), the
squaring identity of section 3.1 (eq. squarephi) and phi_l(0) = I / l!.
"""

import cmath
import math

import numpy as np
import pytest

from oracle.phi import phi_functions, phi_series
from workloads import dirichlet_d2, dirichlet_d1, periodic_d2


def phi_scalar(z, ell):
    """Scalar phi_l(z): series for |z| < 1, else phi_0 = e^z and
    phi_l(z) = (phi_{l-1}(z) - 1/(l-1)!) / z."""
    z = complex(z)
    if abs(z) < 1.0:
        term, acc = 1.0 + 0j, 0j
        for i in range(40):
            acc += term / math.factorial(i + ell)
            term *= z
        return acc
    val = cmath.exp(z)
    for k in range(1, ell + 1):
        val = (val - 1.0 / math.factorial(k - 1)) / z
    return val


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 5, 17])
def test_phi_matches_taylor_definition(n, cplx):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n)) * (0.4 / np.sqrt(n))
    if cplx:
        X = X + 1j * rng.standard_normal((n, n)) * (0.4 / np.sqrt(n))
    phis = phi_functions(X, 3)
    for ell in range(4):
        ref = phi_series(X, ell)
        assert np.max(np.abs(phis[ell] - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("ell", [0, 1, 2])
def test_phi_at_zero(ell):
    phis = phi_functions(np.zeros((6, 6)), 2)
    assert np.array_equal(phis[ell], np.eye(6) / math.factorial(ell))


@pytest.mark.parametrize("n,c,tau", [(64, 0.01, 1e-3), (129, 0.02, 2e-3), (48, 0.02, 0.3)])
def test_phi_dirichlet_sine_basis(n, c, tau):
    """phi_l(tau c D2) = S diag(phi_l(tau c lambda_k)) S, S_jk = sqrt(2h) sin(j k pi h)."""
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    S = np.sqrt(2 * h) * np.sin(np.outer(j, j) * np.pi * h)
    lam = -(4.0 / h ** 2) * np.sin(j * np.pi * h / 2) ** 2
    phis = phi_functions(tau * c * dirichlet_d2(n, h), 2)
    for ell in range(3):
        f = np.array([phi_scalar(tau * c * l, ell).real for l in lam])
        ref = S @ np.diag(f) @ S
        err = np.max(np.abs(phis[ell] - ref)) / np.max(np.abs(ref))
        assert err < 5e-14, (ell, err)


@pytest.mark.parametrize("n", [16, 48])
def test_phi_periodic_fourier_basis_complex(n):
    """(i/2) D2 periodic is a circulant: diagonalised by the DFT,
    lambda_k = -(4/h^2) sin^2(pi k / n)."""
    tau = 1e-3
    h = 2 * np.pi / n
    k = np.arange(n)
    F = np.exp(2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)
    lam = -(4.0 / h ** 2) * np.sin(np.pi * k / n) ** 2
    A = 0.5j * periodic_d2(n, h)
    phis = phi_functions(tau * A, 2)
    for ell in range(3):
        f = np.array([phi_scalar(tau * 0.5j * l, ell) for l in lam])
        ref = F @ np.diag(f) @ F.conj().T
        err = np.max(np.abs(phis[ell] - ref)) / np.max(np.abs(ref))
        assert err < 5e-14, (ell, err)
    # e^{tau A} is unitary for skew-Hermitian A
    U = phis[0]
    assert np.max(np.abs(U.conj().T @ U - np.eye(n))) < 1e-13


def test_phi_nonsymmetric_tridiagonal_closed_form():
    """tridiag(a, b, c) (a below, c above the diagonal, a c > 0) has eigenpairs
    b + 2 sqrt(a c) cos(k pi/(n+1)) and v_k(j) = (a/c)^{j/2} sin(j k pi/(n+1))."""
    n, eps, alpha, tau = 40, 0.75, 0.1, 1.0 / 40
    h = 1.0 / (n + 1)
    A = eps * dirichlet_d2(n, h) + alpha * dirichlet_d1(n, h)
    a, b, c = A[1, 0], A[0, 0], A[0, 1]
    j = np.arange(1, n + 1)
    S = np.sqrt(2 * h) * np.sin(np.outer(j, j) * np.pi * h)
    D = np.diag((a / c) ** (j / 2.0))
    Dinv = np.diag((a / c) ** (-j / 2.0))
    lam = b + 2 * np.sqrt(a * c) * np.cos(j * np.pi / (n + 1))
    phis = phi_functions(tau * A, 2)
    for ell in range(3):
        f = np.array([phi_scalar(tau * l, ell).real for l in lam])
        ref = D @ S @ np.diag(f) @ S @ Dinv
        err = np.max(np.abs(phis[ell] - ref)) / np.max(np.abs(ref))
        assert err < 1e-13, (ell, err)


@pytest.mark.parametrize("cplx", [False, True])
def test_squaring_identity(cplx):
    """eq. squarephi: phi_l(2X) = 2^{-l} [e^X phi_l(X) + sum_{k=1}^{l} phi_k(X)/(l-k)!]."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((12, 12)) * 0.7
    if cplx:
        X = X + 1j * rng.standard_normal((12, 12)) * 0.7
    p1 = phi_functions(X, 3)
    p2 = phi_functions(2 * X, 3)
    for ell in range(1, 4):
        rhs = p1[0] @ p1[ell]
        for k in range(1, ell + 1):
            rhs = rhs + p1[k] / math.factorial(ell - k)
        rhs = rhs / 2 ** ell
        assert np.max(np.abs(p2[ell] - rhs)) < 1e-12 * np.max(np.abs(rhs))


def test_phi_recurrence():
    """X phi_l(X) = phi_{l-1}(X) - I/(l-1)! (from eq. seriesdef)."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((9, 9))
    p = phi_functions(X, 3)
    for ell in range(1, 4):
        lhs = X @ p[ell]
        rhs = p[ell - 1] - np.eye(9) / math.factorial(ell - 1)
        assert np.max(np.abs(lhs - rhs)) < 1e-13 * max(1, np.max(np.abs(rhs)))
