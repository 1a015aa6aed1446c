"""Pins of the oracle's exponential Rosenbrock-Euler phisplit step for Riccati-type
matrix equations (eqs. expRosEuler and expRosEulertensor; the Kronecker-sum
Jacobian of the Riccati right-hand side, section 4.1).

* The Jacobian directions J1 = A1 + U B, J2 = A2 + (B U)^T are checked against
  central differences of f, which are exact for a quadratic f up to rounding.
* The split step is checked against the unsplit step with the exact phi_1 of
  the assembled Jacobian (dense brute force on tiny sizes): by Theorem 1 they
  differ by O(tau^3) per step.
* The scheme's order, 2, is observed against a tight-tolerance Runge-Kutta
  reference (scipy DOP853) of the vec form.
"""

import numpy as np
from scipy.integrate import solve_ivp

from oracle.schemes import (riccati_jacobian_directions, riccati_rhs, rosenbrock_euler_riccati_step,
                            rosenbrock_euler_riccati_step_unsplit, run_rosenbrock_euler_riccati)


def _instance(n1, n2, seed, stiff=20.0):
    rng = np.random.default_rng(seed)

    def lap(n):
        h = 1.0 / (n + 1)
        return (np.diag(-2 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) / h**2

    A1 = stiff / (n1 + 1) ** 2 * lap(n1) + 0.3 * rng.standard_normal((n1, n1))
    A2 = stiff / (n2 + 1) ** 2 * lap(n2) + 0.3 * rng.standard_normal((n2, n2))
    B = 0.5 * rng.standard_normal((n2, n1))
    C = 0.5 * rng.standard_normal((n1, n2))
    U0 = 0.5 * rng.standard_normal((n1, n2))
    return A1, A2, B, C, U0


def test_jacobian_directions_match_central_differences():
    A1, A2, B, C, U = _instance(6, 9, 1)
    V = np.random.default_rng(2).standard_normal(U.shape)
    J1, J2 = riccati_jacobian_directions(U, A1, A2, B)
    for eps in (1e-1, 1e-3):
        fd = (riccati_rhs(U + eps * V, A1, A2, B, C) - riccati_rhs(U - eps * V, A1, A2, B, C)) / (2 * eps)
        lin = J1 @ V + V @ J2.T
        assert np.abs(fd - lin).max() <= 1e-11 * np.abs(lin).max() / eps


def test_jacobian_is_the_kronecker_sum():
    """vec(J1 V + V J2^T) = (I (x) J1 + J2 (x) I) vec V with vec first index fastest."""
    A1, A2, B, C, U = _instance(4, 5, 3)
    J1, J2 = riccati_jacobian_directions(U, A1, A2, B)
    V = np.random.default_rng(4).standard_normal(U.shape)
    K = np.kron(np.eye(5), J1) + np.kron(J2, np.eye(4))
    assert np.allclose(K @ V.reshape(-1, order="F"), (J1 @ V + V @ J2.T).reshape(-1, order="F"), rtol=1e-13,
                       atol=1e-13)


def test_split_step_differs_from_unsplit_by_third_order():
    A1, A2, B, C, U = _instance(4, 5, 5)
    d = []
    for tau in (0.005, 0.0025, 0.00125, 0.000625):  # tau ||J|| from 0.2 down
        a = rosenbrock_euler_riccati_step(U, tau, A1, A2, B, C)
        b = rosenbrock_euler_riccati_step_unsplit(U, tau, A1, A2, B, C)
        d.append(np.abs(a - b).max())
    ratios = [d[k] / d[k + 1] for k in range(len(d) - 1)]
    assert all(6.5 < r < 9.0 for r in ratios), ratios


def test_observed_order_two():
    A1, A2, B, C, U0 = _instance(5, 6, 7, stiff=10.0)
    T = 0.4

    def rhs(t, u):
        U = u.reshape((5, 6), order="F")
        return riccati_rhs(U, A1, A2, B, C).reshape(-1, order="F")

    ref = solve_ivp(rhs, (0.0, T), U0.reshape(-1, order="F"), method="DOP853", rtol=1e-13, atol=1e-14)
    Uref = ref.y[:, -1].reshape((5, 6), order="F")
    errs = []
    for m in (20, 40, 80):
        U = run_rosenbrock_euler_riccati(U0, T / m, m, A1, A2, B, C)
        errs.append(np.abs(U - Uref).max() / np.abs(Uref).max())
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(1.8 < o < 2.3 for o in orders), (errs, orders)


def test_planted_mistake_in_jacobian_is_caught():
    """Dropping the U B V term of the derivative breaks the central-difference pin."""
    A1, A2, B, C, U = _instance(6, 9, 1)
    V = np.random.default_rng(2).standard_normal(U.shape)
    J1_wrong = A1  # missing U B
    J1, J2 = riccati_jacobian_directions(U, A1, A2, B)
    eps = 1e-3
    fd = (riccati_rhs(U + eps * V, A1, A2, B, C) - riccati_rhs(U - eps * V, A1, A2, B, C)) / (2 * eps)
    assert np.abs(fd - (J1_wrong @ V + V @ J2.T)).max() > 1e-3 * np.abs(fd).max()
