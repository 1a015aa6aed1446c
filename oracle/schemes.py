"""Exponential integrators in tensor (phisplit) form (oracle; test infrastructure only).

Section 3.2 of the paper, with two readings of its ETD2RK tensor formula:

* the factor (l!)^{d-1} of the direction-split phi_l (Theorem 1, eq. dsphi, and
  the definition of P_l^(2) right after it) is applied to every split stage:
  it is 1 for phi_1 and 2^{d-1} for phi_2;
* tau multiplies the whole bracket (K u_n + g_n) in the first ETD2RK stage, as
  in eq. ETD2RK and eq. expEulertensor.

The direction matrices phi_l(tau A_mu) come from ``oracle.phi`` unless the
caller passes them in.
"""

from __future__ import annotations

import math
from typing import Callable, List, Optional, Sequence

import numpy as np

from .phi import direction_phis
from .tensor import kron_sum_action, tucker

SCHEME_ELL_MAX = {"lawson_euler": 0, "lawson2b": 0, "exp_euler": 1, "etd2rk": 2}


def split_factor(ell: int, d: int) -> float:
    """(l!)^{d-1}, the scalar of the direction-split phi_l (eq. dsphi)."""
    return float(math.factorial(ell) ** (d - 1))


def lawson_euler_step(U, t, tau, E, g):
    """eq. lawsoneulertensor: U_{n+1} = (U_n + tau G(t_n, U_n)) x_mu e^{tau A_mu}."""
    return tucker(U + tau * g(t, U), E)


def lawson2b_step(U, t, tau, E, g):
    """eq. lawson2tensor: U_n2 = (U_n + tau G_n) x_mu e^{tau A_mu};
    U_{n+1} = (U_n + tau/2 G_n) x_mu e^{tau A_mu} + tau/2 G(t_{n+1}, U_n2)."""
    Gn = g(t, U)
    Un2 = tucker(U + tau * Gn, E)
    return tucker(U + 0.5 * tau * Gn, E) + 0.5 * tau * g(t + tau, Un2)


def exp_euler_step(U, t, tau, A, P1, g):
    """eq. expEulertensor: U_{n+1} = U_n + (tau (sum_mu U_n x_mu A_mu + G_n)) x_mu phi_1(tau A_mu).

    The split factor (1!)^{d-1} equals 1."""
    W = tau * (kron_sum_action(U, A) + g(t, U))
    return U + split_factor(1, U.ndim) * tucker(W, P1)


def etd2rk_step(U, t, tau, A, P1, P2, g):
    """ETD2RK phisplit (eq. ETD2RKtensor read with the factor (l!)^{d-1} and tau on
    the whole first bracket):
        U_n2    = U_n + (tau (K U_n + G_n)) x_mu phi_1(tau A_mu)
        U_{n+1} = U_n2 + (2!)^{d-1} (tau (G(t_{n+1}, U_n2) - G_n)) x_mu phi_2(tau A_mu)."""
    d = U.ndim
    Gn = g(t, U)
    Un2 = U + split_factor(1, d) * tucker(tau * (kron_sum_action(U, A) + Gn), P1)
    W2 = tau * (g(t + tau, Un2) - Gn)
    return Un2 + split_factor(2, d) * tucker(W2, P2)


class Integrator:
    """Constant-step integrator: builds phi_l(tau A_mu) once (section 3.1 / 4.2), then steps."""

    def __init__(self, A_list: Sequence[np.ndarray], tau: float, scheme: str,
                 g: Callable, phis: Optional[List[List[np.ndarray]]] = None):
        if scheme not in SCHEME_ELL_MAX:
            raise ValueError(f"unknown scheme {scheme!r}")
        self.A = [np.asarray(a) for a in A_list]
        self.tau = float(tau)
        self.scheme = scheme
        self.g = g
        self.phis = phis if phis is not None else direction_phis(self.A, self.tau, SCHEME_ELL_MAX[scheme])

    def phi(self, ell):
        return [p[ell] for p in self.phis]

    def step(self, U, t):
        tau, g = self.tau, self.g
        if self.scheme == "lawson_euler":
            return lawson_euler_step(U, t, tau, self.phi(0), g)
        if self.scheme == "lawson2b":
            return lawson2b_step(U, t, tau, self.phi(0), g)
        if self.scheme == "exp_euler":
            return exp_euler_step(U, t, tau, self.A, self.phi(1), g)
        return etd2rk_step(U, t, tau, self.A, self.phi(1), self.phi(2), g)

    def run(self, U0, t0: float, steps: int, callback: Optional[Callable] = None):
        U = np.array(U0)
        t = float(t0)
        for k in range(steps):
            U = self.step(U, t)
            t = t0 + (k + 1) * self.tau
            if callback is not None:
                callback(k + 1, t, U)
        return U


def integrator_for(problem, phis=None) -> Integrator:
    """Integrator for a ``workloads.Problem``."""
    from .nonlinear import make_g
    return Integrator(problem.A, problem.tau, problem.scheme,
                      make_g(problem.g, problem.g_params), phis=phis)


def run_problem(problem, steps: Optional[int] = None, phis=None, callback=None):
    """Integrate a ``workloads.Problem`` for ``steps`` (default: problem.steps) steps."""
    integ = integrator_for(problem, phis)
    return integ.run(problem.u0, problem.t0, problem.steps if steps is None else steps, callback)


# ---------------------------------------------------------------------------
# Exponential Rosenbrock-Euler for Riccati-type matrix equations
# ---------------------------------------------------------------------------

def riccati_rhs(U, A1, A2, B, C):
    """f(U) = A1 U + U A2^T + C + U B U (section 1, eq. Riccati, in the matrix form
    whose vec is K u + g(u) with K = A2 (+) A1, eq. ODE2d)."""
    return A1 @ U + U @ A2.T + C + U @ B @ U


def riccati_jacobian_directions(U, A1, A2, B):
    """Directions of the Jacobian of ``riccati_rhs`` at U.

    The derivative of f at U in direction V is A1 V + V A2^T + V B U + U B V
    = J1 V + V J2^T with J1 = A1 + U B and J2 = A2 + (B U)^T, so the Jacobian is the
    Kronecker sum J2 (+) J1 that the Rosenbrock-Euler phisplit scheme assumes
    (section 3.2 before eq. expRosEulertensor; the Kronecker structure of the
    Riccati Jacobian in section 4.1)."""
    return A1 + U @ B, A2 + (B @ U).T


def rosenbrock_euler_riccati_step(U, tau, A1, A2, B, C):
    """One exponential Rosenbrock-Euler phisplit step (eq. expRosEulertensor):
    U + (tau f(U)) x_1 phi_1(tau J1) x_2 phi_1(tau J2), with tau on the whole bracket
    as in eq. expRosEuler.  A 2-tensor times M1 in mode 1 and M2 in mode 2 is
    M1 V M2^T."""
    from .phi import phi_functions
    J1, J2 = riccati_jacobian_directions(U, A1, A2, B)
    P1 = phi_functions(tau * J1, 1)[1]
    P2 = phi_functions(tau * J2, 1)[1]
    return U + P1 @ (tau * riccati_rhs(U, A1, A2, B, C)) @ P2.T


def rosenbrock_euler_riccati_step_unsplit(U, tau, A1, A2, B, C):
    """The same step with the exact phi_1 of the whole Jacobian K_n = I (x) J1 + J2 (x) I
    (eq. expRosEuler on vec U, first index fastest): a dense brute force for tiny sizes."""
    from .phi import phi_functions
    n1, n2 = U.shape
    J1, J2 = riccati_jacobian_directions(U, A1, A2, B)
    Kn = np.kron(np.eye(n2), J1) + np.kron(J2, np.eye(n1))
    f = riccati_rhs(U, A1, A2, B, C).reshape(-1, order="F")
    u = U.reshape(-1, order="F") + tau * (phi_functions(tau * Kn, 1)[1] @ f)
    return u.reshape((n1, n2), order="F")


def run_rosenbrock_euler_riccati(U0, tau, steps, A1, A2, B, C):
    U = np.array(U0, dtype=float)
    for _ in range(steps):
        U = rosenbrock_euler_riccati_step(U, tau, A1, A2, B, C)
    return U
