"""Nonlinearities g(t, U) of the workloads (oracle; test infrastructure only)."""

from __future__ import annotations

import numpy as np


def allen_cahn(t, U, **_):
    """g(u) = u - u^3."""
    return U - U ** 3


def u2_1mu(t, U, **_):
    """g(u) = u^2 (1 - u)."""
    return U * U * (1.0 - U)


def cubic_nls(t, U, kappa=1.0, **_):
    """g(u) = -i kappa |u|^2 u."""
    return -1j * kappa * (np.abs(U) ** 2) * U


def riccati(t, U, B=None, C=None, **_):
    """g(U) = C + U B U (paper eq. Riccati, with U an n1 x n2 matrix)."""
    return C + U @ B @ U


def none(t, U, **_):
    return np.zeros_like(U)


def adr_exact(t, grids):
    """Exact solution u = e^t * 64 prod x_mu (1 - x_mu) of eq. ADR (section 4.2)."""
    q = [x * (1 - x) for x in grids]
    return np.exp(t) * 64.0 * np.einsum("i,j,k->ijk", *q)


def adr_paper(t, U, eps=0.75, alpha=0.1, grids=None, **_):
    """g = 1/(1 + u^2) + Psi(t, x) of eq. ADR, with Psi chosen so that e^t u0 solves
    u_t = eps Laplace(u) + alpha (d_1 + d_2 + d_3) u + g.

    With q_mu = x_mu (1 - x_mu): Laplace(u) = 64 e^t sum_mu q_mu'' prod_{nu != mu} q_nu
    (q'' = -2) and sum_mu d_mu u = 64 e^t sum_mu q_mu' prod_{nu != mu} q_nu
    (q' = 1 - 2x); u_t = u."""
    x1, x2, x3 = grids
    q = [x * (1 - x) for x in grids]
    dq = [1 - 2 * x for x in grids]
    e = np.exp(t) * 64.0
    lap = e * (-2.0) * (np.einsum("i,j,k->ijk", np.ones_like(x1), q[1], q[2])
                        + np.einsum("i,j,k->ijk", q[0], np.ones_like(x2), q[2])
                        + np.einsum("i,j,k->ijk", q[0], q[1], np.ones_like(x3)))
    adv = e * (np.einsum("i,j,k->ijk", dq[0], q[1], q[2])
               + np.einsum("i,j,k->ijk", q[0], dq[1], q[2])
               + np.einsum("i,j,k->ijk", q[0], q[1], dq[2]))
    u = adr_exact(t, grids)
    psi = u - eps * lap - alpha * adv - 1.0 / (1.0 + u * u)
    return 1.0 / (1.0 + U * U) + psi


REGISTRY = {
    "none": none,
    "allen_cahn": allen_cahn,
    "u2_1mu": u2_1mu,
    "cubic_nls": cubic_nls,
    "riccati": riccati,
    "adr_paper": adr_paper,
}


def make_g(name, params=None):
    """Bind g's parameters: returns g(t, U)."""
    f = REGISTRY[name]
    params = dict(params or {})
    return lambda t, U: f(t, U, **params)
