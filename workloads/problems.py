"""Problem definitions (operators, initial data, g, step size) for every workload.

Finite-difference operators follow the semidiscretisation of paper section 4.2
(second-order centred differences, homogeneous Dirichlet conditions, n inner
points on [0, 1]); the periodic operator is the same 3-point stencil wrapped
around.  Every random draw comes from ``numpy.random.default_rng(seed)``
(PCG64), drawn in memory order (first index fastest), so a problem is fully
determined by its constructor arguments.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

SCHEMES = ("lawson_euler", "lawson2b", "exp_euler", "etd2rk")
NONLINEARITIES = ("none", "allen_cahn", "u2_1mu", "cubic_nls", "adr_paper", "riccati")


# ---------------------------------------------------------------------------
# layout helpers
# ---------------------------------------------------------------------------

def to_memory_order(U: np.ndarray) -> np.ndarray:
    """Natural-index tensor (n_1..n_d) -> C-contiguous (n_d..n_1) array whose
    memory is vec(U) (first index fastest)."""
    return np.ascontiguousarray(U.T)


def from_memory_order(Um: np.ndarray) -> np.ndarray:
    """Inverse of :func:`to_memory_order` (returns a natural-index view)."""
    return np.asarray(Um).T


# ---------------------------------------------------------------------------
# 1-D operators (dense, float64), the building blocks of A_mu
# ---------------------------------------------------------------------------

def dirichlet_d2(n: int, h: float) -> np.ndarray:
    """tridiag(1, -2, 1) / h^2 on n inner points (homogeneous Dirichlet)."""
    D = np.zeros((n, n))
    idx = np.arange(n)
    D[idx, idx] = -2.0
    D[idx[1:], idx[:-1]] = 1.0
    D[idx[:-1], idx[1:]] = 1.0
    return D / (h * h)


def dirichlet_d1(n: int, h: float) -> np.ndarray:
    """Centred first derivative tridiag(-1, 0, +1) / (2h): (D1 u)_j = (u_{j+1} - u_{j-1}) / 2h."""
    D = np.zeros((n, n))
    idx = np.arange(n)
    D[idx[1:], idx[:-1]] = -1.0
    D[idx[:-1], idx[1:]] = 1.0
    return D / (2.0 * h)


def periodic_d2(n: int, h: float) -> np.ndarray:
    """Circulant 3-point second difference on n periodic points."""
    D = np.zeros((n, n))
    idx = np.arange(n)
    D[idx, idx] = -2.0
    D[idx, (idx + 1) % n] += 1.0
    D[idx, (idx - 1) % n] += 1.0
    return D / (h * h)


# ---------------------------------------------------------------------------
# problem records
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """u' = K u + g(t, u), K = A_d (+) ... (+) A_1, in tensor form.

    ``A`` are the dense direction matrices (column index = the index the
    matrix contracts), ``u0`` the natural-index initial tensor.  ``g`` names
    the nonlinearity; ``g_params`` holds its parameters (for ``adr_paper``
    the grid and the coefficients the manufactured source needs).
    """

    name: str
    n: Tuple[int, ...]
    A: List[np.ndarray]
    tau: float
    steps: int
    scheme: str
    g: str
    u0: np.ndarray
    g_params: Dict = field(default_factory=dict)
    t0: float = 0.0
    seed: Optional[int] = None

    @property
    def d(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.u0) or any(np.iscomplexobj(a) for a in self.A)


@dataclass
class RiccatiInstance:
    """One instance of U' = A_1 U + U A_2^T + C + U B U (paper eq. Riccati)."""

    n1: int
    n2: int
    A1: np.ndarray
    A2: np.ndarray
    B: np.ndarray  # n2 x n1
    C: np.ndarray  # n1 x n2
    U0: np.ndarray  # n1 x n2


def _uniform_natural(rng, n, lo, hi):
    """Uniform draws in memory order, returned in natural index order."""
    return from_memory_order(rng.uniform(lo, hi, size=tuple(reversed(n))))


def _normal_natural(rng, n):
    return from_memory_order(rng.standard_normal(size=tuple(reversed(n))))


def _inner_grid(n: int) -> Tuple[np.ndarray, float]:
    h = 1.0 / (n + 1)
    return h * np.arange(1, n + 1), h


# ---------------------------------------------------------------------------
# the five synthetic workloads
# ---------------------------------------------------------------------------

def allen_cahn_2d(n: int = 64, steps: int = 50, tau: float = 1e-3, seed: int = 1) -> Problem:
    """2-D Allen-Cahn: A_mu = 0.01 * D2 (Dirichlet, h = 1/(n+1)), g(u) = u - u^3,
    u0 ~ U(-0.9, 0.9), exponential Euler with the split phi_1."""
    rng = np.random.default_rng(seed)
    _, h = _inner_grid(n)
    A = 0.01 * dirichlet_d2(n, h)
    u0 = _uniform_natural(rng, (n, n), -0.9, 0.9)
    return Problem("allen_cahn_2d", (n, n), [A, A.copy()], tau, steps, "exp_euler",
                   "allen_cahn", np.array(u0, dtype=np.float64), seed=seed)


def adr_3d(n: int = 128, steps: int = 100, tau: float = 2e-3, seed: int = 2,
           beta=(0.5, -0.3, 0.2), scheme: str = "etd2rk") -> Problem:
    """3-D advection-diffusion-reaction: A_mu = 0.02 * D2 + beta_mu * D1 (centred,
    Dirichlet, h = 1/(n+1)), g(u) = u^2 (1 - u), u0 = Gaussian bump of width 0.1
    centred at (1/2, 1/2, 1/2) plus 1e-3 * U(-1, 1) noise; ETD2RK."""
    rng = np.random.default_rng(seed)
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    A, grids = [], []
    for mu in range(3):
        x, h = _inner_grid(nn[mu])
        grids.append(x)
        A.append(0.02 * dirichlet_d2(nn[mu], h) + beta[mu] * dirichlet_d1(nn[mu], h))
    X1, X2, X3 = np.meshgrid(*grids, indexing="ij")
    r2 = (X1 - 0.5) ** 2 + (X2 - 0.5) ** 2 + (X3 - 0.5) ** 2
    u0 = np.exp(-r2 / (2 * 0.1 ** 2)) + 1e-3 * _uniform_natural(rng, nn, -1.0, 1.0)
    return Problem("adr_3d", nn, A, tau, steps, scheme, "u2_1mu", u0, seed=seed)


def nls_3d(n: int = 192, steps: int = 200, tau: float = 1e-3, seed: int = 3,
           kappa: float = 1.0) -> Problem:
    """3-D cubic Schroedinger, periodic on [-pi, pi)^3: A_mu = (i/2) * D2 (periodic,
    h = 2 pi / n), g(u) = -i kappa |u|^2 u, u0 = Gaussian packet (width 0.6) times
    exp(2 i x_1) times seeded phase noise exp(0.1 i xi), xi ~ N(0, 1); Lawson-Euler."""
    rng = np.random.default_rng(seed)
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    A, grids = [], []
    for mu in range(3):
        h = 2 * np.pi / nn[mu]
        grids.append(-np.pi + h * np.arange(nn[mu]))
        A.append(0.5j * periodic_d2(nn[mu], h))
    X1, X2, X3 = np.meshgrid(*grids, indexing="ij")
    xi = _normal_natural(rng, nn)
    u0 = (np.exp(-(X1 ** 2 + X2 ** 2 + X3 ** 2) / (2 * 0.6 ** 2))
          * np.exp(2j * X1) * np.exp(0.1j * xi))
    return Problem("nls_3d", nn, A, tau, steps, "lawson_euler", "cubic_nls",
                   u0.astype(np.complex128), g_params={"kappa": kappa, "h": grids[0][1] - grids[0][0]},
                   seed=seed)


def diffusion_reaction_3d(n: int = 384, steps: int = 20, tau: float = 2e-3, seed: int = 4) -> Problem:
    """3-D diffusion-reaction: A_mu = 0.02 * D2 (Dirichlet, h = 1/(n+1)),
    g(u) = u^2 (1 - u), u0 ~ U(0, 1); ETD2RK."""
    rng = np.random.default_rng(seed)
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    A = []
    for mu in range(3):
        _, h = _inner_grid(nn[mu])
        A.append(0.02 * dirichlet_d2(nn[mu], h))
    u0 = _uniform_natural(rng, nn, 0.0, 1.0)
    return Problem("diffusion_reaction_3d", nn, A, tau, steps, "etd2rk", "u2_1mu",
                   np.array(u0, dtype=np.float64), seed=seed)


def riccati_batch(count: int = 64, nmin: int = 32, nmax: int = 512, seed: int = 5,
                  perturb: float = 0.1, bc_std: float = 0.1) -> List[RiccatiInstance]:
    """Batched Riccati-type instances: n1, n2 ~ U{nmin..nmax}; A_mu = Delta_h +
    perturb * N(0, 1) (Delta_h = tridiag(1, -2, 1) / h^2, h = 1/(n_mu + 1)),
    B (n2 x n1), C (n1 x n2) ~ N(0, bc_std^2), U0 = 0.  Sizes are drawn first,
    then per instance A1, A2, B, C in that order (each in memory order)."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=(count, 2))
    out = []
    for n1, n2 in sizes:
        n1, n2 = int(n1), int(n2)
        A1 = dirichlet_d2(n1, 1.0 / (n1 + 1)) + perturb * rng.standard_normal((n1, n1)).T
        A2 = dirichlet_d2(n2, 1.0 / (n2 + 1)) + perturb * rng.standard_normal((n2, n2)).T
        B = bc_std * rng.standard_normal((n1, n2)).T  # memory order of an n2 x n1 matrix
        C = bc_std * rng.standard_normal((n2, n1)).T  # memory order of an n1 x n2 matrix
        out.append(RiccatiInstance(n1, n2, np.ascontiguousarray(A1), np.ascontiguousarray(A2),
                                   np.ascontiguousarray(B), np.ascontiguousarray(C),
                                   np.zeros((n1, n2))))
    return out


# ---------------------------------------------------------------------------
# the paper's own advection-diffusion-reaction experiment (section 4.2)
# ---------------------------------------------------------------------------

def adr_paper(n=(40, 41, 42), steps: int = 40, scheme: str = "etd2rk",
              eps: float = 0.75, alpha: float = 0.1, T: float = 1.0) -> Problem:
    """Paper section 4.2, eq. ADR: A_mu = eps * D2 + alpha * D1 on n_mu inner points
    of [0, 1], u0 = 64 prod x_mu (1 - x_mu), g = 1/(1 + u^2) + Psi(t, x) with Psi
    manufactured so that u = e^t u0; integrated to T with constant steps."""
    A, grids = [], []
    for nm in n:
        x, h = _inner_grid(nm)
        grids.append(x)
        A.append(eps * dirichlet_d2(nm, h) + alpha * dirichlet_d1(nm, h))
    q = [x * (1 - x) for x in grids]
    u0 = 64.0 * np.einsum("i,j,k->ijk", *q)
    return Problem("adr_paper", tuple(n), A, T / steps, steps, scheme, "adr_paper", u0,
                   g_params={"eps": eps, "alpha": alpha, "grids": grids})


def random_dense_problem(n, seed: int = 7, scale: float = 1.0, tau: float = 0.05,
                         steps: int = 3, scheme: str = "etd2rk", g: str = "u2_1mu",
                         complex_: bool = False) -> Problem:
    """Small problem with dense random A_mu (N(0, scale^2 / n_mu) entries) and
    u0 ~ U(-1, 1); used for brute-force and parity cases of any shape."""
    rng = np.random.default_rng(seed)
    A = []
    for nm in n:
        M = rng.standard_normal((nm, nm)).T * (scale / np.sqrt(nm))
        if complex_:
            M = M + 1j * rng.standard_normal((nm, nm)).T * (scale / np.sqrt(nm))
        A.append(np.ascontiguousarray(M))
    u0 = _uniform_natural(rng, tuple(n), -1.0, 1.0)
    if complex_:
        u0 = u0 + 1j * _uniform_natural(rng, tuple(n), -1.0, 1.0)
    return Problem("random_dense", tuple(n), A, tau, steps, scheme, g, np.array(u0), seed=seed)
