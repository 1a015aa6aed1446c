"""phi-functions of small dense matrices (oracle; test infrastructure only).

Definitions (paper section 1, eqs. integraldef and seriesdef):
    phi_0(X) = e^X,
    phi_l(X) = 1/(l-1)! * int_0^1 e^{(1-s)X} s^{l-1} ds = sum_{i>=0} X^i / (i+l)!,  l > 0.

Here all of phi_0 .. phi_p are read off one matrix exponential: for the
block upper-triangular matrix

    Z = [[X, I, 0, ..., 0],
         [0, 0, I, ..., 0],
         ...
         [0, 0, 0, ..., I],
         [0, 0, 0, ..., 0]]          ((p+1) x (p+1) blocks of size n),

the first block row of e^Z is [phi_0(X), phi_1(X), ..., phi_p(X)]
(Al-Mohy & Higham, SIAM J. Sci. Comput. 33 (2011), Thm. 2.1; Sidje's Expokit).
The exponential itself is SciPy's ``expm`` (a library step).
"""

from __future__ import annotations

import math
from typing import List

import numpy as np
from scipy.linalg import expm


def phi_functions(X: np.ndarray, ell_max: int) -> List[np.ndarray]:
    """Return [phi_0(X), ..., phi_{ell_max}(X)] for a square X (float64 or complex128)."""
    X = np.asarray(X)
    n = X.shape[0]
    p = int(ell_max)
    dtype = np.result_type(X.dtype, np.float64)
    Z = np.zeros(((p + 1) * n, (p + 1) * n), dtype=dtype)
    Z[:n, :n] = X
    eye = np.eye(n, dtype=dtype)
    for k in range(p):
        Z[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = eye
    E = expm(Z)
    return [np.array(E[:n, k * n:(k + 1) * n]) for k in range(p + 1)]


def phi_series(X: np.ndarray, ell: int, terms: int = 60) -> np.ndarray:
    """Truncated Taylor series of eq. seriesdef, sum_{i<terms} X^i/(i+ell)!.

    Plain definition, usable only where ||X|| is small enough for the
    truncation and the cancellation to be harmless (test pins)."""
    X = np.asarray(X)
    n = X.shape[0]
    term = np.eye(n, dtype=np.result_type(X.dtype, np.float64))
    acc = term / math.factorial(ell)
    for i in range(1, terms):
        term = term @ X
        acc = acc + term / math.factorial(i + ell)
    return acc


def direction_phis(A_list, tau: float, ell_max: int) -> List[List[np.ndarray]]:
    """phi_0 .. phi_{ell_max} of tau*A_mu for every direction mu (section 3.1:
    the small matrices are computed once before the time stepping)."""
    return [phi_functions(tau * np.asarray(A), ell_max) for A in A_list]
