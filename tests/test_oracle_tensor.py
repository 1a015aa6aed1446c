"""Pins of the oracle's tensor algebra: element loop, dense Kronecker forms,
the exact l = 0 identity and the split error of Theorem 1."""

import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.phi import phi_functions
from oracle.tensor import (dense_kron_product, dense_kron_sum, forloop_tucker, tucker_entry,
                           kron_sum_action, mode_product, tucker, unvec, vec)


def _rand(shape, seed, cplx=False):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    if cplx:
        x = x + 1j * rng.standard_normal(shape)
    return x


@pytest.mark.parametrize("n", [(3,), (2, 3), (3, 4, 2), (2, 3, 2, 2)])
@pytest.mark.parametrize("cplx", [False, True])
def test_tucker_equals_element_loop(n, cplx):
    """eq. forloop, written out as a plain loop, versus the mode-product chain."""
    V = _rand(n, 1, cplx)
    Ms = [_rand((k, k), 10 + i, cplx) for i, k in enumerate(n)]
    assert np.allclose(tucker(V, Ms), forloop_tucker(V, Ms), rtol=1e-13, atol=1e-13)


def test_mode_product_is_not_transposed():
    """A single mode product against a hand-written contraction for d = 3."""
    V = _rand((3, 4, 5), 2)
    M = _rand((4, 4), 3)
    ref = np.zeros_like(V)
    for i1 in range(3):
        for i2 in range(4):
            for i3 in range(5):
                ref[i1, i2, i3] = sum(M[i2, j] * V[i1, j, i3] for j in range(4))
    assert np.allclose(mode_product(V, M, 2), ref, rtol=1e-14, atol=1e-14)


def test_mode_product_rectangular_shape():
    V = _rand((3, 4, 5), 4)
    M = _rand((7, 5), 5)
    assert mode_product(V, M, 3).shape == (3, 4, 7)


def test_vec_is_column_stacking():
    U = np.arange(6.0).reshape(2, 3)  # U[i, j]
    assert np.array_equal(vec(U), np.array([0.0, 3.0, 1.0, 4.0, 2.0, 5.0]))
    assert np.array_equal(unvec(vec(U), (2, 3)), U)


def test_dense_kron_sum_2d_matches_explicit_formula():
    """eq. ODE2d: K = I_2 (x) A_1 + A_2 (x) I_1, built here with explicit kron calls."""
    A1, A2 = _rand((3, 3), 6), _rand((4, 4), 7)
    K = np.kron(np.eye(4), A1) + np.kron(A2, np.eye(3))
    assert np.allclose(dense_kron_sum([A1, A2]), K)
    U = _rand((3, 4), 8)
    # the Sylvester form of the same operator: A_1 U + U A_2^T
    assert np.allclose(unvec(K @ vec(U), (3, 4)), A1 @ U + U @ A2.T)
    assert np.allclose(kron_sum_action(U, [A1, A2]), A1 @ U + U @ A2.T)


@pytest.mark.parametrize("n", [(3, 4, 5), (2, 3, 2, 3)])
def test_kron_sum_action_matches_dense(n):
    As = [_rand((k, k), 20 + i) for i, k in enumerate(n)]
    U = _rand(n, 9)
    K = dense_kron_sum(As)
    assert np.allclose(vec(kron_sum_action(U, As)), K @ vec(U), rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("n", [(3, 4, 5), (4, 3)])
def test_exponential_identity_exact(n):
    """eq. vecexp = eq. tuckerexp: e^{tau K} v = V x_1 e^{tau A_1} ... x_d e^{tau A_d}."""
    tau = 0.3
    As = [_rand((k, k), 30 + i) for i, k in enumerate(n)]
    V = _rand(n, 31)
    lhs = expm(tau * dense_kron_sum(As)) @ vec(V)
    E = [phi_functions(tau * A, 0)[0] for A in As]
    assert np.allclose(vec(tucker(V, E)), lhs, rtol=1e-12, atol=1e-12)
    assert np.allclose(dense_kron_product(E) @ vec(V), lhs, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("ell,c", [(1, -1.0 / 12.0), (2, -1.0 / 36.0)])
def test_theorem1_split_error_leading_term(ell, c):
    """Theorem 1 (eq. dsphi): phi_l(tau K) = (l!)^{d-1} (x)_mu phi_l(tau A_mu) + O(tau^2).

    Expanding both sides in tau gives the leading split error
    tau^2 c_l sum_{mu<nu} A_(x)mu A_(x)nu with c_l = l!/((l+1)!)^2 - 2/(l+2)!
    (c_1 = -1/12, c_2 = -1/36); after removing it the residual must fall like tau^3."""
    n = (3, 4, 5)
    d = len(n)
    As = [_rand((k, k), 40 + i) for i, k in enumerate(n)]
    N = int(np.prod(n))
    # the embedded A_(x)mu = I_d (x) .. A_mu .. (x) I_1
    Aemb = []
    for mu in range(d):
        Aemb.append(dense_kron_sum([A if i == mu else np.zeros_like(A) for i, A in enumerate(As)]))
    cross = sum(Aemb[m] @ Aemb[v] for m in range(d) for v in range(m + 1, d))
    K = dense_kron_sum(As)
    res = []
    for tau in [0.04, 0.02, 0.01]:
        exact = phi_functions(tau * K, ell)[ell]
        split = math.factorial(ell) ** (d - 1) * dense_kron_product(
            [phi_functions(tau * A, ell)[ell] for A in As])
        diff = split - exact
        assert np.max(np.abs(diff)) > 1e-9  # the split is not exact
        res.append(np.max(np.abs(diff - tau ** 2 * c * cross)))
    r1 = math.log(res[0] / res[1]) / math.log(2)
    r2 = math.log(res[1] / res[2]) / math.log(2)
    assert r1 > 2.8 and r2 > 2.8, (res, r1, r2)
    assert N == 60


def test_split_exact_when_operators_vanish():
    """A_mu = 0: (l!)^{d-1} prod (1/l!) = 1/l!, so the split equals phi_l(0) = I/l!."""
    for ell in (1, 2):
        split = math.factorial(ell) ** 2 * dense_kron_product(
            [phi_functions(np.zeros((k, k)), ell)[ell] for k in (2, 3, 2)])
        assert np.allclose(split, np.eye(12) / math.factorial(ell), atol=1e-15)


def test_tucker_entry_matches_forloop_and_tucker():
    """Single entries (the full-size GPU tests sample them) against the element loop
    eq. forloop on a tiny tensor and against the whole Tucker operator on a larger one,
    real and complex; the absolute-value sum bounds the entry."""
    rng = np.random.default_rng(11)
    n = (3, 4, 2)
    V = rng.standard_normal(n)
    Ms = [rng.standard_normal((k, k)) for k in n]
    ref = forloop_tucker(V, Ms)
    for i in [(0, 0, 0), (2, 3, 1), (1, 2, 0)]:
        e, a = tucker_entry(V, Ms, i)
        assert abs(e - ref[i]) <= 1e-14 * a
        assert a >= abs(ref[i])
    n = (9, 7, 8, 5)
    V = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Ms = [rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)) for k in n]
    full = tucker(V, Ms)
    for i in [(0, 0, 0, 0), (8, 6, 7, 4), (3, 1, 5, 2)]:
        e, a = tucker_entry(V, Ms, i)
        assert abs(e - full[i]) <= 1e-14 * a
    # a transposed factor (M_2^T for M_2) is caught
    e, a = tucker_entry(V, [Ms[0], Ms[1].T, Ms[2], Ms[3]], (3, 1, 5, 2))
    assert abs(e - full[3, 1, 5, 2]) > 1e-6 * a
