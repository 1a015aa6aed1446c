"""The paper's construction of the phi matrices (section 3.1, eq. phiquad with the
squaring recurrence eq. squarephi): phi_setup(..., method="quad") against the
oracle's augmented-matrix exponential, closed forms and the Taylor construction.

Host code only (the library builds phi on the CPU in FP64); no GPU needed.
"""

import ctypes
import math

import numpy as np
import pytest

import paper_2304_02327_amd as px
from paper_2304_02327_amd import _binding as B
from oracle.phi import phi_functions
import workloads as W


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("norm", [0.0, 0.3, 0.999, 1.0, 7.5, 300.0])
@pytest.mark.parametrize("cplx", [False, True])
def test_quad_matches_oracle_across_norms(norm, cplx):
    """||tau A||_1 from 0 (no scaling) through 1 (the scaling threshold) to many squarings.
    The bar grows with the norm: the exponential's relative condition number is of order
    ||X|| (both constructions and the oracle's expm miss by about ||X|| eps at 300)."""
    rng = np.random.default_rng(int(norm * 10) + 3 * cplx)
    A = rng.standard_normal((13, 13))
    if cplx:
        A = A + 1j * rng.standard_normal((13, 13))
    A -= 2.0 * np.eye(13) * np.abs(A).sum(0).max()  # stable: eigenvalues in the left half plane
    A *= norm / max(np.abs(A).sum(0).max(), 1e-300)
    got = px.phi_setup(A, 1.0, 3, method="quad")
    ref = phi_functions(A, 3)
    for ell, (g, r) in enumerate(zip(got, ref)):
        assert _rel(g, r) <= 5e-14 * max(1.0, norm / 4), (ell, _rel(g, r))


@pytest.mark.parametrize("name,tau,ell", [("c1", 1e-3, 1), ("c2", 2e-3, 2), ("c4", 2e-3, 2)])
def test_quad_on_the_workload_operators(name, tau, ell):
    if name == "c1":
        A = W.allen_cahn_2d().A[0]
    elif name == "c2":
        A = W.adr_3d(n=128).A[1]
    else:
        A = W.diffusion_reaction_3d(n=384, steps=1).A[0]
    got = px.phi_setup(A, tau, ell, method="quad")
    ref = phi_functions(tau * A, ell)
    for g, r in zip(got, ref):
        assert _rel(g, r) <= 1e-13


def test_quad_complex_skew_hermitian():
    p = W.nls_3d(n=64)
    got = px.phi_setup(p.A[0], p.tau, 2, method="quad")
    ref = phi_functions(p.tau * p.A[0], 2)
    for g, r in zip(got, ref):
        assert _rel(g, r) <= 1e-13


def test_quad_sine_basis_closed_form():
    """Independent of the oracle: phi_l(tau c D2) = S diag(phi_l(tau c lambda_k)) S, with
    phi_1(z) = (e^z - 1)/z and phi_2(z) = (e^z - 1 - z)/z^2."""
    n, c, tau = 96, 0.02, 2e-3
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    S = np.sqrt(2 * h) * np.sin(np.outer(j, j) * np.pi * h)
    z = tau * c * (-(4.0 / h ** 2) * np.sin(j * np.pi * h / 2) ** 2)
    got = px.phi_setup(c * W.dirichlet_d2(n, h), tau, 2, method="quad")
    for g, f in ((got[0], np.exp(z)), (got[1], np.expm1(z) / z), (got[2], (np.expm1(z) - z) / z ** 2)):
        ref = S @ np.diag(f) @ S
        assert _rel(g, ref) <= 1e-13


def test_quad_scalar_closed_forms():
    """n = 1: phi_l(z) of a scalar by its series eq. seriesdef, summed in 80-digit decimal
    arithmetic, for z on both sides of the scaling threshold."""
    from decimal import Decimal, getcontext
    getcontext().prec = 80
    for z in (-0.4, 0.9, -1.0, -37.0, 2.5):
        got = px.phi_setup(np.array([[z]]), 1.0, 3, method="quad")
        zd = Decimal(z)
        for ell, g in enumerate(got):
            s = sum(zd ** i / math.factorial(i + ell) for i in range(250))
            assert abs(Decimal(g[0, 0]) - s) <= Decimal(4e-16) * abs(s) * (1 + abs(zd)), (z, ell, g[0, 0], s)


def test_quad_equals_taylor_construction():
    A = W.adr_3d(n=(40, 41, 42)).A[2]
    a = px.phi_setup(A, 2e-3, 2, method="quad")
    b = px.phi_setup(A, 2e-3, 2, method="taylor")
    for x, y in zip(a, b):
        assert _rel(x, y) <= 1e-14


def test_quad_tau_zero():
    """phi_l(0) = I / l!: exact for l = 0, and for l > 0 the quadrature of theta^{l-1}/(l-1)!,
    exact in real arithmetic, up to the rounding of the weights (a few ulp)."""
    A = np.random.default_rng(1).standard_normal((7, 7))
    got = px.phi_setup(A, 0.0, 3, method="quad")
    assert np.array_equal(got[0], np.eye(7))
    for ell in range(1, 4):
        assert np.allclose(got[ell], np.eye(7) / math.factorial(ell), rtol=0, atol=4e-16)


def test_quad_rejects_bad_arguments():
    A = np.eye(3)
    with pytest.raises(px.ExpintError) as e:
        px.phi_setup(A, float("nan"), 1, method="quad")
    assert e.value.code == B.ENUMERIC
    with pytest.raises(px.ExpintError) as e:
        px.phi_setup(A, 0.1, 4, method="quad")
    assert e.value.code == B.EINVAL
    dp = ctypes.POINTER(ctypes.c_double)
    src = np.eye(3)
    out = np.zeros(27)
    assert B.lib.phi_setup_ex(3, src.ctypes.data_as(dp), 3, 0.1, 2, 7, B.F64, out.ctypes.data_as(dp), 3) == B.EINVAL
    assert B.lib.phi_setup_ex(3, src.ctypes.data_as(dp), 3, 0.1, 2, 1, 5, out.ctypes.data_as(dp), 3) == B.EINVAL


def test_planted_wrong_quadrature_is_caught():
    """A rule with too few nodes (4 Gauss-Lobatto nodes, exact to degree 5 only) misses
    the oracle by far more than the bar the quad construction meets: the pins above
    would catch a dropped node or a wrong weight."""
    from numpy.polynomial import legendre as L
    import scipy.linalg as sl
    q = 4
    c = np.zeros(q); c[-1] = 1
    x = np.concatenate(([-1.0], np.sort(L.legroots(L.legder(c))), [1.0]))
    w = 1.0 / (q * (q - 1) * L.legval(x, c) ** 2)
    th = (x + 1) / 2
    Y = np.random.default_rng(2).standard_normal((6, 6))
    Y *= 0.99 / np.abs(Y).sum(0).max()
    phi1 = sum(wi * sl.expm((1 - ti) * Y) for wi, ti in zip(w, th))
    assert _rel(phi1, phi_functions(Y, 1)[1]) > 1e-9
