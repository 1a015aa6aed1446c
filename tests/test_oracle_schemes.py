"""Pins of the oracle's time-stepping schemes.

* the relative errors the paper prints for its ADR experiment (section 4.2),
  to at least 9 significant digits, and the printed observed orders;
* brute force with dense phi_l(tau K) on tiny sizes;
* special cases (d = 1, g = 0, constant g) and the NLS mass identity.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import nonlinear, norms, schemes
from oracle.phi import phi_functions
from oracle.tensor import dense_kron_sum, tucker, unvec, vec
from workloads import adr_paper, nls_3d, random_dense_problem, riccati_batch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adr_printed_errors.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _case(n, scheme):
    for c in _golden():
        if tuple(c["n"]) == tuple(n) and c["scheme"] == scheme:
            return c
    raise KeyError((n, scheme))


def _adr_error(n, scheme, steps):
    p = adr_paper(n, steps=steps, scheme=scheme)
    U = schemes.run_problem(p)
    return norms.rel_inf(U, nonlinear.adr_exact(1.0, p.g_params["grids"]))


# (n, scheme, index into the printed series); the cheap ones run on every CPU pass
PRINTED = [
    ((40, 41, 42), "etd2rk", 0),
    ((40, 41, 42), "etd2rk", 1),
    ((40, 41, 42), "exp_euler", 0),
    ((40, 41, 42), "exp_euler", 1),
    ((40, 41, 42), "lawson_euler", 0),
    ((40, 41, 42), "lawson2b", 0),
    ((80, 81, 82), "etd2rk", 0),
    ((80, 81, 82), "exp_euler", 0),
]


@pytest.mark.parametrize("n,scheme,k", PRINTED)
def test_printed_adr_error(n, scheme, k):
    c = _case(n, scheme)
    err = _adr_error(n, scheme, c["steps"][k])
    printed = c["errors"][k]
    assert abs(err - printed) <= 2e-9 * printed, (err, printed)


@pytest.mark.parametrize("scheme", ["etd2rk", "exp_euler"])
def test_printed_order(scheme):
    c = _case((40, 41, 42), scheme)
    errs = [_adr_error((40, 41, 42), scheme, m) for m in c["steps"][:2]]
    order = norms.observed_orders(errs, c["steps"][:2])[0]
    assert round(order, 2) == c["orders"][1]


def test_etd2rk_needs_split_factor():
    """Without (2!)^{d-1} the printed ETD2RK error is not reproduced (reading of eq. ETD2RKtensor)."""
    p = adr_paper((40, 41, 42), steps=40, scheme="etd2rk")
    g = nonlinear.make_g(p.g, p.g_params)
    integ = schemes.integrator_for(p)
    U, t = p.u0.copy(), 0.0
    for k in range(40):
        Gn = g(t, U)
        Un2 = U + tucker(p.tau * (sum(np.moveaxis(np.tensordot(A, U, axes=([1], [m])), 0, m)
                                      for m, A in enumerate(p.A)) + Gn), integ.phi(1))
        U = Un2 + tucker(p.tau * (g(t + p.tau, Un2) - Gn), integ.phi(2))  # factor dropped
        t = (k + 1) * p.tau
    err = norms.rel_inf(U, nonlinear.adr_exact(1.0, p.g_params["grids"]))
    assert abs(err - _case((40, 41, 42), "etd2rk")["errors"][0]) > 1e-3


def _dense_phi_step(scheme, U, t, tau, As, g):
    """The same schemes with the unsplit phi_l(tau K) applied to vec(U) (brute force)."""
    n = U.shape
    K = dense_kron_sum(As)
    ph = phi_functions(tau * K, 2)
    u = vec(U)
    G = lambda tt, x: vec(g(tt, unvec(x, n)))
    if scheme == "exp_euler":
        un = u + tau * ph[1] @ (K @ u + G(t, u))
    elif scheme == "etd2rk":
        u2 = u + tau * ph[1] @ (K @ u + G(t, u))
        un = u2 + tau * ph[2] @ (G(t + tau, u2) - G(t, u))
    elif scheme == "lawson_euler":
        un = ph[0] @ (u + tau * G(t, u))
    else:
        u2 = ph[0] @ (u + tau * G(t, u))
        un = ph[0] @ (u + 0.5 * tau * G(t, u)) + 0.5 * tau * G(t + tau, u2)
    return unvec(un, n)


@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk", "lawson_euler", "lawson2b"])
def test_one_dimension_has_no_split(scheme):
    """d = 1: the split phi is phi itself, so the tensor scheme equals the dense scheme."""
    p = random_dense_problem((7,), seed=11, tau=0.2, scheme=scheme)
    g = nonlinear.make_g(p.g, p.g_params)
    integ = schemes.integrator_for(p)
    U1 = integ.step(p.u0, 0.0)
    U2 = _dense_phi_step(scheme, p.u0, 0.0, p.tau, p.A, g)
    assert np.allclose(U1, U2, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("scheme", ["lawson_euler", "lawson2b"])
def test_lawson_schemes_have_no_split_error(scheme):
    p = random_dense_problem((3, 4, 2), seed=12, tau=0.1, scheme=scheme)
    g = nonlinear.make_g(p.g, p.g_params)
    U1 = schemes.integrator_for(p).step(p.u0, 0.0)
    U2 = _dense_phi_step(scheme, p.u0, 0.0, p.tau, p.A, g)
    assert np.allclose(U1, U2, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk"])
def test_split_local_error_is_third_order(scheme):
    """One phisplit step differs from the unsplit step by O(tau^3) (Theorem 1 with the
    tau in front of every phi), so halving tau divides the difference by ~8."""
    diffs = []
    for tau in (0.08, 0.04, 0.02):
        p = random_dense_problem((3, 4, 3), seed=13, tau=tau, scheme=scheme)
        g = nonlinear.make_g(p.g, p.g_params)
        U1 = schemes.integrator_for(p).step(p.u0, 0.0)
        U2 = _dense_phi_step(scheme, p.u0, 0.0, tau, p.A, g)
        diffs.append(np.max(np.abs(U1 - U2)))
    rates = [math.log(diffs[i] / diffs[i + 1]) / math.log(2) for i in range(2)]
    assert all(r > 2.7 for r in rates), (diffs, rates)


def test_lawson_euler_linear_homogeneous_is_exact():
    """g = 0: m Lawson-Euler steps equal one Tucker with e^{m tau A_mu} (exactness for
    linear homogeneous problems, section 2)."""
    p = random_dense_problem((4, 3, 5), seed=14, tau=0.05, scheme="lawson_euler", g="none")
    U = schemes.run_problem(p, steps=6)
    E6 = [expm(6 * p.tau * A) for A in p.A]
    assert np.allclose(U, tucker(p.u0, E6), rtol=1e-12, atol=1e-13)


def test_exp_euler_constant_forcing_is_exact():
    """d = 1, g = const: exponential Euler is exact for linear constant-coefficient problems
    (section 2): u(t) = e^{tA} u0 + t phi_1(tA) c."""
    rng = np.random.default_rng(15)
    A = rng.standard_normal((6, 6))
    c = rng.standard_normal(6)
    u0 = rng.standard_normal(6)
    integ = schemes.Integrator([A], 0.05, "exp_euler", lambda t, U: c)
    U = integ.run(u0, 0.0, 8)
    ph = phi_functions(0.4 * A, 1)
    assert np.allclose(U, ph[0] @ u0 + 0.4 * ph[1] @ c, rtol=1e-12, atol=1e-13)


def test_nls_mass_identity():
    """Lawson-Euler for A_mu = (i/2) D2 (skew-Hermitian, so e^{tau A_mu} is unitary) and
    g = -i |u|^2 u: sum |U_{n+1}|^2 = sum |U_n|^2 (1 + tau^2 |U_n|^4) exactly."""
    p = nls_3d(n=16, steps=3)
    integ = schemes.integrator_for(p)
    U = p.u0
    for k in range(3):
        Un = integ.step(U, k * p.tau)
        lhs = np.sum(np.abs(Un) ** 2)
        rhs = np.sum(np.abs(U) ** 2 * (1 + p.tau ** 2 * np.abs(U) ** 4))
        assert abs(lhs - rhs) < 1e-13 * rhs
        U = Un


def test_riccati_tensor_form_matches_vector_form():
    """eq. Riccati vs eq. ODE2d: ETD2RK phisplit in matrix form (A_1 U + U A_2^T, C + U B U)
    equals the same scheme on vec(U) with K = I (x) A_1 + A_2 (x) I and the split phi built
    as an explicit Kronecker product."""
    inst = riccati_batch(count=1, nmin=5, nmax=7, seed=21)[0]
    tau = 1e-2
    rng = np.random.default_rng(22)
    U0 = 0.3 * rng.standard_normal((inst.n1, inst.n2))
    g = nonlinear.make_g("riccati", {"B": inst.B, "C": inst.C})
    integ = schemes.Integrator([inst.A1, inst.A2], tau, "etd2rk", g)
    U1 = integ.step(U0, 0.0)
    K = np.kron(np.eye(inst.n2), inst.A1) + np.kron(inst.A2, np.eye(inst.n1))
    P1 = np.kron(phi_functions(tau * inst.A2, 1)[1], phi_functions(tau * inst.A1, 1)[1])
    P2 = 2.0 * np.kron(phi_functions(tau * inst.A2, 2)[2], phi_functions(tau * inst.A1, 2)[2])
    G = lambda u: vec(inst.C + unvec(u, U0.shape) @ inst.B @ unvec(u, U0.shape))
    u = vec(U0)
    u2 = u + P1 @ (tau * (K @ u + G(u)))
    un = u2 + P2 @ (tau * (G(u2) - G(u)))
    assert np.allclose(vec(U1), un, rtol=1e-12, atol=1e-13)
