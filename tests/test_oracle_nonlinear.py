"""Pins of the oracle's nonlinearities g against solutions the mathematics fixes.

With every A_mu = 0 each scheme of section 2 reduces to a textbook one-step
method for u' = g(u): phi_l(0) = I / l!, so exponential Euler and Lawson-Euler
are the explicit Euler method and ETD2RK (with its split factor 2^{d-1} against
the (1/2)^d of phi_2(0) along d directions) and Lawson2b are Heun's method.
Their solutions must then converge, with order 1 and 2, to the exact solution
of the scalar (or matrix) ODE, which is known in closed form for every g:

* u' = u - u^3 (Allen-Cahn): u(t) = u0 e^t / sqrt(1 + u0^2 (e^{2t} - 1))
  (a Bernoulli equation: v = u^-2 solves v' = 2 - 2v);
* u' = u^2 (1 - u): F(u(t)) = F(u0) + t with F(u) = ln(u / (1 - u)) - 1/u,
  whose derivative is 1 / (u^2 (1 - u)); solved for u by bracketing;
* u' = -i kappa |u|^2 u (cubic NLS): |u| is constant, so
  u(t) = u0 exp(-i kappa |u0|^2 t), which fixes the sign of i and kappa;
* U' = A1 U + U A2^T + C + U B U (eq. Riccati): Radon's lemma, U = Y X^{-1}
  with d/dt [X; Y] = [[-A2^T, -B], [C, A1]] [X; Y], X(0) = I, Y(0) = U0, so the
  exact solution is one matrix exponential of a linear system.

Every pin is also run against planted mistakes in g (u^2 for u^3, u (1 - u) for
u^2 (1 - u), +i for -i, B transposed in U B U, C dropped), each of which must
miss the exact solution by far more than the bound.
"""

import math

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.optimize import brentq

from oracle import nonlinear, norms, schemes


def _zero_ops(shape, dtype=float):
    return [np.zeros((n, n), dtype=dtype) for n in shape]


def _run(scheme, g, U0, T, steps, shape=None, A=None):
    """The oracle integrator with the given g from U0 to T in `steps` steps."""
    if A is None:
        A = _zero_ops(shape or U0.shape, np.result_type(U0.dtype, float))
    integ = schemes.Integrator(A, T / steps, scheme, g)
    return integ.run(U0, 0.0, steps)


def _errors(scheme, g, U0, T, exact, steps_list, A=None):
    return [norms.rel_inf(_run(scheme, g, U0, T, m, A=A), exact) for m in steps_list]


STEPS = (40, 80, 160)
ORDER = {"exp_euler": 1, "lawson_euler": 1, "etd2rk": 2, "lawson2b": 2}


def _check_order(errs, scheme, tol=0.15):
    orders = norms.observed_orders(errs, STEPS)
    assert all(abs(o - ORDER[scheme]) < tol for o in orders), (scheme, errs, orders)


# ---------------------------------------------------------------------------
# closed-form solutions
# ---------------------------------------------------------------------------

def allen_cahn_exact(u0, t):
    e = math.exp(t)
    return u0 * e / np.sqrt(1.0 + u0 * u0 * (e * e - 1.0))


def u2_1mu_exact(u0, t):
    F = lambda u: math.log(u / (1.0 - u)) - 1.0 / u
    out = np.empty_like(u0)
    for idx, a in np.ndenumerate(u0):
        c = F(a) + t
        out[idx] = brentq(lambda u: F(u) - c, a, 1.0 - 1e-15, xtol=1e-16, rtol=1e-15, maxiter=200)
    return out


def nls_exact(u0, t, kappa):
    return u0 * np.exp(-1j * kappa * np.abs(u0) ** 2 * t)


def riccati_exact(U0, t, A1, A2, B, C):
    n1, n2 = U0.shape
    H = np.block([[-A2.T, -B], [C, A1]])
    Z = expm(t * H) @ np.vstack([np.eye(n2), U0])
    X, Y = Z[:n2], Z[n2:]
    return np.linalg.solve(X.T, Y.T).T  # Y X^{-1}


# ---------------------------------------------------------------------------
# the closed forms themselves, against a high-order reference
# ---------------------------------------------------------------------------

def test_closed_forms_solve_their_odes():
    """The closed forms against SciPy's DOP853 on the same right-hand sides written
    out here (not the oracle's), so that a slip in a closed form cannot make a
    wrong g look right."""
    from scipy.integrate import solve_ivp
    u0 = np.array([-0.7, 0.2, 0.55])
    ref = solve_ivp(lambda t, y: y - y ** 3, (0, 1.0), u0, method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    assert np.max(np.abs(allen_cahn_exact(u0, 1.0) - ref)) < 1e-11
    v0 = np.array([0.1, 0.4, 0.8])
    ref = solve_ivp(lambda t, y: y * y * (1 - y), (0, 1.0), v0, method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    assert np.max(np.abs(u2_1mu_exact(v0, 1.0) - ref)) < 1e-11
    z0 = np.array([0.3 + 0.4j, -0.9 + 0.1j])
    f = lambda t, y: (lambda z: np.concatenate([(-1j * 1.5 * np.abs(z) ** 2 * z).real,
                                                (-1j * 1.5 * np.abs(z) ** 2 * z).imag]))(y[:2] + 1j * y[2:])
    ref = solve_ivp(f, (0, 1.0), np.concatenate([z0.real, z0.imag]), method="DOP853", rtol=1e-13,
                    atol=1e-15).y[:, -1]
    assert np.max(np.abs(nls_exact(z0, 1.0, 1.5) - (ref[:2] + 1j * ref[2:]))) < 1e-11
    rng = np.random.default_rng(7)
    n1, n2 = 3, 4
    A1, A2 = -np.eye(n1) + 0.3 * rng.standard_normal((n1, n1)), -np.eye(n2) + 0.3 * rng.standard_normal((n2, n2))
    B, C = 0.5 * rng.standard_normal((n2, n1)), 0.5 * rng.standard_normal((n1, n2))
    U0 = 0.3 * rng.standard_normal((n1, n2))
    rhs = lambda t, y: (lambda U: (A1 @ U + U @ A2.T + C + U @ B @ U).ravel())(y.reshape(n1, n2))
    ref = solve_ivp(rhs, (0, 0.5), U0.ravel(), method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1].reshape(n1, n2)
    assert np.max(np.abs(riccati_exact(U0, 0.5, A1, A2, B, C) - ref)) < 1e-11


# ---------------------------------------------------------------------------
# pointwise nonlinearities
# ---------------------------------------------------------------------------

U0_AC = np.array([[-0.85, -0.3, 0.05], [0.4, 0.7, 0.88]])          # a 2-tensor (d = 2)
U0_U2 = np.array([[[0.05, 0.3], [0.6, 0.9]], [[0.15, 0.45], [0.75, 0.97]]])  # d = 3, values in (0, 1)
U0_NLS = np.array([[0.3 + 0.4j, -0.9 + 0.1j, 0.2 - 0.7j], [1.1 + 0.0j, -0.2 - 0.2j, 0.05 + 0.6j]])
KAPPA = 1.5


AC_BOUND = {"exp_euler": 5e-3, "lawson_euler": 5e-3, "etd2rk": 2e-5, "lawson2b": 2e-5}


@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk", "lawson_euler", "lawson2b"])
def test_allen_cahn_closed_form(scheme):
    T = 1.0
    exact = allen_cahn_exact(U0_AC, T)
    errs = _errors(scheme, nonlinear.make_g("allen_cahn"), U0_AC, T, exact, STEPS)
    _check_order(errs, scheme)
    assert errs[-1] < AC_BOUND[scheme]


U2_BOUND = {"exp_euler": 3e-3, "lawson_euler": 3e-3, "etd2rk": 2e-5, "lawson2b": 2e-5}


@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk", "lawson_euler", "lawson2b"])
def test_u2_1mu_closed_form(scheme):
    T = 1.0
    exact = u2_1mu_exact(U0_U2, T)
    errs = _errors(scheme, nonlinear.make_g("u2_1mu"), U0_U2, T, exact, STEPS)
    _check_order(errs, scheme)
    assert errs[-1] < U2_BOUND[scheme]


NLS_BOUND = {"exp_euler": 3e-2, "lawson_euler": 3e-2, "etd2rk": 2e-4, "lawson2b": 2e-4}


@pytest.mark.parametrize("scheme", ["lawson_euler", "lawson2b", "exp_euler", "etd2rk"])
def test_cubic_nls_exact_rotation(scheme):
    T = 1.0
    exact = nls_exact(U0_NLS, T, KAPPA)
    errs = _errors(scheme, nonlinear.make_g("cubic_nls", {"kappa": KAPPA}), U0_NLS, T, exact, STEPS)
    _check_order(errs, scheme)
    assert errs[-1] < NLS_BOUND[scheme]


def _riccati_case(n1, n2, seed):
    rng = np.random.default_rng(seed)
    A1 = -2.0 * np.eye(n1) + 0.4 * rng.standard_normal((n1, n1))
    A2 = -1.0 * np.eye(n2) + 0.4 * rng.standard_normal((n2, n2))
    B = 0.6 * rng.standard_normal((n2, n1))
    C = 0.6 * rng.standard_normal((n1, n2))
    U0 = 0.4 * rng.standard_normal((n1, n2))
    return A1, A2, B, C, U0


RIC_BOUND = {"exp_euler": 5e-3, "etd2rk": 5e-5}


@pytest.mark.parametrize("n1,n2", [(1, 1), (3, 3), (3, 5), (4, 2)])
@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk"])
def test_riccati_radon_exact(n1, n2, scheme):
    """The oracle's matrix g = C + U B U inside the Kronecker-form schemes (A1 and
    A2 are the direction matrices, so these runs split) against the exact
    solution: the split error and the time error both vanish with tau, at the
    scheme's order."""
    A1, A2, B, C, U0 = _riccati_case(n1, n2, 10 * n1 + n2)
    T = 0.5
    exact = riccati_exact(U0, T, A1, A2, B, C)
    g = nonlinear.make_g("riccati", {"B": B, "C": C})
    errs = _errors(scheme, g, U0, T, exact, STEPS, A=[A1, A2])
    _check_order(errs, scheme, tol=0.2)
    assert errs[-1] < RIC_BOUND[scheme]


def test_riccati_scalar_closed_form():
    """n1 = n2 = 1: u' = b u^2 + (a1 + a2) u + c with constant coefficients,
    solved through its two real roots r1 > r2 of b r^2 + (a1 + a2) r + c:
    (u - r1) / (u - r2) = (u0 - r1) / (u0 - r2) e^{b (r1 - r2) t}."""
    a1, a2, b, c, u0 = -1.3, -0.4, 0.8, 0.5, 0.2
    r1, r2 = sorted(np.roots([b, a1 + a2, c]).real, reverse=True)
    T = 0.7
    k = (u0 - r1) / (u0 - r2) * math.exp(b * (r1 - r2) * T)
    exact = (r1 - k * r2) / (1.0 - k)
    assert abs(riccati_exact(np.array([[u0]]), T, np.array([[a1]]), np.array([[a2]]),
                             np.array([[b]]), np.array([[c]]))[0, 0] - exact) < 1e-13
    g = nonlinear.make_g("riccati", {"B": np.array([[b]]), "C": np.array([[c]])})
    U = _run("etd2rk", g, np.array([[u0]]), T, 400, A=[np.array([[a1]]), np.array([[a2]])])
    assert abs(U[0, 0] - exact) < 1e-7


def test_rosenbrock_riccati_radon_exact():
    """The oracle's Rosenbrock-Euler Riccati stepper (its own right-hand side and
    Jacobian directions) converges with order 2 to the exact solution."""
    A1, A2, B, C, U0 = _riccati_case(3, 4, 99)
    T = 0.5
    exact = riccati_exact(U0, T, A1, A2, B, C)
    errs = [norms.rel_inf(schemes.run_rosenbrock_euler_riccati(U0, T / m, m, A1, A2, B, C), exact)
            for m in STEPS]
    orders = norms.observed_orders(errs, STEPS)
    assert all(abs(o - 2) < 0.2 for o in orders), (errs, orders)
    assert errs[-1] < 5e-5


# ---------------------------------------------------------------------------
# planted mistakes: each one must miss the exact solution by far more than the bound
# ---------------------------------------------------------------------------

PLANTED = {
    "allen_cahn u^2 for u^3": ("allen_cahn", lambda t, U: U - U ** 2),
    "allen_cahn sign": ("allen_cahn", lambda t, U: U + U ** 3),
    "u2_1mu u(1-u) for u^2(1-u)": ("u2_1mu", lambda t, U: U * (1.0 - U)),
    "u2_1mu u^2(1+u)": ("u2_1mu", lambda t, U: U * U * (1.0 + U)),
    "cubic_nls +i": ("cubic_nls", lambda t, U: 1j * KAPPA * np.abs(U) ** 2 * U),
    "cubic_nls kappa dropped": ("cubic_nls", lambda t, U: -1j * np.abs(U) ** 2 * U),
    "cubic_nls |u| for |u|^2": ("cubic_nls", lambda t, U: -1j * KAPPA * np.abs(U) * U),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_pointwise_mistakes_fail(name):
    which, bad = PLANTED[name]
    T = 1.0
    if which == "allen_cahn":
        U0, exact, bound = U0_AC, allen_cahn_exact(U0_AC, T), AC_BOUND["etd2rk"]
    elif which == "u2_1mu":
        U0, exact, bound = U0_U2, u2_1mu_exact(U0_U2, T), U2_BOUND["etd2rk"]
    else:
        U0, exact, bound = U0_NLS, nls_exact(U0_NLS, T, KAPPA), NLS_BOUND["etd2rk"]
    with np.errstate(all="ignore"):  # some planted variants blow up to inf / nan
        err = norms.rel_inf(_run("etd2rk", bad, U0, T, STEPS[-1]), exact)
    assert not err <= 100 * bound, (name, err)


@pytest.mark.parametrize("mistake", ["B transposed", "C dropped", "U U B order", "A2 untransposed"])
def test_planted_riccati_mistakes_fail(mistake):
    A1, A2, B, C, U0 = _riccati_case(3, 3, 33)  # square: every variant has valid shapes
    T = 0.5
    exact = riccati_exact(U0, T, A1, A2, B, C)
    if mistake == "B transposed":
        g = lambda t, U: C + U @ B.T @ U
        A = [A1, A2]
    elif mistake == "C dropped":
        g = lambda t, U: U @ B @ U
        A = [A1, A2]
    elif mistake == "U U B order":
        g = lambda t, U: C + U @ U @ B
        A = [A1, A2]
    else:  # the second direction applied as U A2 instead of U A2^T
        g = nonlinear.make_g("riccati", {"B": B, "C": C})
        A = [A1, A2.T]
    with np.errstate(all="ignore"):
        err = norms.rel_inf(_run("etd2rk", g, U0, T, STEPS[-1], A=A), exact)
    assert not err <= 100 * RIC_BOUND["etd2rk"], (mistake, err)
