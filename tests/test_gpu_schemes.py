"""GPU parity of the time-stepping plans against the oracle.

FP64 bar: relative max-norm error <= 1e-12 on the final state (and on
intermediate states where checked).  The GPU builds phi with its own host
routine and contracts on FP64 MFMA; the oracle uses SciPy's expm of an
augmented matrix and NumPy contractions, so agreement is to rounding only.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import schemes
from oracle.norms import rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _plan(p, **kw):
    g_param = p.g_params.get("kappa", 0.0) if p.g == "cubic_nls" else 0.0
    return px.Plan(p.A, p.tau, p.scheme, p.g, g_param=g_param, **kw)


def _gpu_run(p, steps, use_graph=False, phis=None):
    plan = _plan(p)
    if phis is not None:
        for mu, per in enumerate(phis):
            for ell in range(1 if p.scheme in ("exp_euler", "etd2rk") else 0, len(per)):
                plan.set_phi(mu, ell, per[ell])
    U = px.tensor_to_device(p.u0)
    if use_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.run(U, steps, use_graph=True, stream=s)
        torch.cuda.current_stream().wait_stream(s)
    else:
        plan.run(U, steps)
    torch.cuda.synchronize()
    out = px.tensor_from_device(U)
    plan.close()
    return out


def test_allen_cahn_2d_full():
    """2-D Allen-Cahn 64^2, exponential Euler, 50 steps: the whole workload."""
    p = W.allen_cahn_2d()
    got = _gpu_run(p, p.steps, use_graph=True)
    ref = schemes.run_problem(p)
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("scheme", ["lawson_euler", "lawson2b", "exp_euler", "etd2rk"])
@pytest.mark.parametrize("n", [(9,), (23, 31), (17, 12, 9)])
def test_dense_operators_all_schemes(scheme, n):
    """Dense random A_mu: K u runs as mu-mode products (the non-stencil path)."""
    p = W.random_dense_problem(n, seed=len(n) + 5, tau=0.05, scheme=scheme, g="u2_1mu")
    got = _gpu_run(p, 6)
    ref = schemes.run_problem(p, steps=6)
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("scheme", ["lawson_euler", "lawson2b", "exp_euler", "etd2rk"])
def test_adr_stencil_ragged_all_schemes(scheme):
    """Tridiagonal A_mu (stencil K u), ragged sizes spanning several tiles."""
    p = W.adr_3d(n=(40, 41, 42), scheme=scheme)
    got = _gpu_run(p, 12)
    ref = schemes.run_problem(p, steps=12)
    assert rel_inf(got, ref) <= TOL


def test_adr_3d_full_size_graph():
    """3-D ADR 128^3, ETD2RK, in the graph-replay configuration the benchmark times;
    10 steps compared element by element."""
    p = W.adr_3d(n=128)
    got = _gpu_run(p, 10, use_graph=True)
    ref = schemes.run_problem(p, steps=10)
    assert rel_inf(got, ref) <= TOL


def test_graph_equals_direct_bitwise():
    p = W.adr_3d(n=(33, 34, 35))
    a = _gpu_run(p, 7, use_graph=True)
    b = _gpu_run(p, 7, use_graph=False)
    assert np.array_equal(a, b)


def test_injected_oracle_phi():
    """With the oracle's phi matrices injected, only contraction/stepping rounding remains."""
    p = W.adr_3d(n=(24, 20, 28))
    integ = schemes.integrator_for(p)
    got = _gpu_run(p, 8, phis=integ.phis)
    ref = integ.run(p.u0, 0.0, 8)
    assert rel_inf(got, ref) <= 1e-13


@pytest.mark.parametrize("n", [(1, 5, 7), (6, 1, 1), (1, 1, 1)])
def test_degenerate_directions(n):
    p = W.random_dense_problem(n, seed=3, tau=0.1, scheme="etd2rk")
    got = _gpu_run(p, 3)
    ref = schemes.run_problem(p, steps=3)
    assert rel_inf(got, ref) <= TOL


def test_nls_complex_lawson_and_mass_identity():
    """Cubic NLS (complex128, periodic stencil not used by Lawson): state parity and the
    per-step mass identity sum|U_{n+1}|^2 = sum|U_n|^2 (1 + tau^2 |U_n|^4)."""
    p = W.nls_3d(n=24)
    plan = _plan(p)
    U = px.tensor_to_device(p.u0)
    prev = p.u0
    for k in range(5):
        plan.step(U)
        torch.cuda.synchronize()
        cur = px.tensor_from_device(U)
        lhs = np.sum(np.abs(cur) ** 2)
        rhs = np.sum(np.abs(prev) ** 2 * (1 + p.tau ** 2 * np.abs(prev) ** 4))
        assert abs(lhs - rhs) <= 1e-13 * rhs
        prev = cur
    ref = schemes.run_problem(p, steps=5)
    assert rel_inf(prev, ref) <= TOL


def test_nls_complex_exp_euler_periodic_stencil():
    """Complex periodic tridiagonal A_mu through the stencil path (exponential Euler)."""
    p = W.nls_3d(n=(20, 16, 12))
    p.scheme = "exp_euler"
    got = _gpu_run(p, 4)
    ref = schemes.run_problem(p, steps=4)
    assert rel_inf(got, ref) <= TOL


def test_zero_steps_is_identity():
    p = W.allen_cahn_2d(n=16)
    got = _gpu_run(p, 0)
    assert np.array_equal(got, p.u0)


@pytest.mark.parametrize("n", [(1, 5, 7), (6, 1, 1), (1, 1, 1), (70, 3, 2), (2, 40, 3)])
def test_stencil_degenerate_shapes(n):
    """Tridiagonal operators with size-1/2/3 directions through the stencil stage."""
    p = W.adr_3d(n=n)
    got = _gpu_run(p, 4)
    ref = schemes.run_problem(p, steps=4)
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("n", [(3, 4, 5), (5, 3, 2), (33, 17, 20)])
def test_stencil_periodic_small(n):
    """Periodic 3-point operators (corner entries) including n = 3 directions."""
    p = W.nls_3d(n=n)
    p.scheme = "etd2rk"
    got = _gpu_run(p, 3)
    ref = schemes.run_problem(p, steps=3)
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk"])
def test_stencil_variable_coefficients(scheme):
    """Tridiagonal but not Toeplitz (diagonals vary along the direction): coefficients
    are read from the device arrays instead of kernel arguments."""
    p = W.adr_3d(n=(20, 21, 22), scheme=scheme)
    rng = np.random.default_rng(44)
    for mu in range(3):
        n = p.A[mu].shape[0]
        p.A[mu] = p.A[mu] + np.diag(rng.uniform(-5, 5, n)) + np.diag(rng.uniform(-2, 2, n - 1), 1)
    got = _gpu_run(p, 5)
    ref = schemes.run_problem(p, steps=5)
    assert rel_inf(got, ref) <= TOL
