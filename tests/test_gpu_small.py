"""Fused small two-dimensional path: a whole run in one workgroup.

Plans with d = 2, n1, n2 <= 64, real FP64 data and FP64 contraction run all
steps in one launch with the state in LDS.  Each case is checked against the
oracle and against the general kernel sequence of the same plan
(EXPINT_SMALL_FUSED=0), for every scheme, with stencil (Dirichlet and
periodic) and dense operators, ragged and degenerate shapes.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import schemes
from oracle.norms import rel_inf

pytestmark = pytest.mark.gpu

SCHEMES = ["exp_euler", "etd2rk", "lawson_euler", "lawson2b"]


def _run(p, fused, monkeypatch, use_graph=False, stepwise=False):
    monkeypatch.setenv("EXPINT_SMALL_FUSED", "1" if fused else "0")
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, g_param=p.g_params.get("kappa", 0.0))
    U = px.tensor_to_device(p.u0)
    if stepwise:
        for k in range(p.steps):
            plan.step(U, t=k * p.tau)
    elif use_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.run(U, p.steps, use_graph=True, stream=s)
        torch.cuda.current_stream().wait_stream(s)
    else:
        plan.run(U, p.steps)
    torch.cuda.synchronize()
    out = px.tensor_from_device(U)
    plan.close()
    return out


def _stencil_problem(n, scheme, periodic=False, steps=7):
    rng = np.random.default_rng(21)
    A = [0.05 * (W.periodic_d2(k, 2 * np.pi / k) if periodic else W.dirichlet_d2(k, 1.0 / (k + 1)))
         for k in n]
    u0 = rng.uniform(-0.9, 0.9, size=n)
    return W.Problem("small", tuple(n), A, 1e-3, steps, scheme, "allen_cahn", u0)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("n", [(64, 64), (33, 17), (1, 5), (64, 1), (7, 64)])
def test_fused_stencil_matches_oracle_and_general_path(scheme, n, monkeypatch):
    p = _stencil_problem(n, scheme)
    ref = schemes.run_problem(p)
    fused = _run(p, True, monkeypatch)
    general = _run(p, False, monkeypatch)
    assert rel_inf(fused, ref) <= 1e-12
    assert rel_inf(fused, general) <= 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
def test_fused_periodic(scheme, monkeypatch):
    p = _stencil_problem((48, 40), scheme, periodic=True)
    assert rel_inf(_run(p, True, monkeypatch), schemes.run_problem(p)) <= 1e-12


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("n", [(24, 20), (64, 64)])
def test_fused_dense_operators(scheme, n, monkeypatch):
    p = W.random_dense_problem(n, seed=9, tau=0.05, steps=5, scheme=scheme)
    ref = schemes.run_problem(p)
    assert rel_inf(_run(p, True, monkeypatch), ref) <= 1e-12
    assert rel_inf(_run(p, True, monkeypatch), _run(p, False, monkeypatch)) <= 1e-13


def test_allen_cahn_workload(monkeypatch):
    """The 64^2 Allen-Cahn workload: 50 exponential Euler steps in one launch."""
    p = W.allen_cahn_2d()
    ref = schemes.run_problem(p)
    assert rel_inf(_run(p, True, monkeypatch), ref) <= 1e-12
    assert rel_inf(_run(p, True, monkeypatch, use_graph=True), ref) <= 1e-12


def test_stepwise_equals_run(monkeypatch):
    p = _stencil_problem((40, 30), "etd2rk", steps=5)
    a = _run(p, True, monkeypatch)
    b = _run(p, True, monkeypatch, stepwise=True)
    assert np.array_equal(a, b)


def test_larger_problems_stay_on_general_path(monkeypatch):
    """65 points in a direction exceeds the fused path: the result still matches."""
    p = _stencil_problem((65, 20), "exp_euler", steps=3)
    assert rel_inf(_run(p, True, monkeypatch), schemes.run_problem(p)) <= 1e-12
