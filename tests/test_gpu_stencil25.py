"""The 2.5-D stage stencil (three directions, real data, n1 a multiple of 64 and
n2 of 8): a workgroup streams along i3 with its planes in registers and LDS.

It sums each element's terms in the same order as the one-element-per-thread
and vectorised kernels, so a plan's steps are bitwise equal with it forced on
(EXPINT_STENCIL25=1) and off (=0); the shapes cover several tiles, runs of planes
that end inside the tensor (n3 not a multiple of 32), Dirichlet and periodic
directions and a direction-dependent (non-Toeplitz) operator.  The paper's
time-dependent source agrees to rounding.  The forced runs are also checked
against the oracle."""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import schemes
from oracle.norms import rel_inf

pytestmark = pytest.mark.gpu


def _run(p, steps, monkeypatch, flag, **kw):
    monkeypatch.setenv("EXPINT_STENCIL25", flag)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, **kw)
    U = px.tensor_to_device(p.u0)
    plan.run(U, steps, t0=0.0)
    torch.cuda.synchronize()
    out = px.tensor_from_device(U)
    plan.close()
    return out


def _periodic_problem(n, seed=12):
    rng = np.random.default_rng(seed)
    A = [0.01 * W.problems.periodic_d2(m, 2 * np.pi / m) for m in n]
    u0 = rng.uniform(0, 1, size=n)
    return W.problems.Problem("periodic_dr", tuple(n), A, 1e-3, 3, "etd2rk", "u2_1mu", u0, seed=seed)


def _row_scaled_problem(n, seed=13):
    """Tridiagonal but not Toeplitz: a different diagonal in every row."""
    rng = np.random.default_rng(seed)
    A = []
    for m in n:
        D = W.problems.dirichlet_d2(m, 1.0 / (m + 1))
        D[np.arange(m), np.arange(m)] *= 1.0 + 0.1 * rng.uniform(size=m)
        A.append(0.01 * D)
    u0 = rng.uniform(0, 1, size=n)
    return W.problems.Problem("rowscaled_dr", tuple(n), A, 1e-3, 3, "etd2rk", "u2_1mu", u0, seed=seed)


@pytest.mark.parametrize("n", [(64, 16, 37), (128, 24, 50), (64, 8, 1), (192, 8, 70)])
def test_dirichlet_bitwise_and_oracle(n, monkeypatch):
    p = W.adr_3d(n=n)
    print("stencil25 adr", n, flush=True)
    on = _run(p, 3, monkeypatch, "1")
    off = _run(p, 3, monkeypatch, "0")
    assert np.array_equal(on, off)
    assert rel_inf(on, schemes.run_problem(p, steps=3)) <= 1e-12


@pytest.mark.parametrize("make", [_periodic_problem, _row_scaled_problem])
def test_periodic_and_row_dependent_bitwise(make, monkeypatch):
    p = make((128, 16, 45))
    print("stencil25", p.name, flush=True)
    on = _run(p, 3, monkeypatch, "1")
    off = _run(p, 3, monkeypatch, "0")
    assert np.array_equal(on, off)
    assert rel_inf(on, schemes.run_problem(p, steps=3)) <= 1e-12


def test_paper_source(monkeypatch):
    """The paper's manufactured source: its polynomial in the grid coordinates is
    contracted into FMAs by the compiler per kernel, so the two kernels agree to
    rounding (not bitwise); both stay on the manufactured solution."""
    p = W.adr_paper((64, 16, 40), steps=4)
    print("stencil25 adr_paper", flush=True)
    kw = dict(g_param=p.g_params["eps"], g_param2=p.g_params["alpha"])
    on = _run(p, 4, monkeypatch, "1", **kw)
    off = _run(p, 4, monkeypatch, "0", **kw)
    assert rel_inf(on, off) <= 1e-14
    assert rel_inf(on, schemes.run_problem(p, steps=4)) <= 1e-12
