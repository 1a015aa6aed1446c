"""Four-dimensional problems: plans with d = 4 (K = A_4 (+) A_3 (+) A_2 (+) A_1,
the split factor (2!)^{d-1} = 8 on the ETD2RK phi_2 stage) against the oracle,
with dense operators (K u by mu-mode products) and with Dirichlet stencils."""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import schemes
from oracle.norms import rel_inf

pytestmark = pytest.mark.gpu

SCHEMES = ["exp_euler", "etd2rk", "lawson_euler", "lawson2b"]


def _gpu(p, precision="fp64"):
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=precision)
    U = px.tensor_to_device(p.u0)
    plan.run(U, p.steps)
    torch.cuda.synchronize()
    out = px.tensor_from_device(U)
    plan.close()
    return out


@pytest.mark.parametrize("scheme", SCHEMES)
def test_dense_d4(scheme):
    p = W.random_dense_problem((5, 4, 6, 3), seed=17, tau=0.05, steps=4, scheme=scheme)
    assert rel_inf(_gpu(p), schemes.run_problem(p)) <= 1e-12


@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk"])
def test_stencil_d4(scheme):
    n = (9, 7, 8, 6)
    rng = np.random.default_rng(18)
    A = [0.05 * W.dirichlet_d2(k, 1.0 / (k + 1)) for k in n]
    p = W.Problem("d4", n, A, 2e-3, 5, scheme, "u2_1mu", rng.uniform(0, 1, size=n))
    assert rel_inf(_gpu(p), schemes.run_problem(p)) <= 1e-12


def test_d4_exact_slice():
    p = W.random_dense_problem((12, 10, 9, 8), seed=19, tau=0.05, steps=3, scheme="etd2rk")
    assert rel_inf(_gpu(p, "slice"), schemes.run_problem(p)) <= 1e-10
