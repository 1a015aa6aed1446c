"""Status reporting and per-direction phi replacement on the GPU.

* expint_plan_set_phi on a direction whose bitwise-equal A made other
  directions share its device matrix replaces phi of that direction only, in
  FP64 and in exact-slice precision (the sharers keep their matrix and digits);
* exponential Rosenbrock-Euler flags a Jacobian direction that needs more
  squarings (section 3.1 scaling rule, eq. squarephi) than the plan provides,
  and expint_batch_status reports it once as ENUMERIC;
* the finite checks report inf / nan states as ENONFINITE.
Every kernel here runs to its normal end; the flags are set by the kernels'
own bounded logic.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import nonlinear, schemes
from oracle.norms import rel_inf
from oracle.phi import direction_phis

pytestmark = pytest.mark.gpu


def _equal_a_problem(n=20):
    p = W.diffusion_reaction_3d(n=n)
    assert all(np.array_equal(p.A[0], a) for a in p.A)
    return p


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("slice", 1e-10)])
@pytest.mark.parametrize("mu", [0, 1])
def test_set_phi_on_a_shared_direction_changes_only_that_direction(precision, tol, mu):
    p = _equal_a_problem()
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=precision)
    phis = direction_phis(p.A, p.tau, 2)
    # a different operator for direction mu only (its phi_1 and phi_2)
    Aalt = 1.7 * p.A[mu] + 0.3 * np.diag(np.ones(p.n[mu] - 1), 1)
    alt = direction_phis([Aalt], p.tau, 2)[0]
    plan.set_phi(mu, 1, alt[1])
    plan.set_phi(mu, 2, alt[2])
    U = px.tensor_to_device(p.u0)
    plan.run(U, 2)
    torch.cuda.synchronize()
    mixed = [list(ph) for ph in phis]
    mixed[mu] = list(alt)
    integ = schemes.Integrator(p.A, p.tau, p.scheme, nonlinear.make_g(p.g, p.g_params), phis=mixed)
    ref = integ.run(p.u0, 0.0, 2)
    assert rel_inf(px.tensor_from_device(U), ref) <= tol
    # graph replay after the replacement uses the new matrices too
    U2 = px.tensor_to_device(p.u0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(U2, 2, use_graph=True, stream=s)
    s.synchronize()
    assert torch.equal(U2, U)
    plan.close()


def test_check_finite_reports_and_clears():
    p = _equal_a_problem(12)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g)
    U = px.tensor_to_device(p.u0)
    plan.run(U, 3)
    assert plan.check_finite(U)
    bad = U.clone()
    bad.view(-1)[777] = float("nan")
    assert not plan.check_finite(bad)
    bad.view(-1)[777] = float("inf")
    assert not plan.check_finite(bad)
    assert plan.check_finite(U)  # the flag was cleared by the previous report
    # a run that blows up is seen too: g = u^2 (1 - u) from a large start
    big = px.tensor_to_device(np.full(p.u0.shape, -1e120))
    plan.run(big, 3)
    assert not plan.check_finite(big)
    plan.close()


def _small_batch(seed=11):
    insts = W.riccati_batch(count=3, seed=seed, nmin=16, nmax=40)
    rng = np.random.default_rng(seed)
    for x in insts:
        x.U0 = 0.1 * rng.standard_normal((x.n1, x.n2))
    return insts


def test_rosenbrock_status_ok_on_the_workload_scale():
    insts = _small_batch()
    batch = px.RiccatiBatch(insts, 1e-3, scheme="rosenbrock_euler")
    U = batch.state_to_device([x.U0 for x in insts])
    batch.run(U, 3)
    assert batch.status(U) == px._binding.OK
    batch.close()


def test_rosenbrock_flags_too_few_squarings():
    """A state far larger than the plan's operators makes ||tau (A1 + U B)||_1 need
    more squaring phases than the plan fixed at creation: the step still runs to
    its end, and the status call reports ENUMERIC once."""
    insts = _small_batch()
    batch = px.RiccatiBatch(insts, 1e-3, scheme="rosenbrock_euler")
    U = batch.state_to_device([1e6 * np.sign(x.U0) for x in insts])
    batch.step(U)
    assert batch.status() == px._binding.ENUMERIC
    assert "squarings" in px._binding.lib.expint_last_error().decode()
    assert batch.status() == px._binding.OK  # reported once, then cleared
    batch.close()


def test_batch_status_sees_a_non_finite_state():
    insts = _small_batch()
    batch = px.RiccatiBatch(insts, 1e-3, scheme="etd2rk")
    U = batch.state_to_device([x.U0 for x in insts])
    batch.run(U, 2)
    assert batch.status(U) == px._binding.OK
    U.view(-1)[5] = float("nan")
    assert batch.status(U) == px._binding.ENONFINITE
    U.view(-1)[5] = 0.0
    assert batch.status(U) == px._binding.OK
    batch.close()
