"""Checkpoint and resume: a run's state is (U_n, t_n, plan parameters), and every
kernel is deterministic (no atomics, no split-K; fixed launch configurations), so
n steps in one go equal k steps, a copy of the state to host memory, a new plan
and n - k more steps from that copy, bitwise.  Autonomous nonlinearities here; a
time-dependent source resumes at t_k = k tau, which the device clock forms as
t_0 + j tau (same value to rounding, covered by the paper-ADR tests)."""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W

pytestmark = pytest.mark.gpu


def _plan(p):
    g_param = p.g_params.get("kappa", 0.0) if p.g == "cubic_nls" else 0.0
    return px.Plan(p.A, p.tau, p.scheme, p.g, g_param=g_param)


def _steps(p, u0, steps, use_graph):
    plan = _plan(p)
    U = px.tensor_to_device(u0)
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


@pytest.mark.parametrize("make,graph", [(lambda: W.adr_3d(n=(33, 34, 35)), False),
                                        (lambda: W.adr_3d(n=(64, 16, 40)), True),
                                        (lambda: W.nls_3d(n=(20, 16, 12)), False),
                                        (lambda: W.allen_cahn_2d(n=32), False)])
def test_resume_from_host_copy_is_bitwise(make, graph):
    p = make()
    print("resume", p.name, p.n, flush=True)
    full = _steps(p, p.u0, 6, graph)
    half = _steps(p, p.u0, 3, graph)
    resumed = _steps(p, np.array(half, copy=True), 3, graph)
    assert np.array_equal(full, resumed)


def test_batched_riccati_resume_is_bitwise():
    insts = W.riccati_batch(count=6, nmin=20, nmax=140, seed=51)
    rng = np.random.default_rng(52)
    for x in insts:
        x.U0 = 0.2 * rng.standard_normal((x.n1, x.n2))

    def run(states, steps):
        batch = px.RiccatiBatch(insts, 1e-3)
        U = batch.state_to_device(states)
        batch.run(U, steps)
        torch.cuda.synchronize()
        out = batch.state_from_device(U)
        batch.close()
        return out

    full = run([x.U0 for x in insts], 6)
    half = run([x.U0 for x in insts], 3)
    resumed = run(half, 3)
    for a, b in zip(full, resumed):
        assert np.array_equal(a, b)
