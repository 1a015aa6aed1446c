"""Whole-state parity at the benchmark workloads' full sizes.

The GPU steps each workload at its full size, in the configuration bench.py
times (graph replay), and the whole final state is compared with the oracle's
(relative max-norm, section 4.2's error measure).  The oracle's step counts
are bounded so that it finishes in about a minute on the host:

* 384^3 diffusion-reaction, ETD2RK, tau = 2e-3: 5 steps (of the workload's 20)
  in FP64 (<= 1e-12), FP32 (<= 1e-5), bf16x3 (<= 1e-4) and exact slice
  (<= 1e-10), all against one FP64 oracle run; the 20-step runs of the reduced
  precisions are compared with the 20-step FP64 run;
* 192^3 cubic NLS, Lawson-Euler, tau = 1e-3: 20 steps (of 200) in complex128
  (<= 1e-12) and complex64 (<= 1e-4), and the mass identity of every step;
* the 64 Riccati-type instances (n1, n2 in 32..512): every instance, 5 ETD2RK
  steps and 2 Rosenbrock-Euler steps (<= 1e-12).
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import nonlinear, schemes
from oracle.norms import rel_inf

pytestmark = pytest.mark.gpu

DR_STEPS = 5
BOUND = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4, "slice": 1e-10}


def _run_graph(plan, U, steps):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(U, steps, use_graph=True, stream=s)
    s.synchronize()
    return U


@pytest.fixture(scope="module")
def dr384():
    p = W.diffusion_reaction_3d(n=384)
    print(f"oracle: 384^3 diffusion-reaction, {DR_STEPS} ETD2RK steps", flush=True)
    ref = schemes.run_problem(p, steps=DR_STEPS)
    return p, ref


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "slice"])
def test_dr384_whole_state(dr384, precision):
    p, ref = dr384
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=precision)
    U = _run_graph(plan, px.tensor_to_device(p.u0), DR_STEPS)
    got = px.tensor_from_device(U)
    err = rel_inf(got, ref)
    print(f"384^3 {precision}: rel-inf vs oracle after {DR_STEPS} steps = {err:.3e}", flush=True)
    assert err <= BOUND[precision]
    if precision != "fp64":
        assert err > 1e-16  # the reduced contraction really ran
    plan.close()


def test_dr384_twenty_steps_reduced_vs_fp64():
    p = W.diffusion_reaction_3d(n=384)
    U0 = px.tensor_to_device(p.u0)
    out = {}
    for prec in ("fp64", "fp32", "bf16x3", "slice"):
        plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=prec)
        out[prec] = _run_graph(plan, U0.clone(), p.steps)
        assert plan.check_finite(out[prec])
        plan.close()
    ref = out["fp64"]
    scale = ref.abs().max().item()
    for prec in ("fp32", "bf16x3", "slice"):
        err = (out[prec] - ref).abs().max().item() / scale
        print(f"384^3 {prec}: rel-inf vs FP64 after {p.steps} steps = {err:.3e}", flush=True)
        assert err <= BOUND[prec]


NLS_STEPS = 20


@pytest.fixture(scope="module")
def nls192():
    p = W.nls_3d(n=192)
    ref = schemes.run_problem(p, steps=NLS_STEPS)
    return p, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_nls192_whole_state(nls192, precision, tol):
    p, ref = nls192
    kappa = p.g_params.get("kappa", 0.0)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, g_param=kappa, precision=precision)
    U = _run_graph(plan, px.tensor_to_device(p.u0), NLS_STEPS)
    err = rel_inf(px.tensor_from_device(U), ref)
    print(f"192^3 NLS {precision}: rel-inf vs oracle after {NLS_STEPS} steps = {err:.3e}", flush=True)
    assert err <= tol
    plan.close()


def test_nls192_mass_identity_every_step():
    """Lawson-Euler with the unitary e^{tau A_mu}: sum |U_{n+1}|^2 = sum |U_n|^2 (1 + tau^2 kappa^2 |U_n|^4)
    at every step, to complex128 rounding."""
    p = W.nls_3d(n=192)
    kappa = p.g_params.get("kappa", 1.0)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, g_param=kappa)
    U = px.tensor_to_device(p.u0)
    for _ in range(NLS_STEPS):
        prev = U.clone()
        plan.step(U)
        torch.cuda.synchronize()
        a2 = prev.abs() ** 2
        lhs = (U.abs() ** 2).sum().item()
        rhs = (a2 * (1 + (p.tau * kappa) ** 2 * a2 * a2)).sum().item()
        assert abs(lhs - rhs) <= 1e-12 * rhs
    plan.close()


def _riccati_oracle_etd2rk(x, tau, steps):
    g = nonlinear.make_g("riccati", {"B": x.B, "C": x.C})
    return schemes.Integrator([x.A1, x.A2], tau, "etd2rk", g).run(x.U0, 0.0, steps)


@pytest.mark.parametrize("scheme,steps", [("etd2rk", 5), ("rosenbrock_euler", 2)])
def test_riccati64_every_instance(scheme, steps):
    insts = W.riccati_batch()
    tau = 1e-3
    batch = px.RiccatiBatch(insts, tau, scheme=scheme)
    U = batch.state_to_device([x.U0 for x in insts])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(U, steps, use_graph=True, stream=s)
    s.synchronize()
    assert batch.status(U) == px._binding.OK
    got = batch.state_from_device(U)
    batch.close()
    print(f"oracle: 64 Riccati instances, {steps} {scheme} steps", flush=True)
    worst = 0.0
    for i, x in enumerate(insts):
        if scheme == "etd2rk":
            ref = _riccati_oracle_etd2rk(x, tau, steps)
        else:
            ref = schemes.run_rosenbrock_euler_riccati(x.U0, tau, steps, x.A1, x.A2, x.B, x.C)
        err = rel_inf(got[i], ref)
        worst = max(worst, err)
        assert err <= 1e-12, (i, x.n1, x.n2, err)
    print(f"64 Riccati instances {scheme}: worst rel-inf = {worst:.3e}", flush=True)
