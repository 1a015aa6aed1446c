"""Batched exponential Rosenbrock-Euler phisplit on the GPU against the oracle.

Every instance of U' = A1 U + U A2^T + C + U B U is stepped with
eq. expRosEulertensor: the device rebuilds phi_1 of the Jacobian directions
tau J1 = tau (A1 + U B) and tau J2^T = tau (A2^T + B U) at every step (scaling
and squaring of a degree-13 Taylor series) and applies one Tucker operator.
The oracle builds the same phi_1 with an augmented-matrix exponential, so the
two agree to the rounding of two different phi builders.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle.norms import rel_inf
from oracle.schemes import run_rosenbrock_euler_riccati

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _with_random_start(insts, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    for x in insts:
        x.U0 = scale * rng.standard_normal((x.n1, x.n2))
    return insts


def _oracle(x, tau, steps):
    return run_rosenbrock_euler_riccati(x.U0, tau, steps, x.A1, x.A2, x.B, x.C)


def _gpu(insts, tau, steps, use_graph=False):
    batch = px.RiccatiBatch(insts, tau, scheme="rosenbrock_euler")
    U = batch.state_to_device([x.U0 for x in insts])
    if use_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batch.run(U, steps, use_graph=True, stream=s)
        torch.cuda.current_stream().wait_stream(s)
    else:
        batch.run(U, steps)
    torch.cuda.synchronize()
    out = batch.state_from_device(U)
    batch.close()
    return out


def test_small_uneven_batch():
    insts = _with_random_start(W.riccati_batch(count=7, nmin=5, nmax=70, seed=41), 42)
    tau = 1e-3
    got = _gpu(insts, tau, 6)
    for x, u in zip(insts, got):
        err = rel_inf(u, _oracle(x, tau, 6))
        assert err <= TOL, (x.n1, x.n2, err)


def test_tiny_and_non_square_instances():
    insts = _with_random_start(W.riccati_batch(count=5, nmin=1, nmax=9, seed=43), 44)
    tau = 2e-3
    got = _gpu(insts, tau, 4)
    for x, u in zip(insts, got):
        err = rel_inf(u, _oracle(x, tau, 4))
        assert err <= TOL, (x.n1, x.n2, err)


def test_graph_replay_equals_direct():
    insts = _with_random_start(W.riccati_batch(count=5, nmin=20, nmax=90, seed=45), 46)
    a = _gpu(insts, 1e-3, 5, use_graph=False)
    b = _gpu(insts, 1e-3, 5, use_graph=True)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_full_batch_sampled_instances():
    """The 64-instance workload (sizes 32..512, stiff directions needing up to a
    dozen squarings): three steps, every eighth instance against the oracle."""
    insts = _with_random_start(W.riccati_batch(), 47, scale=0.1)
    tau = 1e-3
    got = _gpu(insts, tau, 3)
    for k in range(0, len(insts), 8):
        err = rel_inf(got[k], _oracle(insts[k], tau, 3))
        assert err <= TOL, (k, insts[k].n1, insts[k].n2, err)


def test_scheme_difference_matches_the_oracle():
    """The GPU Rosenbrock-Euler and ETD2RK results differ by the same amount as the
    oracle's two schemes (the plan really runs the scheme it was asked for)."""
    from oracle import nonlinear, schemes
    insts = _with_random_start(W.riccati_batch(count=3, nmin=20, nmax=40, seed=48), 49)
    tau = 1e-3
    ros = _gpu(insts, tau, 5)
    batch = px.RiccatiBatch(insts, tau)
    U = batch.state_to_device([x.U0 for x in insts])
    batch.run(U, 5)
    torch.cuda.synchronize()
    etd = batch.state_from_device(U)
    batch.close()
    for x, a, b in zip(insts, ros, etd):
        g = nonlinear.make_g("riccati", {"B": x.B, "C": x.C})
        ref_etd = schemes.Integrator([x.A1, x.A2], tau, "etd2rk", g).run(x.U0, 0.0, 5)
        ref_ros = _oracle(x, tau, 5)
        d_gpu, d_ref = a - b, ref_ros - ref_etd
        assert np.abs(d_ref).max() > 1e-6
        assert np.abs(d_gpu - d_ref).max() <= 1e-8 * np.abs(d_ref).max()
