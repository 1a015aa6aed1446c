"""GPU parity of the fused launch of modes 1 and 2 (k_modes12) against the oracle.

For FP64 real data with n2 <= 128 a Tucker operator runs modes 1 and 2 as one
launch that keeps M1(rows, :) V_b in LDS (eq. tuckerexp for the slabs V_b of
modes 1 and 2).  Bar: relative max-norm error <= 1e-13 against the oracle's
float64 Tucker operator, as for the single-mode kernel; against the unfused
launches (EXPINT_FUSE12=0), which sum in the same order, <= 1e-15.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle.norms import rel_inf
from oracle.tensor import tucker

pytestmark = pytest.mark.gpu

TOL = 1e-13

# ragged row blocks (n1 mod 32) and column counts on both sides of 64, one-element
# slabs, d = 2 (the fused launch carries the final epilogue), d = 4, and the
# largest n1 and n2 the fused kernel takes
SHAPES = [(1, 1), (1, 1, 1), (5, 3), (31, 33), (64, 64), (33, 65, 2), (37, 70, 5), (40, 41, 42),
          (128, 128, 4), (200, 128, 3), (7, 100, 1, 3), (3, 4, 5, 6), (4096, 128), (4096, 3, 2)]


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, size=shape)


def _apply(n, seed, monkeypatch, fuse, alpha=1.0, beta=0.0):
    monkeypatch.setenv("EXPINT_FUSE12", "1" if fuse else "0")
    V = _rand(n, seed)
    Ms = [_rand((k, k), seed + 1 + mu) / np.sqrt(k) for mu, k in enumerate(n)]
    W0 = _rand(n, seed + 99)
    Vd = px.tensor_to_device(V)
    Wd = px.tensor_to_device(W0)
    px.tucker_apply([px.matrix_to_device(M) for M in Ms], Vd, Wd, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    return px.tensor_from_device(Wd), alpha * tucker(V, Ms) + beta * W0


@pytest.mark.parametrize("n", SHAPES)
def test_fused_matches_oracle(n, monkeypatch):
    got, ref = _apply(n, sum(n), monkeypatch, fuse=True)
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("n", SHAPES)
def test_fused_matches_unfused(n, monkeypatch):
    a, _ = _apply(n, 7 + sum(n), monkeypatch, fuse=True)
    b, _ = _apply(n, 7 + sum(n), monkeypatch, fuse=False)
    assert rel_inf(a, b) <= 1e-15


@pytest.mark.parametrize("n", [(37, 70), (40, 41, 42)])
def test_fused_with_alpha_beta(n, monkeypatch):
    got, ref = _apply(n, 3 + sum(n), monkeypatch, fuse=True, alpha=-0.75, beta=2.5)
    assert rel_inf(got, ref) <= TOL


def test_identity_mode_keeps_the_chain_unfused(monkeypatch):
    """M_2 = None: modes 1 and 3 only, through the single-mode kernel."""
    monkeypatch.setenv("EXPINT_FUSE12", "1")
    n = (37, 20, 11)
    V = _rand(n, 5)
    Ms = [_rand((k, k), 6 + mu) for mu, k in enumerate(n)]
    Vd = px.tensor_to_device(V)
    Wd = torch.empty_like(Vd)
    px.tucker_apply([px.matrix_to_device(Ms[0]), None, px.matrix_to_device(Ms[2])], Vd, Wd)
    torch.cuda.synchronize()
    ref = tucker(V, [Ms[0], np.eye(20), Ms[2]])
    assert rel_inf(px.tensor_from_device(Wd), ref) <= TOL


@pytest.mark.parametrize("scheme", ["etd2rk", "exp_euler", "lawson_euler", "lawson2b"])
@pytest.mark.parametrize("d", [2, 3])
def test_plan_steps_fused_equal_unfused(scheme, d, monkeypatch):
    """Whole steps of every scheme, 2-D (ETD2RK's first stage writes W_2 over its own
    input, so that launch stays unfused) and 3-D, with and without the fused launch."""
    out = []
    for fuse in ("1", "0"):
        monkeypatch.setenv("EXPINT_FUSE12", fuse)
        p = W.allen_cahn_2d(n=80) if d == 2 else W.adr_3d(n=(24, 20, 28))
        plan = px.Plan(p.A, p.tau, scheme, p.g)
        assert not plan.fused
        U = px.tensor_to_device(p.u0)
        plan.run(U, 4)
        torch.cuda.synchronize()
        out.append(px.tensor_from_device(U))
        plan.close()
    assert rel_inf(out[0], out[1]) <= 1e-14


@pytest.mark.parametrize("shape", ["r32w4", "r32w8", "r16w4", "r64w8", "r64w16", "r32w8p", "r32w8i", "r64w16p", "r64w16i"])
@pytest.mark.parametrize("n", [(5, 3), (37, 70, 5), (40, 41, 42), (200, 128, 3), (4096, 3, 2)])
def test_every_workgroup_shape(shape, n, monkeypatch):
    """Each workgroup shape of the fused launch (forced through EXPINT_M12)."""
    monkeypatch.setenv("EXPINT_M12", shape)
    got, ref = _apply(n, 11 + sum(n), monkeypatch, fuse=True)
    assert rel_inf(got, ref) <= TOL
