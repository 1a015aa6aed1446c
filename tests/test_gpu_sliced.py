"""Exact-slice contraction (EXPINT_PREC_SLICED) against the FP64 oracle.

Every operand fibre is cut into five balanced base-254 int8 digits under a
power-of-two exponent 2^E <= 4 max|x|, and the digit products a_i b_j with
i + j <= 5 are summed exactly on int8 MFMA.  For one contraction
y = sum_k a_k b_k the library states the bound
    |y_hat - y| <= 2^-38.9 (max|b| sum|a| + max|a| sum|b|) + K 2^-44.3 max|a| max|b|
plus FP64 rounding of the combination; the single-mode tests check it element
by element against the oracle's mu-mode product (a wrong digit weight, level
or exponent breaks it by many orders of magnitude).  Tucker chains and whole
integrator steps are held to the stated target: rel-inf <= 1e-10 against the
FP64 oracle.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import schemes
from oracle.norms import rel_inf
from oracle.tensor import mode_product, tucker

pytestmark = pytest.mark.gpu


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, size=shape)


def _bound(V, M, mu):
    """Per-element bound of the sliced mode-mu product V x_mu M."""
    K = M.shape[1]
    aM = np.abs(M)
    aV = np.abs(V)
    maxa = aM.max(axis=1)                  # per output index i_mu
    suma = aM.sum(axis=1)
    maxb = aV.max(axis=mu, keepdims=True)  # per fibre
    sumb = aV.sum(axis=mu, keepdims=True)
    shape = [1] * V.ndim
    shape[mu] = -1
    maxa = maxa.reshape(shape)
    suma = suma.reshape(shape)
    dot = mode_product(aV, aM, mu + 1)     # sum_k |a_k| |b_k|
    return (2.0 ** -38.9 * (maxb * suma + maxa * sumb) + K * 2.0 ** -44.3 * maxa * maxb
            + 8 * np.finfo(float).eps * dot)


def _sliced_tucker(Ms, V, alpha=1.0, beta=0.0, W0=None):
    Vd = px.tensor_to_device(V)
    Wd = px.tensor_to_device(W0) if W0 is not None else torch.zeros_like(Vd)
    px.tucker_apply([None if M is None else px.matrix_to_device(M) for M in Ms], Vd, Wd, alpha=alpha, beta=beta,
                    precision="slice")
    torch.cuda.synchronize()
    return px.tensor_from_device(Wd)


@pytest.mark.parametrize("n,mu", [((70, 45), 0), ((70, 45), 1), ((37, 64, 129), 0), ((37, 64, 129), 1),
                                  ((37, 64, 129), 2), ((1, 5, 7), 1), ((65, 3, 2), 0), ((6, 200, 9), 1)])
def test_single_mode_within_stated_bound(n, mu):
    rng = np.random.default_rng(11)
    # fibres of very different size: per-fibre exponents must keep each one's digits
    V = rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 6, size=n)
    M = rng.standard_normal((n[mu], n[mu])) * 10.0 ** rng.uniform(-3, 3, size=(n[mu], 1))
    Ms = [M if i == mu else None for i in range(len(n))]
    got = _sliced_tucker(Ms, V)
    ref = mode_product(V, M, mu + 1)
    ratio = float((np.abs(got - ref) / _bound(V, M, mu)).max())
    assert ratio <= 1.0, ratio
    # and the error is far below what FP32 or BF16 operands would give
    err = rel_inf(got, ref)
    assert err < 1e-10, err


@pytest.mark.parametrize("n", [(7,), (33, 65), (40, 41, 42), (128, 128, 128), (17, 1, 70), (3, 4, 5, 6)])
def test_tucker_chain_random(n):
    V = _rand(n, 1)
    Ms = [_rand((k, k), 2 + i) / np.sqrt(k) for i, k in enumerate(n)]
    got = _sliced_tucker(Ms, V)
    err = rel_inf(got, tucker(V, Ms))
    assert err <= 1e-10, err


def test_tucker_alpha_beta_and_skipped_mode():
    n = (33, 20, 70)
    V = _rand(n, 3)
    W0 = _rand(n, 4)
    Ms = [_rand((n[0], n[0]), 5), None, _rand((n[2], n[2]), 6)]
    got = _sliced_tucker(Ms, V, alpha=-0.75, beta=0.5, W0=W0)
    ref = -0.75 * tucker(V, [Ms[0], np.eye(n[1]), Ms[2]]) + 0.5 * W0
    err = rel_inf(got, ref)
    assert err <= 1e-10, err


def test_phi_matrices_of_the_workloads():
    """The contraction the integrators run: phi_1(tau A_mu) of the ADR operators."""
    p = W.adr_3d(n=128)
    Ms = [px.phi_setup(a, p.tau, 1)[1] for a in p.A]
    V = p.u0
    got = _sliced_tucker(Ms, V)
    # stated bound with sum|phi row| ~ 1: a few 2^-38.9 per mode
    err = rel_inf(got, tucker(V, Ms))
    assert err <= 1e-11, err


def test_zero_and_nonfinite_inputs():
    n = (20, 30, 40)
    Ms = [_rand((k, k), 7 + i) + 2.0 for i, k in enumerate(n)]  # no zero entries
    assert np.all(_sliced_tucker(Ms, np.zeros(n)) == 0.0)
    # a nan or inf reaches exactly the outputs whose fibre holds it (mode 1 only)
    V = _rand(n, 8)
    V[3, 4, 5] = np.nan
    V[7, 9, 11] = np.inf
    got = _sliced_tucker([Ms[0], None, None], V)
    ref = mode_product(V, Ms[0], 1)
    bad = ~np.isfinite(ref)
    assert bad.sum() == 2 * n[0]
    assert np.array_equal(~np.isfinite(got), bad)
    err = rel_inf(got[~bad], ref[~bad])
    assert err <= 1e-11, err


@pytest.mark.parametrize("scheme", ["etd2rk", "exp_euler", "lawson_euler", "lawson2b"])
def test_schemes_match_oracle(scheme):
    p = W.random_dense_problem((24, 20, 28), seed=3, tau=0.05, steps=6, scheme=scheme)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision="slice")
    U = px.tensor_to_device(p.u0)
    plan.run(U, p.steps)
    torch.cuda.synchronize()
    got = px.tensor_from_device(U)
    plan.close()
    err = rel_inf(got, schemes.run_problem(p))
    assert err <= 1e-10, err


def test_stencil_path_and_paper_adr():
    """Tridiagonal operators (stencil K u) and the time-dependent source."""
    p = W.adr_paper((40, 41, 42), steps=12, scheme="etd2rk")
    plan = px.Plan(p.A, p.tau, p.scheme, "adr_paper", g_param=p.g_params["eps"], g_param2=p.g_params["alpha"],
                   precision="slice")
    U = px.tensor_to_device(p.u0)
    plan.run(U, p.steps, t0=0.0)
    torch.cuda.synchronize()
    got = px.tensor_from_device(U)
    plan.close()
    err = rel_inf(got, schemes.run_problem(p))
    assert err <= 1e-10, err


def test_diffusion_reaction_384_against_fp64_path():
    """The 384^3 precision-sweep workload, 20 ETD2RK steps in the benchmark's
    launch configuration (graph replay), against the FP64 path (itself
    oracle-checked at this size on sampled entries elsewhere)."""
    p = W.diffusion_reaction_3d(n=384)
    out = {}
    for prec in ("fp64", "slice"):
        plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=prec)
        U = px.tensor_to_device(p.u0)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.run(U, 20, use_graph=True, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        out[prec] = U
        plan.close()
    d = (out["slice"] - out["fp64"]).abs().max().item() / out["fp64"].abs().max().item()
    assert d <= 1e-10, d


def test_set_phi_reslices():
    """Injected phi matrices reach the digit copies the sliced chain reads."""
    p = W.random_dense_problem((12, 10, 14), seed=4, tau=0.05)
    plan = px.Plan(p.A, p.tau, "lawson_euler", "none", precision="slice")
    E = [np.eye(k) * 0.5 for k in p.n]
    for mu in range(3):
        plan.set_phi(mu, 0, E[mu])
    U = px.tensor_to_device(p.u0)
    plan.step(U)
    torch.cuda.synchronize()
    got = px.tensor_from_device(U)
    plan.close()
    # digits of U carry <= 2^-38.9 relative truncation per mode; the original e^{tau A} would be off by O(tau)
    err = rel_inf(got, p.u0 * 0.125)
    assert err <= 1e-11, err


SLICE_TILES = ["64x64w4k64s2o2", "128x64w8k64s2o1", "64x128w8k64s2o1", "64x64w4k32s2o3", "64x64w4k32s4o2",
               "128x64w8k32s4o1"]


@pytest.mark.parametrize("tile", SLICE_TILES)
def test_every_tile_shape(tile, monkeypatch):
    """Each tile shape of the int8 product (forced through EXPINT_SLICE_TILE) on ragged
    sizes: K of one, two and several chunks with a tail, rows and columns past the tile."""
    monkeypatch.setenv("EXPINT_SLICE_TILE", tile)
    rng = np.random.default_rng(21)
    for n, mu in (((37, 70, 133), 0), ((37, 70, 133), 1), ((37, 70, 133), 2), ((200, 3, 5), 0)):
        V = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, size=n)
        M = rng.standard_normal((n[mu], n[mu]))
        Ms = [M if i == mu else None for i in range(len(n))]
        got = _sliced_tucker(Ms, V)
        ref = mode_product(V, M, mu + 1)
        ratio = float((np.abs(got - ref) / _bound(V, M, mu)).max())
        assert ratio <= 1.0, (tile, n, mu, ratio)
