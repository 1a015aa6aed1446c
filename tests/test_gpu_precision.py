"""Reduced contraction precisions against the FP64 oracle.

The phi matrices and the state stay FP64; only the mu-mode contractions run
in FP32 (operands rounded to FP32, FP32 MFMA) or split BF16 (x = hi + lo,
three BF16 MFMA products, FP32 accumulation).  Stated bounds (relative
max-norm against the FP64 oracle): FP32 <= 1e-5, BF16X3 <= 1e-4 per Tucker
operator and over a few steps.  Rounding model: an FP32 operand carries 2^-24
relative error, a bf16 hi/lo pair 2^-18 (the dropped lo*lo term and lo's own
rounding); K-term FP32 accumulation adds ~sqrt(K) 2^-24.  Each check also
asserts the error is not below a floor, which shows the reduced path ran.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import schemes
from oracle.norms import rel_inf
from oracle.tensor import tucker

pytestmark = pytest.mark.gpu

BOUNDS = {"fp32": (1e-5, 1e-9), "bf16x3": (1e-4, 1e-8)}
PREC = {"fp32": px.PREC_FP32, "bf16x3": px.PREC_BF16X3}


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, size=shape)


# (130, 129, 250) gives every mode 512 or more output tiles of the reduced-precision kernels
# (a large grid next to the small ones)
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n", [(7,), (33, 65), (40, 41, 42), (128, 128, 128), (17, 1, 70), (3, 4, 5, 6),
                               (130, 129, 250)])
def test_tucker_reduced_precision(prec, n):
    V = _rand(n, 1)
    Ms = [_rand((k, k), 2 + i) / np.sqrt(k) for i, k in enumerate(n)]
    Vd = px.tensor_to_device(V)
    Wd = torch.empty_like(Vd)
    px.tucker_apply([px.matrix_to_device(M) for M in Ms], Vd, Wd, precision=PREC[prec])
    torch.cuda.synchronize()
    err = rel_inf(px.tensor_from_device(Wd), tucker(V, Ms))
    hi, lo = BOUNDS[prec]
    assert lo < err <= hi, err


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("mu", [0, 1, 2])
def test_single_mode_reduced_precision(prec, mu):
    n = (37, 70, 29)
    V = _rand(n, 5)
    Ms = [_rand((k, k), 6 + i) for i, k in enumerate(n)]
    Md = [px.matrix_to_device(M) if i == mu else None for i, M in enumerate(Ms)]
    Vd = px.tensor_to_device(V)
    Wd = px.tensor_to_device(_rand(n, 9))
    px.tucker_apply(Md, Vd, Wd, alpha=0.5, beta=0.0, precision=PREC[prec])
    torch.cuda.synchronize()
    ref = 0.5 * tucker(V, [M if i == mu else np.eye(k) for i, (k, M) in enumerate(zip(n, Ms))])
    assert rel_inf(px.tensor_from_device(Wd), ref) <= BOUNDS[prec][0]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("scheme", ["exp_euler", "etd2rk", "lawson_euler", "lawson2b"])
def test_stepping_reduced_precision(prec, scheme):
    p = W.adr_3d(n=(40, 41, 42), scheme=scheme)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=prec)
    U = px.tensor_to_device(p.u0)
    plan.run(U, 10)
    torch.cuda.synchronize()
    err = rel_inf(px.tensor_from_device(U), schemes.run_problem(p, steps=10))
    assert err <= BOUNDS[prec][0], err


def test_complex_bf16x3_rejected():
    p = W.nls_3d(n=8)
    with pytest.raises(px.ExpintError):
        px.Plan(p.A, p.tau, p.scheme, p.g, g_param=1.0, precision="bf16x3")


@pytest.mark.parametrize("n", [(5,), (33, 17), (24, 20, 28), (96, 96, 96)])
def test_tucker_complex64(n):
    """complex128 data contracted in complex64 arithmetic (FP32 MFMA, four real products)."""
    rng = np.random.default_rng(sum(n))
    V = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    Ms = [(rng.uniform(-1, 1, (k, k)) + 1j * rng.uniform(-1, 1, (k, k))) / np.sqrt(k) for k in n]
    Vd = px.tensor_to_device(V)
    Wd = torch.empty_like(Vd)
    px.tucker_apply([px.matrix_to_device(M) for M in Ms], Vd, Wd, precision=px.PREC_FP32)
    torch.cuda.synchronize()
    err = rel_inf(px.tensor_from_device(Wd), tucker(V, Ms))
    assert 1e-9 < err <= 1e-5, err


def test_nls_complex64_lawson_mass():
    """Cubic NLS, Lawson-Euler with complex64 contractions: state within 1e-5 of the
    complex128 oracle after 10 steps; the per-step mass identity (exact for a unitary
    e^{tau A}) holds to single-precision level."""
    p = W.nls_3d(n=32)
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, g_param=1.0, precision="fp32")
    U = px.tensor_to_device(p.u0)
    prev = p.u0
    worst = 0.0
    for k in range(10):
        plan.step(U)
        torch.cuda.synchronize()
        cur = px.tensor_from_device(U)
        lhs = np.sum(np.abs(cur) ** 2)
        rhs = np.sum(np.abs(prev) ** 2 * (1 + p.tau ** 2 * np.abs(prev) ** 4))
        worst = max(worst, abs(lhs - rhs) / rhs)
        prev = cur
    assert worst <= 1e-5, worst
    assert rel_inf(prev, schemes.run_problem(p, steps=10)) <= 1e-5
