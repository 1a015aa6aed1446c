"""tucker_apply_noalloc: the Tucker operator with its intermediates in the
library's fixed device scratch array, for callers that cannot allocate.

Each case makes two calls in a row on one device, the second with a smaller
tensor (so the scratch array still holds the first call's larger contents),
and checks each result against tucker_apply's on the same inputs (bitwise:
the same kernels run in the same order) and against the oracle's Tucker
operator (section 1, eq. tuckerexp) at the bar of each contraction precision.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
from oracle.norms import rel_inf
from oracle.tensor import tucker

pytestmark = pytest.mark.gpu

# rel-inf bound against the oracle per contraction precision (FP64 as tucker_apply's
# own parity tests; reduced precisions at their stated per-contraction bounds)
TOL = {"fp64": 1e-13, "fp32": 1e-5, "bf16x3": 1e-4, "slice": 1e-10}


def _case(n, seed, cplx=False, alpha=1.0, beta=0.0):
    rng = np.random.default_rng(seed)
    V = rng.uniform(-1, 1, size=n)
    W0 = rng.uniform(-1, 1, size=n)
    Ms = [rng.uniform(-1, 1, size=(k, k)) / np.sqrt(k) for k in n]
    if cplx:
        V = V + 1j * rng.uniform(-1, 1, size=n)
        W0 = W0 + 1j * rng.uniform(-1, 1, size=n)
        Ms = [M + 1j * rng.uniform(-1, 1, size=M.shape) / np.sqrt(M.shape[0]) for M in Ms]
    ref = alpha * tucker(V, Ms) + beta * W0
    return V, W0, Ms, ref


def _both(n, seed, precision, cplx=False, alpha=1.0, beta=0.0):
    V, W0, Ms, ref = _case(n, seed, cplx, alpha, beta)
    Md = [px.matrix_to_device(M) for M in Ms]
    Vd = px.tensor_to_device(V)
    Wa = px.tensor_to_device(W0)
    Wb = px.tensor_to_device(W0)
    px.tucker_apply(Md, Vd, Wa, alpha=alpha, beta=beta, precision=precision)
    px.tucker_apply_noalloc(Md, Vd, Wb, alpha=alpha, beta=beta, precision=precision)
    torch.cuda.synchronize()
    return Wa, Wb, ref


PAIRS = [
    # (first shape, second smaller shape)
    ((96, 80, 72), (40, 41, 42)),
    ((128, 128, 64), (17, 65, 29)),
    ((300, 250), (7, 5)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "slice"])
@pytest.mark.parametrize("shapes", PAIRS)
def test_noalloc_matches_tucker_apply_two_calls(precision, shapes):
    for k, n in enumerate(shapes):
        print(f"noalloc {precision} call {k + 1}: n = {n}", flush=True)
        Wa, Wb, ref = _both(n, seed=11 * (k + 1) + sum(n), precision=precision, alpha=0.5 + k, beta=0.25 * k)
        assert torch.equal(Wa, Wb)
        err = rel_inf(px.tensor_from_device(Wb), ref)
        assert err <= TOL[precision]
        if precision != "fp64":
            assert err > 1e-17  # the reduced contraction really ran


def test_noalloc_complex_two_calls():
    for k, n in enumerate([(64, 48, 40), (9, 11, 13)]):
        print(f"noalloc complex128 call {k + 1}: n = {n}", flush=True)
        Wa, Wb, ref = _both(n, seed=5 + k, precision="fp64", cplx=True)
        assert torch.equal(Wa, Wb)
        assert rel_inf(px.tensor_from_device(Wb), ref) <= 1e-13


def test_noalloc_fused_modes12_then_single_modes():
    """The first call runs modes 1 and 2 as one launch (n_2 <= 128), the second a
    smaller shape through the single-mode kernels of the FP32 path."""
    n1, n2 = (128, 96, 60), (33, 20, 10)
    assert px.tucker_fuses_modes12(n1)
    Wa, Wb, ref = _both(n1, seed=3, precision="fp64")
    assert torch.equal(Wa, Wb)
    assert rel_inf(px.tensor_from_device(Wb), ref) <= 1e-13
    Wa, Wb, ref = _both(n2, seed=4, precision="fp32")
    assert torch.equal(Wa, Wb)
    assert rel_inf(px.tensor_from_device(Wb), ref) <= 1e-5


def test_noalloc_rejects_shapes_beyond_the_scratch():
    # 192^3 FP64 with three modes needs two 56.6 MB intermediates: more than the array holds
    n = (192, 192, 192)
    assert px.tucker_workspace_size(n) > px.NOALLOC_SCRATCH_BYTES
    V = torch.zeros(n, dtype=torch.float64, device="cuda")
    W = torch.zeros_like(V)
    Md = [torch.eye(k, dtype=torch.float64, device="cuda") for k in n]
    with pytest.raises(px.ExpintError) as e:
        px.tucker_apply_noalloc(Md, V, W)
    assert e.value.code == px._binding.ENOTSUP
    assert "scratch" in str(e.value)
    # a single mode needs no intermediate, so it runs at any size below the operand limit
    Md1 = [Md[0], None, None]
    V.normal_()
    px.tucker_apply_noalloc(Md1, V, W)
    torch.cuda.synchronize()
    assert torch.equal(W, V)
