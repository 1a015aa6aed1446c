"""GPU parity of tucker_apply (FP64 MFMA mu-mode products) against the oracle.

Bar: relative max-norm error <= 1e-13 against the oracle's float64 / complex128
Tucker operator on the same inputs (the MFMA path accumulates in FP64 in a
different order; rounding alone explains differences of a few 1e-16 per term).
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
from oracle.norms import rel_inf
from oracle.tensor import tucker

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _rand(shape, seed, cplx=False):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=shape)
    if cplx:
        x = x + 1j * rng.uniform(-1, 1, size=shape)
    return x


def _run(n, seed, cplx=False, skip=(), alpha=1.0, beta=0.0):
    V = _rand(n, seed, cplx)
    Ms = [_rand((k, k), seed + 1 + mu, cplx) / np.sqrt(k) for mu, k in enumerate(n)]
    W0 = _rand(n, seed + 99, cplx)
    Md = [None if mu in skip else px.matrix_to_device(M) for mu, M in enumerate(Ms)]
    Vd = px.tensor_to_device(V)
    Wd = px.tensor_to_device(W0)
    px.tucker_apply(Md, Vd, Wd, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    ref = tucker(V, [np.eye(k) if mu in skip else M for mu, (k, M) in enumerate(zip(n, Ms))])
    ref = alpha * ref + beta * W0
    return px.tensor_from_device(Wd), ref


SHAPES = [(1,), (7,), (64,), (200,), (1, 1, 1), (5, 3), (31, 33), (64, 64), (65, 130),
          (40, 41, 42), (17, 65, 129), (100, 1, 70), (1, 200, 3), (128, 128, 128), (3, 4, 5, 6)]


@pytest.mark.parametrize("n", SHAPES)
def test_tucker_real(n):
    got, ref = _run(n, seed=sum(n))
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("n", SHAPES)
def test_tucker_real_single_mode_launches(n, monkeypatch):
    """The same shapes with modes 1 and 2 as separate launches (EXPINT_FUSE12=0)."""
    monkeypatch.setenv("EXPINT_FUSE12", "0")
    got, ref = _run(n, seed=sum(n))
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("n", [(5,), (5, 7, 3), (48, 48, 48), (33, 17), (96, 96, 96)])
def test_tucker_complex(n):
    got, ref = _run(n, seed=3 + sum(n), cplx=True)
    assert rel_inf(got, ref) <= TOL


@pytest.mark.parametrize("mu", [0, 1, 2])
def test_single_mode_products(mu):
    n = (37, 70, 29)
    skip = tuple(k for k in range(3) if k != mu)
    got, ref = _run(n, seed=50 + mu, skip=skip)
    assert rel_inf(got, ref) <= TOL


def test_alpha_beta_epilogue():
    got, ref = _run((33, 34, 35), seed=61, alpha=-0.75, beta=2.5)
    assert rel_inf(got, ref) <= TOL


def test_deterministic_bitwise():
    n = (64, 80, 48)
    V = px.tensor_to_device(_rand(n, 70))
    Ms = [px.matrix_to_device(_rand((k, k), 71 + i)) for i, k in enumerate(n)]
    W1 = torch.empty_like(V)
    W2 = torch.empty_like(V)
    px.tucker_apply(Ms, V, W1)
    px.tucker_apply(Ms, V, W2)
    torch.cuda.synchronize()
    assert torch.equal(W1, W2)


def test_rejects_aliasing_and_short_workspace():
    V = px.tensor_to_device(_rand((8, 9, 10), 80))
    Ms = [px.matrix_to_device(np.eye(k)) for k in (10, 9, 8)[::-1]]
    with pytest.raises(px.ExpintError):
        px.tucker_apply(Ms, V, V)
    W = torch.empty_like(V)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(px.ExpintError):
        px.tucker_apply(Ms, V, W, ws=ws)


@pytest.mark.parametrize("tile", ["64x64", "64x32", "32x64", "128x64", "64x128", "32x32",
                                  "64x64w8", "128x64w8", "128x128w8", "128x128", "128x64w8k32",
                                  "128x128w8k32", "128x64w8p3", "128x64w8p4", "64x64w8p3",
                                  "64x64w8p4", "64x64k32"])
@pytest.mark.parametrize("cplx", [False, True])
def test_every_tile_shape(tile, cplx, monkeypatch):
    """Each tile shape the launcher can pick (forced through EXPINT_TILE) on ragged sizes."""
    monkeypatch.setenv("EXPINT_TILE", tile)
    got, ref = _run((37, 70, 133), seed=90, cplx=cplx)
    assert rel_inf(got, ref) <= TOL
