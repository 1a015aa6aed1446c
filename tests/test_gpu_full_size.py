"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times: one Tucker operator (the phi matrices of the workload's scheme)
through tucker_apply, checked on sampled entries that the oracle computes one
by one from eq. forloop.

* 384^3 diffusion-reaction, FP64 (single-mode launches, 128x64 tiles);
* 192^3 cubic NLS, complex128 (e^{tau A_mu}, 64x64 complex tiles);
* 128^3 ADR, FP64 (modes 1 and 2 in one fused launch, then mode 3).

Bar per entry: |gpu - oracle| <= 1e-13 * sum_j |M_1[i_1, j_1] ... V[j]|, the
rounding bound of a sum of up to 3 * 384 products accumulated in another order.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle.tensor import tucker_entry

pytestmark = pytest.mark.gpu


def _samples(n, count, seed):
    rng = np.random.default_rng(seed)
    idx = [tuple(0 for _ in n), tuple(k - 1 for k in n), tuple(k // 2 for k in n)]
    idx += [tuple(int(rng.integers(0, k)) for k in n) for _ in range(count)]
    return idx


@pytest.mark.parametrize("name", ["dr384", "nls192", "adr128"])
def test_full_size_tucker_sampled_entries(name):
    p = {"dr384": lambda: W.diffusion_reaction_3d(n=384),
         "nls192": lambda: W.nls_3d(n=192),
         "adr128": lambda: W.adr_3d(n=128)}[name]()
    ell = 0 if p.scheme.startswith("lawson") else 1
    Ms = [px.phi_setup(a, p.tau, ell)[ell] for a in p.A]
    Vd = px.tensor_to_device(p.u0)
    Wd = torch.empty_like(Vd)
    px.tucker_apply([px.matrix_to_device(M) for M in Ms], Vd, Wd)
    torch.cuda.synchronize()
    print(f"{name}: modes 1 and 2 fused = {px.tucker_fuses_modes12(p.n, px.C128 if p.is_complex else px.F64)}",
          flush=True)
    V = np.asarray(p.u0)
    for i in _samples(p.n, 12, seed=len(name)):
        got = Wd[tuple(reversed(i))].item()
        ref, bound = tucker_entry(V, Ms, i)
        assert abs(got - ref) <= 1e-13 * bound, (name, i, got, ref, bound)
