"""Grouped tile schemes of the batched engine (one persistent launch per phase,
with one or two tile classes) and their autotuning (expint_batch_tune).

* Every scheme computes each output element's K sum in index order, so the
  states after a few ETD2RK or Rosenbrock-Euler steps are bitwise equal across
  schemes, and across workgroup orders (the XCD-aware map and the plain one);
  the instances span both classes (M below and above 128, Q below and above
  128) and ragged tile edges.
* Tuning runs on a copy of the state: U and the status words are unchanged,
  every phase then holds a tuned choice, and the tuned plan's steps equal the
  untuned ones bitwise.  The result is checked against the oracle too.
"""

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle import nonlinear, schemes
from oracle.norms import rel_inf

pytestmark = pytest.mark.gpu

TILES = ["64x64k16", "64x64k16o4", "64x64", "64x64w4", "128x64", "128x64k8", "64x64+128x64",
         "64x64k16+128x64k8"]
SCHEMES = TILES + [t + ",lpt64" for t in TILES]  # each tile scheme with both workgroup maps


def _instances(seed=41):
    insts = W.riccati_batch(count=9, nmin=20, nmax=300, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for x in insts:
        x.U0 = 0.3 * rng.standard_normal((x.n1, x.n2))
    return insts


def _run(insts, scheme, steps, tune=False):
    batch = px.RiccatiBatch(insts, 1e-3, scheme=scheme)
    U = batch.state_to_device([x.U0 for x in insts])
    if tune:
        before = U.clone()
        batch.tune(U)
        torch.cuda.synchronize()
        assert torch.equal(U, before)
        assert batch.status() == 0
        text = batch.describe()
    else:
        text = None
    batch.run(U, steps)
    torch.cuda.synchronize()
    out = U.clone()
    got = batch.state_from_device(U)
    batch.close()
    return out, got, text


@pytest.mark.parametrize("scheme", ["etd2rk", "rosenbrock_euler"])
def test_every_grouped_scheme_gives_the_same_bits(scheme, monkeypatch):
    insts = _instances()
    sizes = [(x.n1, x.n2) for x in insts]
    assert any(n1 >= 128 for n1, _ in sizes) and any(n1 < 128 for n1, _ in sizes), sizes
    assert any(min(n1, n2) >= 128 for n1, n2 in sizes), sizes
    ref = None
    for name in SCHEMES:
        print(f"{scheme} grouped scheme {name}", flush=True)
        monkeypatch.setenv("EXPINT_GROUPED", name)
        out, got, _ = _run(insts, scheme, 3)
        if ref is None:
            ref = out
            if scheme == "etd2rk":
                x = insts[0]
                g = nonlinear.make_g("riccati", {"B": x.B, "C": x.C})
                want = schemes.Integrator([x.A1, x.A2], 1e-3, "etd2rk", g).run(x.U0, 0.0, 3)
                assert rel_inf(got[0], want) <= 1e-12
        else:
            assert torch.equal(out, ref), name
    # the plain workgroup order instead of the XCD-aware map
    monkeypatch.setenv("EXPINT_GROUPED", "64x64k16")
    monkeypatch.setenv("EXPINT_GROUPED_FLAT", "1")
    out, _, _ = _run(insts, scheme, 3)
    assert torch.equal(out, ref)


@pytest.mark.parametrize("scheme", ["etd2rk", "rosenbrock_euler"])
def test_tuned_plan_leaves_the_state_and_matches_untuned(scheme, monkeypatch):
    insts = _instances(seed=43)
    monkeypatch.setenv("EXPINT_GROUPED", "64x64k16")
    ref, _, _ = _run(insts, scheme, 2)
    monkeypatch.delenv("EXPINT_GROUPED")
    out, got, text = _run(insts, scheme, 2, tune=True)
    lines = text.splitlines()
    assert len(lines) >= 9 and all("tuned" in l for l in lines), text
    assert all(l.split(": ")[1].split(" ")[0] in SCHEMES for l in lines), text
    assert torch.equal(out, ref)
