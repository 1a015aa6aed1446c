"""The autotuner (tucker_tune, and expint_problem.tune at plan creation).

* Every candidate launch configuration of a family computes the same sums in
  the same order, so the results of all FP64 tiles, of the fused and unfused
  modes 1 and 2 and of all exact-slice tiles are bitwise equal; a tuned plan
  therefore equals a plan forced to its chosen configuration, bitwise.
* A tuned shape is not timed again: in one process the table answers, and
  with EXPINT_TUNE_CACHE a second process reads the first one's choices
  (the cache file gains no lines and the choices are the same).
* Tuned Tucker operators stay within the oracle tolerance (eq. tuckerexp).
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import paper_2304_02327_amd as px
import workloads as W
from oracle.norms import rel_inf
from oracle.tensor import tucker

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, size=shape)


def _apply(n, seed, precision="fp64"):
    V = _rand(n, seed)
    Ms = [_rand((k, k), seed + 1 + i) / np.sqrt(k) for i, k in enumerate(n)]
    Vd = px.tensor_to_device(V)
    Wd = torch.zeros_like(Vd)
    px.tucker_apply([px.matrix_to_device(M) for M in Ms], Vd, Wd, precision=precision)
    torch.cuda.synchronize()
    return Wd, V, Ms


FP64_TILES = ["64x64", "64x32", "32x64", "128x64", "64x128", "32x32", "64x64w8", "128x64w8", "128x128w8",
              "128x128", "128x64w8k32", "128x128w8k32", "128x64w8p3", "128x64w8p4", "64x64w8p3", "64x64w8p4",
              "64x64k32", "128x64w8i", "64x64w8i"]


def test_every_fp64_tile_gives_the_same_bits(monkeypatch):
    n = (37, 70, 133)
    ref, V, Ms = _apply(n, 5)
    assert rel_inf(px.tensor_from_device(ref), tucker(V, Ms)) <= 1e-13
    for t in FP64_TILES:
        monkeypatch.setenv("EXPINT_TILE", t)
        got, _, _ = _apply(n, 5)
        assert torch.equal(got, ref), t


def test_fused_and_unfused_modes12_give_the_same_bits(monkeypatch):
    n = (64, 96, 40)
    assert px.tucker_fuses_modes12(n)
    ref, V, Ms = _apply(n, 7)
    for shape in ["r32w4", "r32w8", "r16w4", "r64w8", "r64w16", "r32w8p", "r32w8i", "r64w16p", "r64w16i", "off"]:
        monkeypatch.setenv("EXPINT_M12", shape)
        got, _, _ = _apply(n, 7)
        assert torch.equal(got, ref), shape
    monkeypatch.delenv("EXPINT_M12")
    monkeypatch.setenv("EXPINT_FUSE12", "0")
    got, _, _ = _apply(n, 7)
    assert torch.equal(got, ref)


def test_every_slice_tile_gives_the_same_bits(monkeypatch):
    n = (40, 70, 129)
    ref, V, Ms = _apply(n, 9, "slice")
    for t in ["64x64w4k64s2o2", "128x64w8k64s2o1", "64x128w8k64s2o1", "64x64w4k32s2o3", "64x64w4k32s4o2",
              "128x64w8k32s4o1"]:
        monkeypatch.setenv("EXPINT_SLICE_TILE", t)
        got, _, _ = _apply(n, 9, "slice")
        assert torch.equal(got, ref), t


LP_TILES = {"fp32": ["128x64w8", "64x64w4", "128x128w8", "128x128w16", "256x128w16"],
            "bf16x3": ["64x64w4", "128x128w8", "128x128w8t", "256x128w8", "128x256w8t"]}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_every_reduced_precision_tile_gives_the_same_bits(precision, monkeypatch):
    """Ragged sizes around every tile (FP64 first mode, FP32 inner mode, FP64 last mode)."""
    n = (37, 300, 133)
    ref, V, Ms = _apply(n, 13, precision)
    err = rel_inf(px.tensor_from_device(ref), tucker(V, Ms))
    assert 1e-17 < err <= (1e-5 if precision == "fp32" else 1e-4)
    for t in LP_TILES[precision]:
        monkeypatch.setenv("EXPINT_LP_TILE", t)
        got, _, _ = _apply(n, 13, precision)
        assert torch.equal(got, ref), t


TOL = {"fp64": 1e-13, "slice": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}


@pytest.mark.parametrize("precision", ["fp64", "slice", "fp32", "bf16x3"])
def test_tuned_tucker_matches_oracle(precision):
    n = (48, 100, 36)
    px.tucker_tune(list(n), precision=precision)
    got, V, Ms = _apply(n, 11, precision)
    assert rel_inf(px.tensor_from_device(got), tucker(V, Ms)) <= TOL[precision]


def test_tuned_plan_equals_forced_plan_bitwise(monkeypatch):
    p = W.adr_3d(n=(72, 80, 96), steps=3)
    tuned = px.Plan(p.A, p.tau, p.scheme, p.g, tune=True)
    text = tuned.describe()
    assert "tuned" in text, text
    U1 = px.tensor_to_device(p.u0)
    tuned.run(U1, p.steps)
    torch.cuda.synchronize()
    # force the choice of mode 3 on every single-mode launch, with modes 1 and 2 unfused
    mode3 = [l for l in text.splitlines() if l.startswith("mode 3:")][0]
    tile = mode3.split(": ")[-1].split(" ")[0]
    assert tile in FP64_TILES, mode3
    monkeypatch.setenv("EXPINT_TILE", tile)
    forced = px.Plan(p.A, p.tau, p.scheme, p.g, tune=False)
    U2 = px.tensor_to_device(p.u0)
    forced.run(U2, p.steps)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)
    tuned.close()
    forced.close()


CHILD = r"""
import json, os, sys
sys.path.insert(0, {root!r})
import torch
import paper_2304_02327_amd as px
import workloads as W
p = W.diffusion_reaction_3d(n=(40, 41, 42))
plan = px.Plan(p.A, p.tau, p.scheme, p.g, tune=True)
U = px.tensor_to_device(p.u0)
plan.run(U, 2)
torch.cuda.synchronize()
print(json.dumps({{"describe": plan.describe(), "sum": float(U.sum().item())}}))
"""


def test_tune_cache_file_is_reused_across_processes(tmp_path):
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, EXPINT_TUNE_CACHE=str(cache))
    env.pop("EXPINT_TILE", None)
    code = CHILD.format(root=ROOT)
    outs = []
    for k in range(2):
        print(f"tune cache child {k + 1}", flush=True)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
        if k == 0:
            lines = cache.read_text().splitlines()
            assert len(lines) >= 3, lines  # three mode products (and modes 1 and 2) were tuned
    assert cache.read_text().splitlines() == lines  # the second process timed nothing
    assert outs[0]["describe"] == outs[1]["describe"]
    assert outs[0]["sum"] == outs[1]["sum"]
