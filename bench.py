"""Benchmark: direction-split exponential integrator steps on one MI355X.

Default workload: the precision sweep on 3-D diffusion-reaction, 384^3,
ETD2RK phisplit, tau = 2e-3 (A_mu = 0.02 D2, g = u^2 (1 - u), u0 ~ U(0, 1)).
A "step" is one full ETD2RK time step over the whole tensor (stage input with
K u and g, two Tucker operators with the fused stage combinations), replayed
from a HIP graph; inputs are resident in HBM before each timed region starts.
The mu-mode contractions run in four precisions, each timed over the same K
steps: FP32, split BF16 (bf16x3), exact slice (int8 digits) and FP64, which
gives `value`.  Each reduced leg reports its time, its speed-up over FP64,
its error against the FP64 run and against the CPU oracle, and its own
roofline.

Prints one JSON line with DOF-steps/s, the roofline of the dominant kernel
(the FP64 MFMA mu-mode product) and the CPU oracle timed on the host.
Other workloads: --workload adr128 | allen_cahn64 | nls192 | dr384 |
riccati64 | riccati64_ros | adr_paper40 | adr_paper80.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-steps/s + % of MFMA roofline, FP64 vs split-BF16 at stated rel. error"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 MFMA
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 MFMA
PEAK_BF16_TFLOPS = 2516.6  # MI355X dense BF16 MFMA
PEAK_INT8_TOPS = 5000.0    # MI355X dense INT8 MFMA
SLICE_PRODUCTS = 19        # digit products a_i b_j (i + j <= 5) per multiply-add of the exact-slice path
PEAK_HBM_GBS = 8000.0


def make_workload(name: str):
    import workloads as W
    if name == "adr128":
        p = W.adr_3d(n=128)
        desc = "3-D ADR 128^3, ETD2RK phisplit, FP64, tau=2e-3"
    elif name == "allen_cahn64":
        p = W.allen_cahn_2d()
        desc = "2-D Allen-Cahn 64^2, exponential Euler phisplit, FP64, tau=1e-3"
    elif name == "nls192":
        p = W.nls_3d(n=192)
        desc = "3-D cubic NLS 192^3, Lawson-Euler, complex128, tau=1e-3"
    elif name == "dr384":
        p = W.diffusion_reaction_3d(n=384)
        desc = "3-D diffusion-reaction 384^3, ETD2RK phisplit, FP64, tau=2e-3"
    elif name in PAPER_RUNS:
        n, steps, _, _ = PAPER_RUNS[name]
        p = W.adr_paper(n, steps=steps, scheme="etd2rk")
        desc = (f"section 4.2 ADR {n[0]}x{n[1]}x{n[2]} (eps=0.75, alpha=0.1, manufactured source), "
                f"ETD2RK phisplit, {steps} steps to T=1, FP64")
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, desc


# The paper's ETD2RK phisplit runs of the section 4.2 ADR problem at the finest step
# size of its order study (Figures adr_ord12_40 and adr_ord12): grid, steps, wall
# clock in seconds and the printed relative infinity-norm error at T = 1.  Measured
# in MATLAB R2022a on an Intel Core i7-10750H (6 cores), FP64.
PAPER_RUNS = {
    "adr_paper40": ((40, 41, 42), 440, 0.4505, 2.14158850419228e-06),
    "adr_paper80": ((80, 81, 82), 440, 7.8158, 2.14108285352612e-06),
}
PAPER_HW = "MATLAB R2022a, Intel Core i7-10750H (6 cores), FP64"


def plan_kwargs(p):
    """Nonlinearity parameters of a workload as the plan takes them."""
    if p.g == "cubic_nls":
        return {"g_param": p.g_params.get("kappa", 0.0)}
    if p.g == "adr_paper":
        return {"g_param": p.g_params["eps"], "g_param2": p.g_params["alpha"]}
    return {}


# Committed rocprofv3 PMC summaries of the dominant kernel, per workload and
# contraction precision.  Each lists the sources the kernel is compiled from and
# their SHA-256; `traffic` is reported only while that hash matches the tree.
TRAFFIC_FILES = {
    ("adr128", "fp64"): "k_modes12_adr128_hbm_traffic.md",
    ("dr384", "fp64"): "k_mode_product_dr384_hbm_traffic.md",
    ("dr384", "fp32"): "k_mode_product_f32_dr384_hbm_traffic.md",
    ("dr384", "bf16x3"): "k_mode_product_bf16x3_dr384_hbm_traffic.md",
    ("dr384", "slice"): "k_sliced_dr384_hbm_traffic.md",
}


def sources_sha256(rels):
    """SHA-256 over the named source files (paths relative to the repository), or None
    if one of them is missing."""
    import hashlib
    h = hashlib.sha256()
    for rel in rels:
        path = os.path.join(ROOT, rel)
        if not os.path.isfile(path):
            return None
        h.update(rel.encode())
        h.update(open(path, "rb").read())
    return h.hexdigest()


def _summary_fields(path):
    fields = {}
    for line in open(path):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            fields[k] = v
    return fields


def measured_traffic(workload: str, precision: str = "fp64"):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary, or None when
    there is none for this workload and precision or the kernel's sources changed since the
    counters were taken."""
    name = TRAFFIC_FILES.get((workload, precision))
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = _summary_fields(path)
    rels = [r.strip() for r in fields.get("kernel_sources", "").split(",") if r.strip()]
    if not rels or fields.get("kernel_sources_sha256") != sources_sha256(rels):
        return None
    return float(fields["traffic_bytes_per_launch"])


def calibrate_copy():
    """A plain copy kernel of known size: reads and writes 512 MiB per launch, so the
    FETCH_SIZE / WRITE_SIZE counters it produces give their scale factor."""
    import torch
    n = 512 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 8, "launches": 5}))


def tucker_flops_per_step(p) -> float:
    """Algorithmic flops of the Tucker operators of one step (2 N n_mu per real mode
    product, 8 N n_mu per complex one)."""
    per_tucker = sum((8 if p.is_complex else 2) * p.N * nm for nm in p.n)
    tuckers = {"lawson_euler": 1, "exp_euler": 1, "lawson2b": 2, "etd2rk": 2}[p.scheme]
    return tuckers * per_tucker


def riccati_flops_per_step(insts) -> float:
    """Algorithmic flops of one ETD2RK step of every instance: T and G (twice each,
    2 n1 n2 min(n1, n2) apiece), K u (2 n1^2 n2 + 2 n1 n2^2) and two Tucker operators
    (the same again each)."""
    tot = 0.0
    for x in insts:
        n1, n2 = x.n1, x.n2
        tot += n1 * n2 * (8 * min(n1, n2) + 6 * n1 + 6 * n2)
    return tot


def rosenbrock_flops_per_step(insts, tau) -> float:
    """Algorithmic flops of one Rosenbrock-Euler step of the batch: the Jacobian
    directions and W (4 GEMMs), phi_1 of both directions (13 Taylor products and 2
    per squaring, with the squarings that ||tau A_mu||_1 calls for, rounded up to
    even as the device does), and the Tucker operator (2 GEMMs)."""
    import numpy as np
    total = 0.0
    for x in insts:
        n1, n2 = x.n1, x.n2
        total += 2.0 * n1 * n2 * (n1 + n2) * 2 + 2.0 * n1 * n2 * (n1 + n2)
        for A, n in ((x.A1, n1), (x.A2, n2)):
            nu = tau * np.abs(A).sum(axis=0).max()
            s = 0
            while nu > 0.5:
                nu *= 0.5
                s += 1
            s += s & 1
            total += 2.0 * n**3 * (13 + 2 * s)
    return total


def batch_smax(insts, tau) -> int:
    """Squaring phases per Rosenbrock-Euler step, as the plan fixes them."""
    import numpy as np
    nu = max(tau * np.abs(A).sum(axis=0).max() for x in insts for A in (x.A1, x.A2))
    s = 0
    while nu > 0.5 and s < 60:
        nu *= 0.5
        s += 1
    return s + 4 + ((s + 4) & 1)


def bench_riccati(args, scheme="etd2rk"):
    """64 Riccati-type instances, n1, n2 ~ U{32..512}, ETD2RK or Rosenbrock-Euler phisplit, FP64."""
    import numpy as np
    import torch
    import paper_2304_02327_amd as px
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    insts = W.riccati_batch()
    tau = 1e-3
    t = time.perf_counter()
    batch = px.RiccatiBatch(insts, tau, device=dev, scheme=scheme)
    setup_s = time.perf_counter() - t
    U0 = batch.state_to_device([x.U0 for x in insts])
    U = U0.clone()
    N = batch.state_size
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    t = time.perf_counter()
    if not args.no_tune:
        batch.tune(U, stream=stream)  # each phase's grouped tile scheme (U is left as it is)
    tune_s = time.perf_counter() - t
    with torch.cuda.stream(stream):
        batch.run(U, args.warmup, use_graph=True, stream=stream)
    stream.synchronize()
    U.copy_(U0)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    with torch.cuda.stream(stream):
        batch.run(U, args.steps, use_graph=True, stream=stream)
    ev1.record(stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ros = scheme == "rosenbrock_euler"
    flops = rosenbrock_flops_per_step(insts, tau) if ros else riccati_flops_per_step(insts)
    tf = flops * args.steps / (gpu_ms / 1e3) / 1e12
    name = "Rosenbrock-Euler" if ros else "ETD2RK"
    launches = (18 + batch_smax(insts, tau)) if ros else 9
    result = {
        "metric": METRIC, "value": N * args.steps / (gpu_ms / 1e3), "unit": "DOF-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": gpu_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"64 Riccati-type instances, n1,n2 ~ U{{32..512}}, {name} phisplit, FP64, tau=1e-3",
                   "dof": N, "graph": True, "launches_per_step": launches},
        "wall_s_timed_region": wall, "phi_setup_s": setup_s, "tune_s": round(tune_s, 3),
        "launch_configuration": batch.describe().splitlines(),
        "roofline": {"kernel": f"k_grouped_gemm ({launches} persistent FP64 MFMA launches per step)",
                     "bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "flops_per_step": flops, "avg_launch_us": round(gpu_ms * 1e3 / args.steps / launches, 3)},
    }
    if not args.no_cpu_baseline:
        from oracle import nonlinear, schemes
        from oracle.norms import rel_inf
        sample = list(range(0, 64, 2))  # 32 of the 64 instances
        t = time.perf_counter()
        integs = []
        for i in sample:
            x = insts[i]
            g = nonlinear.make_g("riccati", {"B": x.B, "C": x.C})
            if not ros:
                integs.append(schemes.Integrator([x.A1, x.A2], tau, "etd2rk", g))
        osetup = time.perf_counter() - t

        def oracle_run(steps):
            if ros:
                return [schemes.run_rosenbrock_euler_riccati(insts[i].U0, tau, steps, insts[i].A1, insts[i].A2,
                                                             insts[i].B, insts[i].C) for i in sample]
            return [integ.run(insts[i].U0, 0.0, steps) for integ, i in zip(integs, sample)]

        # the number of steps from one timed step: about --cpu-seconds / 2 of CPU work, 2 .. 500 steps
        t = time.perf_counter()
        oracle_run(1)
        one = time.perf_counter() - t
        k = int(max(2, min(500, 0.5 * args.cpu_seconds / max(one, 1e-3))))
        t = time.perf_counter()
        outs = oracle_run(k)
        secs = time.perf_counter() - t
        Ug = U0.clone()
        batch.run(Ug, k)
        torch.cuda.synchronize()
        got = batch.state_from_device(Ug)
        err = max(rel_inf(got[i], o) for i, o in zip(sample, outs))
        dof = sum(insts[i].n1 * insts[i].n2 for i in sample)
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count() or 1
        result["cpu_baseline"] = {"value": dof * k / secs, "unit": "DOF-steps/s", "cores": cores,
                                  "kind": "oracle", "sample": f"{k} steps of the even-numbered 32 of the 64 "
                                  f"instances (oracle phi setup {osetup:.1f} s excluded)", "seconds": round(secs, 3),
                                  "gpu_vs_oracle_rel_inf": err}
    batch.close()
    print(json.dumps(result))


SWEEP_PRECISIONS = ("fp32", "bf16x3", "slice", "fp64")  # FP64 last: its timed region gives `value`
PREC_DTYPE = {"fp64": "f64", "fp32": "f32 (state f64)", "bf16x3": "bf16x3/f32acc (state f64)",
              "slice": "int8 digits x5/int32 acc (state f64)"}
# the stated bound of each precision's error against the FP64 oracle (rel-inf, a few steps)
PREC_BOUND = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4, "slice": 1e-10}


def _event_ms(stream, fn):
    """Time fn() with HIP events recorded on `stream` (the stream its kernels run on)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1)


def time_steps(plan, U0, steps, warmup, stream, repeats=0):
    """W untimed graph-replayed steps (including the one-time capture), then exactly
    `steps` timed ones from U0 with HIP events on the plan's stream, bracketed by
    device synchronisation; optional repeat regions for the spread.  Returns
    (ms of the timed region, wall seconds, final state, repeat ms per step)."""
    import torch
    U = U0.clone()
    with torch.cuda.stream(stream):
        plan.run(U, warmup, t0=0.0, use_graph=True, stream=stream)
    stream.synchronize()
    U.copy_(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = _event_ms(stream, lambda: plan.run(U, steps, t0=0.0, use_graph=True, stream=stream))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    final = U.clone()
    reps = []
    for _ in range(repeats):
        U.copy_(U0)
        torch.cuda.synchronize()
        reps.append(_event_ms(stream, lambda: plan.run(U, steps, t0=0.0, use_graph=True, stream=stream))
                    / max(steps, 1))
    bitwise = bool(torch.equal(U, final)) if repeats else None
    return ms, wall, final, reps, bitwise


def bench_sweep(args):
    """The precision sweep: 384^3 diffusion-reaction, ETD2RK, K steps in FP32, bf16x3,
    exact slice and FP64 contraction; `value` is the FP64 leg."""
    import numpy as np
    import torch
    import paper_2304_02327_amd as px
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = W.diffusion_reaction_3d(n=384)
    if args.steps is None:
        args.steps = p.steps
    desc = ("precision sweep: 3-D diffusion-reaction 384^3, ETD2RK phisplit, tau=2e-3, "
            "mu-mode contractions in FP64 vs FP32 vs split-BF16 (bf16x3) vs exact slice (int8 digits)")
    U0 = px.tensor_to_device(p.u0, device=dev)
    stream = torch.cuda.Stream()  # default priority
    stream.wait_stream(torch.cuda.current_stream())
    legs, finals = {}, {}
    for prec in SWEEP_PRECISIONS:
        t = time.perf_counter()
        plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=prec)
        setup_s = time.perf_counter() - t
        ms, wall, final, reps, bitwise = time_steps(plan, U0, args.steps, args.warmup, stream,
                                                    repeats=5 if prec == "fp64" else 0)
        if not plan.check_finite(final, stream=stream):
            raise SystemExit(f"non-finite state after the timed region ({prec})")
        finals[prec] = final
        leg = {"ms_per_step": ms / args.steps, "value": p.N * args.steps / (ms / 1e3), "unit": "DOF-steps/s",
               "dtype": PREC_DTYPE[prec], "wall_s_timed_region": wall, "plan_setup_s": round(setup_s, 3),
               "launch_configuration": plan.describe().strip().splitlines(),
               "stated_bound_rel_inf": PREC_BOUND[prec],
               "roofline": tucker_roofline(args, p, px, dev, stream, U0, prec, "dr384")}
        if reps:
            leg["repeat_ms_per_step"] = [round(x, 5) for x in reps]
            leg["median_ms_per_step_of_repeats"] = round(sorted(reps)[len(reps) // 2], 5)
            leg["repeats_bitwise_equal_to_timed_state"] = bitwise
        legs[prec] = leg
        plan.close()
    fp = legs["fp64"]
    ref = finals["fp64"]
    scale = ref.abs().max().item()
    reduced = {}
    for prec in SWEEP_PRECISIONS[:-1]:
        leg = legs[prec]
        leg["speedup_vs_fp64"] = fp["ms_per_step"] / leg["ms_per_step"]
        leg[f"rel_inf_vs_fp64_after_{args.steps}_steps"] = (finals[prec] - ref).abs().max().item() / scale
        reduced[prec] = leg
    result = {
        "metric": METRIC,
        "value": fp["value"],
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": list(p.n), "scheme": p.scheme, "tau": p.tau, "graph": True,
                   "value_from": "the FP64 leg; the other legs are in precision_legs"},
        "wall_s_timed_region": fp["wall_s_timed_region"],
        "repeat_ms_per_step": fp["repeat_ms_per_step"],
        "median_ms_per_step_of_repeats": fp["median_ms_per_step_of_repeats"],
        "repeats_bitwise_equal_to_timed_state": fp["repeats_bitwise_equal_to_timed_state"],
        "tucker_tflops_whole_step": round(tucker_flops_per_step(p) * args.steps / (fp["ms_per_step"] * args.steps
                                                                                   / 1e3) / 1e12, 3),
        "roofline": fp["roofline"],
        "launch_configuration": fp["launch_configuration"],
        "precision_legs": reduced,
    }
    if not args.no_cpu_baseline:
        base, oracle_state, k = oracle_sample(p, args.cpu_seconds)
        # every leg against the oracle after the same k steps (direct launches)
        for prec in SWEEP_PRECISIONS:
            plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=prec)
            Ug = U0.clone()
            plan.run(Ug, k)
            torch.cuda.synchronize()
            err = float(np.abs(px.tensor_from_device(Ug) - oracle_state).max() / np.abs(oracle_state).max())
            plan.close()
            if prec == "fp64":
                base["gpu_vs_oracle_rel_inf"] = err
            else:
                reduced[prec][f"rel_inf_vs_oracle_after_{k}_steps"] = err
                reduced[prec]["within_stated_bound"] = bool(err <= PREC_BOUND[prec])
        result["cpu_baseline"] = base
    print(json.dumps(result))


def bench_single(args):
    """One workload in one contraction precision."""
    import numpy as np
    import torch
    import paper_2304_02327_amd as px

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p, desc = make_workload(args.workload)
    if args.steps is None:
        args.steps = p.steps if args.workload in PAPER_RUNS else 100
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    plan = px.Plan(p.A, p.tau, p.scheme, p.g, precision=args.precision, **plan_kwargs(p))
    U0 = px.tensor_to_device(p.u0, device=dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    stream = torch.cuda.Stream()  # default priority
    stream.wait_stream(torch.cuda.current_stream())
    gpu_ms, wall, U, repeats, bitwise = time_steps(plan, U0, args.steps, args.warmup, stream, repeats=5)
    ms_per_step = gpu_ms / max(args.steps, 1)
    value = p.N * args.steps / (gpu_ms / 1e3)
    if not plan.check_finite(U, stream=stream):
        raise SystemExit("non-finite state after the timed region")

    if plan.fused:
        # the whole timed run is one launch of the fused small-problem kernel: its
        # duration is the event time of the timed region, its work the Tucker flops
        # of every step; one workgroup can use at most one CU's share of the peak
        flops_per_launch = tucker_flops_per_step(p) * args.steps
        avg_launch_s = gpu_ms / 1e3
        achieved_tf = flops_per_launch / avg_launch_s / 1e12
        roofline = {
            "kernel": "k_small2d (fused single-workgroup run, FP64 MFMA)",
            "bound": "mfma",
            "achieved": round(achieved_tf, 4),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 5),
            "traffic": None,
            "frac_of_one_cu": round(achieved_tf / (PEAK_FP64_TFLOPS / 256), 4),
            "traffic_unit": "bytes per launch (state read once, written once)",
            "algorithmic_bytes_per_launch": 2 * 8 * p.N,
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "flops_per_launch": flops_per_launch,
            "us_per_step": round(avg_launch_s * 1e6 / max(args.steps, 1), 3),
        }
    else:
        roofline = tucker_roofline(args, p, px, dev, stream, U0, args.precision, args.workload)
    step_tf = tucker_flops_per_step(p) * args.steps / (gpu_ms / 1e3) / 1e12

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("c128" if p.is_complex else "f64") if args.precision == "fp64" else
                 ("c64 (state c128)" if p.is_complex else PREC_DTYPE[args.precision]),
        "data": "synthetic",
        "config": {"workload": desc, "n": list(p.n), "scheme": p.scheme, "tau": p.tau,
                   "precision": args.precision, "graph": True},
        "wall_s_timed_region": wall,
        "launch_configuration": plan.describe().strip().splitlines(),
        "repeat_ms_per_step": [round(x, 5) for x in repeats],
        "median_ms_per_step_of_repeats": round(sorted(repeats)[len(repeats) // 2], 5),
        "repeats_bitwise_equal_to_timed_state": bitwise,
        "tucker_tflops_whole_step": round(step_tf, 3),
        "roofline": roofline,
    }

    if args.workload in PAPER_RUNS and args.steps == p.steps:
        # the whole integration to T = 1, against the paper's run of the same problem
        _, _, paper_s, paper_err = PAPER_RUNS[args.workload]
        exact = math.exp(1.0) * np.asarray(p.u0)  # the manufactured solution e^t u0 at t = 1
        Uh = px.tensor_from_device(U)
        err = float(np.abs(Uh - exact).max() / np.abs(exact).max())
        paper_value = p.N * p.steps / paper_s
        result["vs_baseline"] = value / paper_value
        result["paper_run"] = {
            "hardware": PAPER_HW, "seconds": paper_s, "steps": p.steps,
            "dof_steps_per_s": paper_value, "rel_err_inf_printed": paper_err,
        }
        result["rel_err_inf_vs_exact_at_T"] = err
        result["seconds_setup_plus_steps"] = setup_s + gpu_ms / 1e3
        result["setup_s_phi_on_host_and_upload"] = setup_s
    if args.precision != "fp64":
        # error of the reduced-precision run against the FP64 path after the same steps
        ref_plan = px.Plan(p.A, p.tau, p.scheme, p.g, **plan_kwargs(p))
        Uref = U0.clone()
        ref_plan.run(Uref, args.steps)
        torch.cuda.synchronize()
        d = (U - Uref).abs().max().item() / Uref.abs().max().item()
        result["rel_err_vs_fp64"] = d
        ref_plan.close()
    if p.g == "cubic_nls":
        # Lawson-Euler with a unitary e^{tau A}: sum|U_{n+1}|^2 = sum|U_n|^2 (1 + tau^2 |U_n|^4)
        Um = U0.clone()
        worst = 0.0
        for _ in range(10):
            prev = Um.clone()
            plan.step(Um)
            torch.cuda.synchronize()
            a2 = prev.abs() ** 2
            lhs = (Um.abs() ** 2).sum().item()
            rhs = (a2 * (1 + p.tau ** 2 * a2 * a2)).sum().item()
            worst = max(worst, abs(lhs - rhs) / rhs)
        result["mass_identity_max_rel_residual_10_steps"] = worst
    if not args.no_cpu_baseline:
        base, oracle_state, k = oracle_sample(p, args.cpu_seconds)
        Ug = U0.clone()
        plan.run(Ug, k)
        torch.cuda.synchronize()
        base["gpu_vs_oracle_rel_inf"] = float(np.abs(px.tensor_from_device(Ug) - oracle_state).max()
                                              / np.abs(oracle_state).max())
        result["cpu_baseline"] = base
    plan.close()
    print(json.dumps(result))


def bench_kernel_only(args):
    """Only the roofline timing loop of one workload and precision (tucker_apply with the
    step's shapes): a short program for rocprofv3 PMC passes."""
    import torch
    import paper_2304_02327_amd as px
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p, _ = make_workload(args.workload)
    U0 = px.tensor_to_device(p.u0, device=dev)
    # the launch configurations a plan of this workload would use
    px.tucker_tune(list(p.n), px.C128 if p.is_complex else px.F64, args.precision)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    r = tucker_roofline(args, p, px, dev, stream, U0, args.precision, args.workload)
    print(json.dumps({"kernel_only": args.workload, "precision": args.precision,
                      "avg_launch_us": r["avg_launch_us"], "kernel_reps": args.kernel_reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own count, 20 for the 384^3 sweep, 100 for "
                         "adr128, the paper's step count for adr_paper*)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed graph-replayed steps before each timed region")
    ap.add_argument("--workload", default="dr384_sweep")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "slice"],
                    help="contraction precision of the mu-mode products for a single workload "
                         "(state and phi stay FP64); the default sweep runs all four")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched workloads: keep the default (or EXPINT_GROUPED) grouped tile scheme")
    ap.add_argument("--cpu-seconds", type=float, default=22.0)
    ap.add_argument("--kernel-only", action="store_true",
                    help="only time the dominant kernel of --workload/--precision (for PMC passes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 512 MiB five times (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(sharding is described in the design notes only).", file=sys.stderr)
        sys.exit(2)
    if args.kernel_only:
        bench_kernel_only(args)
        return
    if args.workload in ("riccati64", "riccati64_ros"):
        if args.steps is None:
            args.steps = 20
        bench_riccati(args, "rosenbrock_euler" if args.workload == "riccati64_ros" else "etd2rk")
        return
    if args.workload == "dr384_sweep":
        bench_sweep(args)
        return
    bench_single(args)


def tucker_roofline(args, p, px, dev, stream, U0, precision, workload):
    """Roofline of the dominant kernel: the fused launch of modes 1 and 2 where the
    Tucker operator uses it (FP64 real data, n_2 <= 128), else the mu-mode product.
    tucker_apply with the shapes and launch configuration of the step (the phi_1
    Tucker), timed alone with HIP events on the stream it is launched on."""
    import torch
    ell = 1 if p.scheme in ("exp_euler", "etd2rk") else 0
    Ms = [px.matrix_to_device(px.phi_setup(a, p.tau, ell)[ell], device=dev) for a in p.A]
    Vk = U0.clone()
    Wk = torch.empty_like(Vk)
    prec_code = {"fp64": px.PREC_FP64, "fp32": px.PREC_FP32, "bf16x3": px.PREC_BF16X3,
                 "slice": px.PREC_SLICED}[precision]
    ws = torch.empty(max(px.tucker_workspace_size(p.n, px.C128 if p.is_complex else px.F64, prec_code), 16),
                     dtype=torch.uint8, device=dev)

    def time_per_call(mats):
        with torch.cuda.stream(stream):
            for _ in range(3):
                px.tucker_apply(mats, Vk, Wk, ws=ws, stream=stream, precision=prec_code)
        ms = _event_ms(stream, lambda: [px.tucker_apply(mats, Vk, Wk, ws=ws, stream=stream, precision=prec_code)
                                        for _ in range(args.kernel_reps)])
        return ms / 1e3 / args.kernel_reps

    dt_code = px.C128 if p.is_complex else px.F64
    fused12 = precision == "fp64" and px.tucker_fuses_modes12(p.n, dt_code, prec_code)
    esz = 16 if p.is_complex else 8
    if fused12:
        # the dominant kernel is the fused launch of modes 1 and 2 (M_3.. = identity:
        # one launch per call, storing plainly as inside the step)
        avg_launch_s = time_per_call(list(Ms[:2]) + [None] * (p.d - 2))
        flops_per_launch = 2 * p.N * (p.n[0] + p.n[1])
    else:
        avg_launch_s = time_per_call(Ms) / p.d
        flops_per_launch = sum((8 if p.is_complex else 2) * p.N * nm for nm in p.n) / p.d
    achieved_tf = flops_per_launch / avg_launch_s / 1e12
    traffic = measured_traffic(workload, precision)
    if fused12:
        alg_bytes = 2 * esz * p.N + esz * (p.n[0] ** 2 + p.n[1] ** 2)
        roofline = {
            "kernel": "k_modes12 (modes 1 and 2 of the Tucker operator in one launch, FP64 MFMA)",
            "bound": "mfma",
            "achieved": round(achieved_tf, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4),
            "traffic": traffic,
        }
        if p.d > 2:  # the remaining single-mode launches, timed alone beside it
            rest_s = time_per_call([None, None] + list(Ms[2:]))
            rest_flops = sum(2 * p.N * nm for nm in p.n[2:])
            roofline["other_kernels"] = {
                "k_mode_product (modes 3..d, one launch each)": {
                    "avg_launch_us": round(rest_s / (p.d - 2) * 1e6, 3),
                    "achieved_tflops": round(rest_flops / rest_s / 1e12, 3)}}
    elif precision == "fp64":
        alg_bytes = 2 * esz * p.N
        roofline = {
            "kernel": "k_mode_product (FP64 MFMA mu-mode product)",
            "bound": "mfma",
            "achieved": round(achieved_tf, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4),
            "traffic": traffic,
        }
    elif precision == "slice":
        # one mode of tucker_apply: digits of the tensor (read 8 B, write 5 B per element),
        # then the int8 GEMM (read 5 B, write 8 B per element); the digits of M are small
        alg_bytes = 26 * p.N
        hw_tops = SLICE_PRODUCTS * flops_per_launch / avg_launch_s / 1e12
        roofline = {"kernel": "k_slice_* + k_sliced_gemm (exact-slice mu-mode product, int8 MFMA)",
                    "bound": "mfma", "achieved": round(hw_tops, 2), "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                    "frac": round(hw_tops / PEAK_INT8_TOPS, 4), "traffic": traffic,
                    "algorithmic_tflops_fp64_equivalent": round(achieved_tf, 3),
                    "hardware_op_multiplier": SLICE_PRODUCTS}
    else:
        # a reduced-precision Tucker reads FP64, keeps FP32 intermediates, writes FP64:
        # d modes move (8 + 4) + (4 + 4) (d - 2) + (4 + 8) bytes per element in total
        tot = (12 + 8 * (p.d - 2) + 12) if p.d >= 2 else 16
        alg_bytes = tot * p.N / p.d
        gbs = alg_bytes / avg_launch_s / 1e9
        hw_mult = 1 if precision == "fp32" else 3
        peak_c = PEAK_FP32_TFLOPS if precision == "fp32" else PEAK_BF16_TFLOPS
        intensity = hw_mult * flops_per_launch / alg_bytes
        ridge = peak_c * 1e12 / (PEAK_HBM_GBS * 1e9)
        kname = "k_mode_product_f32" if precision == "fp32" else "k_mode_product_bf16x3"
        if intensity < ridge:
            roofline = {"kernel": f"{kname} ({precision} mu-mode product)",
                        "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic}
        else:
            hw_tf = hw_mult * achieved_tf
            roofline = {"kernel": f"{kname} ({precision} mu-mode product)",
                        "bound": "mfma", "achieved": round(hw_tf, 3), "peak": peak_c, "unit": "TFLOP/s",
                        "frac": round(hw_tf / peak_c, 4), "traffic": traffic}
        roofline["algorithmic_tflops_fp64_equivalent"] = round(achieved_tf, 3)
        roofline["hardware_flop_multiplier"] = hw_mult
    roofline.update({
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_bytes_per_launch": alg_bytes,
        "avg_launch_us": round(avg_launch_s * 1e6, 3),
        "flops_per_launch": flops_per_launch,
    })
    return roofline


def oracle_sample(p, budget_s):
    """The CPU FP64 oracle, timed on the host on a bounded sample of the same workload
    (its first k steps, k chosen for about budget_s seconds); returns the cpu_baseline
    record, the oracle's state after k steps and k."""
    import numpy as np
    from oracle import schemes
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t = time.perf_counter()
    integ = schemes.integrator_for(p)
    setup_s = time.perf_counter() - t
    U = np.array(p.u0)
    t = time.perf_counter()
    U = integ.step(U, 0.0)
    one = time.perf_counter() - t
    k = max(1, min(p.steps, int(math.ceil(budget_s / max(one, 1e-6)))))
    t = time.perf_counter()
    for i in range(1, k):
        U = integ.step(U, i * p.tau)
    total = one + time.perf_counter() - t
    out = {
        "value": p.N * k / total,
        "unit": "DOF-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {k} of {p.steps} steps of the same workload (oracle phi setup "
                  f"{setup_s:.2f} s excluded); host {os.cpu_count()} logical CPUs",
        "seconds": round(total, 3),
    }
    # the same oracle on one thread, over a shorter sample (about a third of the budget),
    # where one step fits in it
    try:
        from threadpoolctl import threadpool_limits
        if one * threads <= budget_s / 3:
            with threadpool_limits(limits=1):
                U1 = np.array(p.u0)
                t = time.perf_counter()
                U1 = integ.step(U1, 0.0)
                one1 = time.perf_counter() - t
                k1 = max(1, min(p.steps, int(math.ceil(budget_s / 3 / max(one1, 1e-6)))))
                t = time.perf_counter()
                for i in range(1, k1):
                    U1 = integ.step(U1, i * p.tau)
                total1 = one1 + time.perf_counter() - t
            out["single_thread"] = {"value": p.N * k1 / total1, "unit": "DOF-steps/s", "cores": 1,
                                    "sample": f"first {k1} of {p.steps} steps", "seconds": round(total1, 3)}
    except ImportError:
        pass
    return out, U, k


if __name__ == "__main__":
    main()
