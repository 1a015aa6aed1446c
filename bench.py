"""Benchmark: direction-split exponential integrator steps on one MI355X.

Default workload: 3-D advection-diffusion-reaction on 128^3, ETD2RK phisplit,
FP64, tau = 2e-3 (A_mu = 0.02 D2 + beta_mu D1, g = u^2 (1 - u)).  A "step" is
one full ETD2RK time step over the whole tensor (stage input with K u and g,
two Tucker operators with the fused stage combinations), replayed from a HIP
graph.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line with DOF-steps/s, the roofline of the dominant kernel
(the FP64 MFMA mu-mode product) and the CPU oracle timed on the host.
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
SLICE_PRODUCTS = 26        # digit products a_i b_j (i + j <= 6) per multiply-add of the exact-slice path
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_modes12_adr128_hbm_traffic.md")


TRAFFIC_SOURCES = ("paper_2304_02327_amd/csrc/modes12.hip", "paper_2304_02327_amd/csrc/mode_product.hip",
                   "paper_2304_02327_amd/csrc/tile_common.h",
                   "paper_2304_02327_amd/csrc/device_common.h", "paper_2304_02327_amd/csrc/internal.h",
                   "include/expint.h")


def kernel_sources_sha256() -> str:
    """SHA-256 over the sources the mu-mode product kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        h.update(rel.encode())
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary, or None when
    the workload differs or the kernel's sources changed since the counters were taken."""
    if workload != "adr128" or not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            fields[k] = v
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256():
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
    launches = (19 + batch_smax(insts, tau)) if ros else 10
    result = {
        "metric": METRIC, "value": N * args.steps / (gpu_ms / 1e3), "unit": "DOF-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": gpu_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"64 Riccati-type instances, n1,n2 ~ U{{32..512}}, {name} phisplit, FP64, tau=1e-3",
                   "dof": N, "graph": True, "launches_per_step": launches},
        "wall_s_timed_region": wall, "phi_setup_s": setup_s,
        "roofline": {"kernel": f"k_grouped_gemm ({launches} persistent FP64 MFMA launches per step)",
                     "bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "flops_per_step": flops, "avg_launch_us": round(gpu_ms * 1e3 / args.steps / launches, 3)},
    }
    if not args.no_cpu_baseline:
        from oracle import nonlinear, schemes
        from oracle.norms import rel_inf
        sample = list(range(0, 64, 8))  # 8 of the 64 instances
        k = 3
        t = time.perf_counter()
        integs = []
        for i in sample:
            x = insts[i]
            g = nonlinear.make_g("riccati", {"B": x.B, "C": x.C})
            if not ros:
                integs.append(schemes.Integrator([x.A1, x.A2], tau, "etd2rk", g))
        osetup = time.perf_counter() - t
        t = time.perf_counter()
        if ros:
            outs = [schemes.run_rosenbrock_euler_riccati(insts[i].U0, tau, k, insts[i].A1, insts[i].A2, insts[i].B,
                                                          insts[i].C) for i in sample]
        else:
            outs = [integ.run(insts[i].U0, 0.0, k) for integ, i in zip(integs, sample)]
        secs = time.perf_counter() - t
        Ug = U0.clone()
        batch.run(Ug, k)
        torch.cuda.synchronize()
        got = batch.state_from_device(Ug)
        err = max(rel_inf(got[i], o) for i, o in zip(sample, outs))
        dof = sum(insts[i].n1 * insts[i].n2 for i in sample)
        result["cpu_baseline"] = {"value": dof * k / secs, "unit": "DOF-steps/s", "cores": os.cpu_count(),
                                  "kind": "oracle", "sample": f"{k} steps of instances {sample} (oracle phi setup "
                                  f"{osetup:.1f} s excluded)", "seconds": round(secs, 3),
                                  "gpu_vs_oracle_rel_inf": err}
    batch.close()
    print(json.dumps(result))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 100; the paper's step count for adr_paper*)")
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed steps before the timed region (default 300: about 30 ms at 128^3, which "
                         "the clocks need to settle; with 20 the timed region ran 6%% slower than later repeats)")
    ap.add_argument("--workload", default="adr128")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "slice"],
                    help="contraction precision of the mu-mode products (state and phi stay FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=22.0)
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
    if args.workload in ("riccati64", "riccati64_ros"):
        if args.steps is None:
            args.steps = 20
        bench_riccati(args, "rosenbrock_euler" if args.workload == "riccati64_ros" else "etd2rk")
        return

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
    U = U0.clone()
    stream = torch.cuda.Stream()  # default priority
    stream.wait_stream(torch.cuda.current_stream())

    # warmup (includes the one-time graph capture)
    with torch.cuda.stream(stream):
        plan.run(U, args.warmup, t0=0.0, use_graph=True, stream=stream)
    stream.synchronize()
    U.copy_(U0)
    torch.cuda.synchronize()

    # timed region: exactly K graph-replayed steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    with torch.cuda.stream(stream):
        plan.run(U, args.steps, t0=0.0, use_graph=True, stream=stream)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / max(args.steps, 1)
    value = p.N * args.steps / (gpu_ms / 1e3)
    if not torch.isfinite(U).all():
        raise SystemExit("non-finite state after the timed region")

    # five more regions of K steps from the same start, after the timed one, for
    # the spread of the figure (the reported value is the timed region above)
    U_timed = U.clone()
    repeats = []
    for _ in range(5):
        U.copy_(U0)
        torch.cuda.synchronize()
        r0 = torch.cuda.Event(enable_timing=True)
        r1 = torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        with torch.cuda.stream(stream):
            plan.run(U, args.steps, t0=0.0, use_graph=True, stream=stream)
        r1.record(stream)
        stream.synchronize()
        repeats.append(r0.elapsed_time(r1) / max(args.steps, 1))

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
        roofline = tucker_roofline(args, p, px, dev, stream, U0)
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
                 ("c64 (state c128)" if p.is_complex else
                  {"fp32": "f32 (state f64)", "bf16x3": "bf16x3/f32acc (state f64)",
                   "slice": "int8 digits x6/int32 acc (state f64)"}[args.precision]),
        "data": "synthetic",
        "config": {"workload": desc, "n": list(p.n), "scheme": p.scheme, "tau": p.tau,
                   "precision": args.precision, "graph": True},
        "wall_s_timed_region": wall,
        "repeat_ms_per_step": [round(x, 5) for x in repeats],
        "median_ms_per_step_of_repeats": round(sorted(repeats)[len(repeats) // 2], 5),
        "repeats_bitwise_equal_to_timed_state": bool(torch.equal(U, U_timed)),
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
        result["cpu_baseline"] = cpu_baseline(p, plan, U0, args.cpu_seconds)
    plan.close()
    print(json.dumps(result))


def tucker_roofline(args, p, px, dev, stream, U0):
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
                 "slice": px.PREC_SLICED}[args.precision]
    ws = torch.empty(max(px.tucker_workspace_size(p.n, px.C128 if p.is_complex else px.F64, prec_code), 16),
                     dtype=torch.uint8, device=dev)
    def time_per_call(mats):
        with torch.cuda.stream(stream):
            for _ in range(3):
                px.tucker_apply(mats, Vk, Wk, ws=ws, stream=stream, precision=prec_code)
            k0 = torch.cuda.Event(enable_timing=True)
            k1 = torch.cuda.Event(enable_timing=True)
            k0.record(stream)
            for _ in range(args.kernel_reps):
                px.tucker_apply(mats, Vk, Wk, ws=ws, stream=stream, precision=prec_code)
            k1.record(stream)
        stream.synchronize()
        return k0.elapsed_time(k1) / 1e3 / args.kernel_reps

    dt_code = px.C128 if p.is_complex else px.F64
    fused12 = args.precision == "fp64" and px.tucker_fuses_modes12(p.n, dt_code, prec_code)
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
    if fused12:
        alg_bytes = 2 * esz * p.N + esz * (p.n[0] ** 2 + p.n[1] ** 2)
        roofline = {
            "kernel": "k_modes12 (modes 1 and 2 of the Tucker operator in one launch, FP64 MFMA)",
            "bound": "mfma",
            "achieved": round(achieved_tf, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4),
            "traffic": measured_traffic(args.workload),
        }
        if p.d > 2:  # the remaining single-mode launches, timed alone beside it
            rest_s = time_per_call([None, None] + list(Ms[2:]))
            rest_flops = sum(2 * p.N * nm for nm in p.n[2:])
            roofline["other_kernels"] = {
                "k_mode_product (modes 3..d, one launch each)": {
                    "avg_launch_us": round(rest_s / (p.d - 2) * 1e6, 3),
                    "achieved_tflops": round(rest_flops / rest_s / 1e12, 3)}}
    elif args.precision == "fp64":
        alg_bytes = 2 * esz * p.N
        roofline = {
            "kernel": "k_mode_product (FP64 MFMA mu-mode product)",
            "bound": "mfma",
            "achieved": round(achieved_tf, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4),
            "traffic": measured_traffic(args.workload),
        }
    elif args.precision == "slice":
        # one mode of tucker_apply: digits of M (n^2) and of the tensor (read 8 B, write
        # 6 B per element), then the int8 GEMM (read 6 B, write 8 B per element)
        alg_bytes = 28 * p.N
        hw_tops = SLICE_PRODUCTS * flops_per_launch / avg_launch_s / 1e12
        roofline = {"kernel": "k_slice_* + k_sliced_gemm (exact-slice mu-mode product, int8 MFMA)",
                    "bound": "mfma", "achieved": round(hw_tops, 2), "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                    "frac": round(hw_tops / PEAK_INT8_TOPS, 4), "traffic": None,
                    "algorithmic_tflops_fp64_equivalent": round(achieved_tf, 3),
                    "hardware_op_multiplier": SLICE_PRODUCTS}
    else:
        # a reduced-precision Tucker reads FP64, keeps FP32 intermediates, writes FP64:
        # d modes move (8 + 4) + (4 + 4) (d - 2) + (4 + 8) bytes per element in total
        tot = (12 + 8 * (p.d - 2) + 12) if p.d >= 2 else 16
        alg_bytes = tot * p.N / p.d
        gbs = alg_bytes / avg_launch_s / 1e9
        hw_mult = 1 if args.precision == "fp32" else 3
        peak_c = PEAK_FP32_TFLOPS if args.precision == "fp32" else PEAK_BF16_TFLOPS
        intensity = hw_mult * flops_per_launch / alg_bytes
        ridge = peak_c * 1e12 / (PEAK_HBM_GBS * 1e9)
        if intensity < ridge:
            roofline = {"kernel": f"k_mode_product_{args.precision} ({args.precision} mu-mode product)",
                        "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None}
        else:
            hw_tf = hw_mult * achieved_tf
            roofline = {"kernel": f"k_mode_product_{args.precision} ({args.precision} mu-mode product)",
                        "bound": "mfma", "achieved": round(hw_tf, 3), "peak": peak_c, "unit": "TFLOP/s",
                        "frac": round(hw_tf / peak_c, 4), "traffic": None}
        roofline["algorithmic_tflops_fp64_equivalent"] = round(achieved_tf, 3)
        roofline["hardware_flop_multiplier"] = hw_mult
    roofline.update({
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_bytes_per_launch": alg_bytes,
        "avg_launch_us": round(avg_launch_s * 1e6, 3),
        "flops_per_launch": flops_per_launch,
    })
    return roofline


def cpu_baseline(p, plan, U0, budget_s):
    """The CPU FP64 oracle, timed on the host on a bounded sample of the same workload;
    its state after the sample is also compared with the GPU's after as many steps."""
    import numpy as np
    import torch
    import paper_2304_02327_amd as px
    from oracle import schemes
    from oracle.norms import rel_inf
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
    rest = time.perf_counter() - t
    total = one + rest
    # the GPU state after the same k steps (direct launches)
    Ug = U0.clone()
    plan.run(Ug, k)
    torch.cuda.synchronize()
    err = rel_inf(px.tensor_from_device(Ug), U)
    out = {
        "value": p.N * k / total,
        "unit": "DOF-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {k} of {p.steps} steps of the same workload (oracle phi setup "
                  f"{setup_s:.2f} s excluded); host {os.cpu_count()} logical CPUs",
        "seconds": round(total, 3),
        "gpu_vs_oracle_rel_inf": err,
    }
    # the same oracle on one thread, over a shorter sample (about a third of the budget)
    try:
        from threadpoolctl import threadpool_limits
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
    return out


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--kernel-sources-sha256":
        print(kernel_sources_sha256())
    else:
        main()
