#!/usr/bin/env python3
"""Throughput of the MI355X QAOA contraction on one GPU.

Workload (the headline configuration): one amplitude <0...0|U|+> of the p=2
QAOA MaxCut ansatz on a seeded random 3-regular graph with n=60 vertices,
step-dependent slicing over 8 variables (256 slices), min-fill orders,
(gamma, beta) drawn uniformly from [0, pi).  One step = one full amplitude:
gate tensors, the serial prefix, all 256 slices, the FP64 slice sum.

Reported beside the optimised complex64 path: the plain complex128 path
(one launch per bucket step per slice), the relative error of both against
the complex128 oracle, per-kernel-class HIP-event timings for the roofline,
and the oracle itself timed on the host.
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAOA amplitudes/s and edge-energies/s vs plain complex128 path at stated error"
HBM_PEAK_GBS = 8000.0


def build_plan(precision, slice_batch=0, plain=False, fold=False, graph=False):
    from paper_2012_02430_amd import api
    from paper_2012_02430_amd import network as N
    from workloads import regular_graph

    n, p, k = 60, 2, 8
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill")
    plan = api.Plan(net, sch.order, sch.groups, precision=precision, slice_batch=slice_batch, plain=plain,
                    fold_prefix=fold, graph=graph)
    return net, sch, plan, edges


def time_calls(plan, g_dev, b_dev, out_dev, stream, steps, warmup):
    import torch

    from paper_2012_02430_amd import _lib as L

    lib = L.load()
    for _ in range(warmup):
        L.check(lib.qt_contract_amplitude(plan.handle, g_dev.data_ptr(), b_dev.data_ptr(), out_dev.data_ptr(),
                                          stream.cuda_stream))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        L.check(lib.qt_contract_amplitude(plan.handle, g_dev.data_ptr(), b_dev.data_ptr(), out_dev.data_ptr(),
                                          stream.cuda_stream))
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(edges, g, b, sch, budget_s):
    """The oracle (numpy complex128, Algorithm 1 slice by slice) on the host."""
    import oracle

    T = oracle.amplitude_network(60, edges, g, b)
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.sliced_values(T, sch.order, sch.groups)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 30:
            break
    return reps / el, reps, el


def energy_bench(steps, warmup, cpu_seconds, waves=0):
    """Edge-energies/s on n=1000, p=3: 1500 lightcones x 32 points per evaluation."""
    import ctypes

    import numpy as np
    import torch

    import oracle
    from paper_2012_02430_amd import _lib as L
    from paper_2012_02430_amd import api, autotune
    from workloads import qaoa_params, regular_graph

    n, p, npt = 1000, 3, 32
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, npt, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    if waves:
        model.set_tuning(waves, 0)
        tuned = {"waves": waves}
    else:
        tuned = autotune.tune_energy(model, npt, repeats=3)
    lib = L.load()
    stream = torch.cuda.current_stream()
    gd = torch.tensor(gs, dtype=torch.float64, device="cuda")
    bd = torch.tensor(bs, dtype=torch.float64, device="cuda")
    Ed = torch.zeros(npt, dtype=torch.float64, device="cuda")

    def call():
        L.check(lib.qt_energy_grad(model._arr, len(edges), npt, gd.data_ptr(), bd.data_ptr(), Ed.data_ptr(), None,
                                   None, None, stream.cuda_stream))

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    rate = len(edges) * npt / el
    # accuracy on sampled edges against the oracle
    E, pe = model.energy(gs, bs, per_edge=True)
    rng = np.random.default_rng(0)
    err = 0.0
    for i in (0, 31):
        for e in rng.choice(len(edges), 4, replace=False):
            u, v = edges[e]
            err = max(err, abs(pe[i, e] - oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real))
    # plain complex128 path on a sample of lightcones: one launch per bucket step
    sample = list(rng.choice(len(edges), 8, replace=False))
    plain = [api.Plan(model.networks[e], model.plans[e].order, precision="c128", plain=True, slice_batch=1)
             for e in sample]
    for pl in plain:
        pl.contract_amplitude(gs[0], bs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl in plain:
        pl.contract_amplitude(gs[0], bs[0])
    plain_rate = len(plain) / (time.perf_counter() - t0)
    # the oracle on the host, same sample of lightcones
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < cpu_seconds:
        u, v = edges[sample[done % len(sample)]]
        oracle.edge_energy(n, edges, gs[0], bs[0], u, v)
        done += 1
    cpu_rate = done / (time.perf_counter() - t0)
    # roofline of the lightcone launch: algorithmic bytes = sum over lightcones of their steps'
    # 8 B x (inputs + output) elements, per point
    alg = sum(pl.info().prefix_bytes for pl in model.plans) * npt
    roof = {"bound": "hbm", "kernel": "k_lds_multi (whole evaluation)", "achieved": alg / el / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / el / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": alg, "traffic": None}
    return {
        "metric": "edge-energies/s",
        "roofline": roof,
        "workload": "QAOA p=3 MaxCut energy, seeded random 3-regular graph n=1000: 1500 per-edge lightcone "
                    "networks x 32 seeded points per evaluation, one batched launch, complex64, FP64 edge sums",
        "value": rate,
        "ms_per_evaluation": 1e3 * el,
        "tuned_waves": tuned["waves"],
        "max_abs_err_vs_oracle_sampled": err,
        "plain_c128": {"value": plain_rate, "unit": "edge-energies/s",
                       "sample": f"{len(plain)} lightcones, one launch per bucket step"},
        "speedup_vs_plain_c128": rate / plain_rate,
        "cpu_oracle": {"value": cpu_rate, "unit": "edge-energies/s", "cores": 1,
                       "sample": f"{done} lightcone contractions in {cpu_seconds:.0f} s"},
    }


def gradient_bench(steps, warmup, cpu_seconds, grad_waves=0, multi_waves=0):
    """Edge-gradients/s on n=200, p=2: energy and dE/dgamma, dE/dbeta over
    300 lightcones x 64 points per evaluation (forward + adjoint, one launch)."""
    import numpy as np
    import torch

    import oracle
    from paper_2012_02430_amd import api, autotune
    from workloads import qaoa_params, regular_graph

    n, p, npt = 200, 2, 64
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, npt, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    if grad_waves:
        model.set_tuning(multi_waves, grad_waves)
        tuned = {"waves": grad_waves}
    else:
        tuned = autotune.tune_energy(model, npt, grad=True, repeats=3)
        autotune.tune_energy(model, npt, grad=False, repeats=3)
    gd = torch.tensor(gs, dtype=torch.float64, device="cuda")
    bd = torch.tensor(bs, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        model.energy_device(gd, bd, grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        model.energy_device(gd, bd, grad=True)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    # forward-only launch on the same workload, for the adjoint's cost
    for _ in range(warmup):
        model.energy_device(gd, bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        model.energy_device(gd, bd)
    torch.cuda.synchronize()
    el_fwd = (time.perf_counter() - t0) / steps
    E, dg, db = model.energy(gs, bs, grad=True)
    err = 0.0
    for i in (0, 63):
        Eo, dgo, dbo, pe, peg = oracle.energy_grad(n, edges, gs[i], bs[i])
        scale = np.abs(pe).sum() + np.abs(peg).sum(axis=0)
        err = max(err, float((np.abs(np.concatenate([dg[i], db[i]]) - np.concatenate([dgo, dbo])) / scale).max()))
    # the oracle on the host (forward-mode tangents), a sample of lightcones
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < cpu_seconds:
        u, v = edges[done % len(edges)]
        oracle.edge_energy_grad(n, edges, gs[0], bs[0], u, v)
        done += 1
    cpu_rate = done / (time.perf_counter() - t0)
    alg = sum(pl.info().prefix_bytes for pl in model.plans) * npt
    roof = {"bound": "hbm", "kernel": "k_lds_grad (whole evaluation)",
            "achieved": alg / el / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg / el / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": alg,
            "note": "forward-step bytes only (a lower bound of the adjoint's)", "traffic": None}
    return {
        "metric": "edge-gradients/s",
        "roofline": roof,
        "workload": "dE/dgamma, dE/dbeta of QAOA p=2 MaxCut energy, seeded random 3-regular graph n=200: 300 "
                    "lightcone networks x 64 seeded points per evaluation, forward + adjoint in one launch, "
                    "complex64, FP64 reductions",
        "value": len(edges) * npt / el,
        "ms_per_evaluation": 1e3 * el,
        "ms_forward_only": 1e3 * el_fwd,
        "tuned_waves": tuned["waves"],
        "max_err_vs_oracle_sampled": err,
        "err_scale": "sum_e |<C_e>| + |d<C_e>/dtheta|",
        "cpu_oracle": {"value": cpu_rate, "unit": "edge-gradients/s", "cores": 1,
                       "sample": f"{done} lightcone value+tangent contractions in {cpu_seconds:.0f} s"},
    }


def mfma_bench():
    """QAOA p=1 amplitude on n=210: the 256 slices of an 8-variable step-dependent slicing plan
    (min-degree order), fused GEMM buckets on MFMA vs the same plan unfused, and the plain path."""
    import numpy as np
    import torch

    from paper_2012_02430_amd import api
    from paper_2012_02430_amd import network as N
    from workloads import qaoa_params, regular_graph

    n, p, k = 210, 1, 8
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_degree")
    g, b = qaoa_params(p, 1, seed=1)
    fused = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32")
    unfused = api.Plan(net, sch.order, sch.groups, precision="c64")
    plain = api.Plan(net, sch.order, sch.groups, precision="c128", plain=True, slice_batch=1)

    def timed(plan, s1):
        plan.contract_batch(g, b, 0, min(s1, 8))
        torch.cuda.synchronize()
        t = time.perf_counter()
        vals, per = plan.contract_batch(g, b, 0, s1, per_slice=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t, vals, per

    el_f, _, per_f = timed(fused, 256)
    fused.profile_enable(True)
    fused.contract_batch(g, b, 0, 256)
    prof = fused.profile_read()
    fused.profile_enable(False)
    el_u, _, per_u = timed(unfused, 256)
    el_p, _, per_p = timed(plain, 4)
    err = float(np.max(np.abs(per_f[0, :4] - per_p[0]) / np.abs(per_p[0])))
    err_u = float(np.max(np.abs(per_u[0, :4] - per_p[0]) / np.abs(per_p[0])))
    gemm = prof.get("gemm", (0, 0.0, 0.0, 0.0))
    st = prof.get("step_stream", (0, 0.0, 0.0, 0.0))
    stream_gbs = st[2] / st[1] / 1e6 if st[1] else 0.0
    gemms = [s for s in fused.describe()["stream_steps"] if "gemm" in s]
    return {
        "metric": "slices/s",
        "workload": "QAOA p=1 single amplitude, seeded random 3-regular graph n=210 (315 edges): 256 slices of a "
                    "step-dependent slicing plan over 8 variables (min-degree order), complex64 with power-of-two "
                    "scaling, FP64 slice sum",
        "value": 256 / el_f,
        "s_per_256_slices": el_f,
        "width": {"fused": fused.info().width, "unfused": unfused.info().width},
        "gemm_buckets": [{"rank": s["rank"], "k_bits": s["gemm"]["k_bits"], "gflop_per_slice": s["gemm"]["flops"] / 1e9}
                         for s in gemms],
        "gemm_kernel": {"launches": gemm[0], "ms": gemm[1], "TFLOP/s": gemm[3] / gemm[1] / 1e9 if gemm[1] else 0,
                        "GB/s": gemm[2] / gemm[1] / 1e6 if gemm[1] else 0, "peak_TFLOP/s": 157.3},
        "roofline": {
            "gemm": {"bound": "mfma", "achieved": gemm[3] / gemm[1] / 1e9 if gemm[1] else 0, "peak": 157.3,
                     "unit": "TFLOP/s", "frac": (gemm[3] / gemm[1] / 1e9 / 157.3) if gemm[1] else 0,
                     "hbm_GB/s": gemm[2] / gemm[1] / 1e6 if gemm[1] else 0, "traffic": None},
            "streaming": {"bound": "hbm", "achieved": stream_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": stream_gbs / HBM_PEAK_GBS, "traffic": None},
        },
        "kernel_classes_ms": {k: round(v[1], 2) for k, v in prof.items()},
        "unfused_c64": {"value": 256 / el_u, "unit": "slices/s"},
        "plain_c128": {"value": 4 / el_p, "unit": "slices/s", "sample": "slices 0-3"},
        "speedup_vs_unfused": el_u / el_f,
        "speedup_vs_plain_c128": (4 / el_p) and (256 / el_f) / (4 / el_p),
        "max_rel_err_vs_c128_slices_0_3": {"fused": err, "unfused": err_u},
    }


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "lds_exec_qaoa_n60_p2_256slices.md")


def measured_traffic(tuning):
    """HBM bytes per launch of the LDS executor on this workload, from the committed FETCH_SIZE/WRITE_SIZE
    measurement, while the kernel sources and launch shape are those it was taken with (else None)."""
    import hashlib

    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^- (\w+): `([^`]*)`", text, re.M))
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2012_02430_amd", "csrc")
    h = hashlib.sha1()
    for f in ("lds_exec.hip", "qt_internal.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    if fields.get("source_sha1") != h.hexdigest():
        return None
    if fields.get("tuning") != f"{tuning['lds_waves']}/{tuning['lds_max_rank']}":
        return None
    return float(fields["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true", help="amplitude section only")
    ap.add_argument("--sections", default="amp,energy,gradient,mfma",
                    help="comma list of amp (the headline line), energy, gradient, mfma")
    ap.add_argument("--lds-waves", type=int, default=0, help="fix the LDS executor launch shape (skips tuning)")
    ap.add_argument("--lds-max-rank", type=int, default=0)
    ap.add_argument("--multi-waves", type=int, default=0, help="fix the lightcone launch shape (skips tuning)")
    ap.add_argument("--grad-waves", type=int, default=0)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="program for rocprofv3 --pmc: a 256 MiB device copy (counter calibration), then 5 "
                         "amplitudes of the headline workload at the given launch shape; prints no JSON")
    args = ap.parse_args()
    sections = set(args.sections.split(","))
    if args.no_energy:
        sections = {"amp"}
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (multi-GPU sharding is "
              "described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_2012_02430_amd import api, autotune
    from workloads import qaoa_params

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    g, b = qaoa_params(2, 1, seed=1)
    g, b = g[0], b[0]

    net, sch, plan, edges = build_plan("c64", fold=True)
    if args.traffic_probe:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        plan.set_tuning(args.lds_waves, args.lds_max_rank)
        gd = torch.tensor(g, dtype=torch.float64, device="cuda")
        bd = torch.tensor(b, dtype=torch.float64, device="cuda")
        time_calls(plan, gd, bd, torch.zeros(3, dtype=torch.float64, device="cuda"), stream, 5, 1)
        print(f"[bench] traffic probe done: tuning {plan.get_tuning()}", flush=True)
        return
    _, _, plain, _ = build_plan("c128", slice_batch=1, plain=True)
    print(f"[bench] plan: width {sch.width} (prefix {sch.prefix_width}, slice {sch.slice_width}), "
          f"unsliced {sch.unsliced_width}, step {sch.step}, 256 slices", flush=True)
    # measured launch shape (untimed; cached by shape signature), or the one given
    if args.lds_waves or args.lds_max_rank:
        plan.set_tuning(args.lds_waves, args.lds_max_rank)
        tuning = dict(plan.get_tuning(), cached=False, ms=float("nan"))
    else:
        tuning = autotune.tune_plan(plan, n_points=1, repeats=3)
    print(f"[bench] tuned: lds_waves {tuning['lds_waves']}, lds_max_rank {tuning['lds_max_rank']} "
          f"({'cached' if tuning['cached'] else 'measured'}: {tuning['ms']:.3f} ms)", flush=True)

    # accuracy against the oracle
    want = complex(oracle.sliced_values(oracle.amplitude_network(60, edges, g, b), sch.order, sch.groups).sum())
    got = plan.contract_amplitude(g, b)
    got_plain = plain.contract_amplitude(g, b)
    err = abs(got - want) / abs(want)
    err_plain = abs(got_plain - want) / abs(want)
    per = oracle.sliced_values(oracle.amplitude_network(60, edges, g, b), sch.order, sch.groups)
    cond = float(np.abs(per).sum() / abs(per.sum()))
    print(f"[bench] amplitude {got:.10e}  oracle {want:.10e}  rel err c64 {err:.2e}  c128 {err_plain:.2e}",
          flush=True)

    g_dev = torch.tensor(g, dtype=torch.float64, device="cuda")
    b_dev = torch.tensor(b, dtype=torch.float64, device="cuda")
    out_dev = torch.zeros(3, dtype=torch.float64, device="cuda")

    el = time_calls(plan, g_dev, b_dev, out_dev, stream, args.steps, args.warmup)
    value = args.steps / el
    print(f"[bench] c64 path: {value:.1f} amplitudes/s ({1e3 * el / args.steps:.3f} ms each)", flush=True)
    el_plain = time_calls(plain, g_dev, b_dev, out_dev, stream, args.plain_steps, 1)
    plain_value = args.plain_steps / el_plain
    print(f"[bench] plain c128 path: {plain_value:.2f} amplitudes/s", flush=True)

    # the same contraction replayed from a captured graph (device-resident inputs and outputs)
    _, _, gplan, _ = build_plan("c64", fold=True, graph=True)
    gplan.set_tuning(tuning["lds_waves"], tuning["lds_max_rank"])
    g2 = g_dev.reshape(1, -1)
    b2 = b_dev.reshape(1, -1)
    o2 = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
    for _ in range(max(1, args.warmup)):
        gplan.contract_device(g2, b2, o2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gplan.contract_device(g2, b2, o2)
    torch.cuda.synchronize()
    graph_value = args.steps / (time.perf_counter() - t0)
    graph_err = abs(api.amp_to_complex(*o2[0].tolist()) - want) / abs(want)
    print(f"[bench] graph replay: {graph_value:.1f} amplitudes/s, rel err {graph_err:.2e}", flush=True)

    # per-kernel-class HIP-event timings over the same number of steps
    plan.profile_enable(True)
    time_calls(plan, g_dev, b_dev, out_dev, stream, args.steps, 0)
    prof = plan.profile_read(reset=True)
    plan.profile_enable(False)
    kernels = {k: {"launches": v[0], "ms": v[1], "avg_us": 1e3 * v[1] / v[0], "GB/s": v[2] / v[1] / 1e6 if v[1] else 0}
               for k, v in prof.items()}
    dom = max((k for k in prof if k != "other"), key=lambda k: prof[k][1])
    launches, ms, bytes_, flops = prof[dom]
    achieved = bytes_ / (ms * 1e-3) / 1e9
    print(f"[bench] dominant kernel class {dom}: {launches} launches, avg {1e3 * ms / launches:.2f} us, "
          f"{achieved:.1f} GB/s algorithmic", flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        rate, reps, cel = cpu_baseline(edges, g, b, sch, args.cpu_seconds)
        cpu = {"value": rate, "unit": "amplitudes/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full amplitudes (all 256 slices) of the same workload in {cel:.1f} s, "
                         "numpy complex128, single thread"}
        print(f"[bench] oracle on host: {rate:.3f} amplitudes/s", flush=True)

    energy = None
    if "energy" in sections:
        energy = energy_bench(max(5, args.steps // 5), 2, 3.0 if not args.no_cpu_baseline else 0.5, args.multi_waves)
        print(f"[bench] energy: {energy['value']:.3e} edge-energies/s ({energy['ms_per_evaluation']:.2f} ms per "
              f"1500x32 evaluation), plain c128 {energy['plain_c128']['value']:.1f}/s, "
              f"max abs err {energy['max_abs_err_vs_oracle_sampled']:.1e}", flush=True)

    gradient = None
    if "gradient" in sections:
        gradient = gradient_bench(max(5, args.steps // 5), 2, 3.0 if not args.no_cpu_baseline else 0.5,
                                  args.grad_waves, args.multi_waves)
        print(f"[bench] gradient: {gradient['value']:.3e} edge-gradients/s ({gradient['ms_per_evaluation']:.2f} ms "
              f"per 300x64 evaluation, forward only {gradient['ms_forward_only']:.2f} ms), "
              f"max rel err {gradient['max_err_vs_oracle_sampled']:.1e}", flush=True)

    mfma = None
    if "mfma" in sections:
        mfma = mfma_bench()
        print(f"[bench] n=210 fused GEMM plan: {mfma['value']:.1f} slices/s (unfused c64 "
              f"{mfma['unfused_c64']['value']:.1f}, plain c128 {mfma['plain_c128']['value']:.1f}); GEMM "
              f"{mfma['gemm_kernel']['TFLOP/s']:.1f} TFLOP/s; rel err {mfma['max_rel_err_vs_c128_slices_0_3']['fused']:.1e}",
              flush=True)

    inf = plan.info()
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "QAOA p=2 MaxCut single amplitude <0|U|+>, seeded random 3-regular graph n=60, "
                        "step-dependent slicing over 8 variables (256 slices), min-fill orders",
            "n": 60, "p": 2, "slice_vars": 8, "slices": 256, "points": 1,
            "precision": "complex64 mantissas + per-tensor power-of-two exponents, FP64 slice sum",
            "width": sch.width, "unsliced_width": sch.unsliced_width, "slice_step": sch.step,
        },
        "rel_err_vs_oracle": err,
        "condition_estimate": cond,
        "plain_c128": {"value": plain_value, "unit": "amplitudes/s", "rel_err_vs_oracle": err_plain,
                       "launches_per_amplitude": plain.info().n_launches},
        "speedup_vs_plain_c128": value / plain_value,
        "graph_replay": {"value": graph_value, "unit": "amplitudes/s", "rel_err_vs_oracle": graph_err},
        "launches_per_amplitude": inf.n_launches,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel_class": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(tuning) if dom == "lds" else None,
                     "algorithmic_bytes_per_launch": bytes_ / launches},
        "cpu_baseline": cpu,
        "tuning": {"lds_waves": tuning["lds_waves"], "lds_max_rank": tuning["lds_max_rank"]},
        "energy": energy,
        "gradient": gradient,
        "mfma_gemm": mfma,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
