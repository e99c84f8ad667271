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
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAOA amplitudes/s and edge-energies/s vs plain complex128 path at stated error"
HBM_PEAK_GBS = 8000.0


def build_plan(precision, slice_batch=0, plain=False, fold=False):
    from paper_2012_02430_amd import api
    from paper_2012_02430_amd import network as N
    from workloads import regular_graph

    n, p, k = 60, 2, 8
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill")
    plan = api.Plan(net, sch.order, sch.groups, precision=precision, slice_batch=slice_batch, plain=plain,
                    fold_prefix=fold)
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


def energy_bench(steps, warmup, cpu_seconds):
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
    return {
        "metric": "edge-energies/s",
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


def gradient_bench(steps, warmup, cpu_seconds):
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
    return {
        "metric": "edge-gradients/s",
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    args = ap.parse_args()
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
    _, _, plain, _ = build_plan("c128", slice_batch=1, plain=True)
    print(f"[bench] plan: width {sch.width} (prefix {sch.prefix_width}, slice {sch.slice_width}), "
          f"unsliced {sch.unsliced_width}, step {sch.step}, 256 slices", flush=True)
    # measured launch shape (untimed; cached by shape signature)
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
    if not args.no_energy:
        energy = energy_bench(max(5, args.steps // 5), 2, 3.0 if not args.no_cpu_baseline else 0.5)
        print(f"[bench] energy: {energy['value']:.3e} edge-energies/s ({energy['ms_per_evaluation']:.2f} ms per "
              f"1500x32 evaluation), plain c128 {energy['plain_c128']['value']:.1f}/s, "
              f"max abs err {energy['max_abs_err_vs_oracle_sampled']:.1e}", flush=True)

    gradient = None
    if not args.no_energy:
        gradient = gradient_bench(max(5, args.steps // 5), 2, 3.0 if not args.no_cpu_baseline else 0.5)
        print(f"[bench] gradient: {gradient['value']:.3e} edge-gradients/s ({gradient['ms_per_evaluation']:.2f} ms "
              f"per 300x64 evaluation, forward only {gradient['ms_forward_only']:.2f} ms), "
              f"max rel err {gradient['max_err_vs_oracle_sampled']:.1e}", flush=True)

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
        "launches_per_amplitude": inf.n_launches,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel_class": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": cpu,
        "tuning": {"lds_waves": tuning["lds_waves"], "lds_max_rank": tuning["lds_max_rank"]},
        "energy": energy,
        "gradient": gradient,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
