#!/usr/bin/env python3
"""Throughput of the MI355X QAOA contraction on one GPU.

Headline workload: one amplitude <0...0|U|+> of the p=1 QAOA MaxCut ansatz
on a seeded random 3-regular graph with n=210 vertices (315 edges), a
step-dependent slicing plan over 8 variables (min-degree orders, 256
slices, per-slice width 28 with fused buckets), (gamma, beta) drawn
uniformly from [0, pi).  One step = one full amplitude: gate tensors, every
bucket step of all 256 slices (streaming steps, LDS segments and fused GEMM
buckets on the matrix cores), the per-slice scalars and the FP64 slice
sum, with parameters and result resident in device memory.

Reported beside it: the same plan unfused, the plain complex128 path (one
launch per bucket step per slice) and the error against it, the roofline of
the dominant kernel from HIP events over the timed region, and the oracle
on the host.  Side sections: the 60-qubit p=2 amplitude (256 slices), the
1000-node p=3 energy (1500 lightcones x 32 points), the 200-node p=2
gradient (300 lightcones x 64 points) and the 16-qubit latency case.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAOA amplitudes/s and edge-energies/s vs plain complex128 path at stated error"
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK_TF = 157.3       # dense FP32 matrix
VALU_FP32_PACKED_TF = 157.3     # 256 CUs x 2.4 GHz x 128 FMA/clk (two per lane with packed FP32)
VALU_FP32_TF = 78.6             # the same without packed FP32 (this library is built without it)
VALU_FP64_TF = 78.6             # 256 CUs x 2.4 GHz x 64 FMA/clk
CSRC = os.path.join(ROOT, "paper_2012_02430_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", flush=True)


def source_sha1(files):
    """sha1 of the sources a kernel is built from; "file:Struct" stands for that struct's definition only."""
    h = hashlib.sha1()
    for f in files:
        name, _, struct = f.partition(":")
        data = open(os.path.join(CSRC, name), "rb").read()
        if struct:
            i = data.index(f"struct {struct} {{".encode())
            data = data[i:data.index(b"\n};", i) + 3]
        h.update(data)
    return h.hexdigest()


def lds_schedule(plan):
    """The launch shape of a plan's LDS executor segments, as the profiles record it: wavefronts per
    workgroup, then per segment its steps, dependency levels and LDS bytes (tunings that give the same
    schedule run the same launches)."""
    d = plan.describe()
    return f"{plan.get_tuning()['lds_waves']}w:" + ",".join(
        f"{s['steps']}s{s['levels']}l{s['lds_bytes']}b" for s in d["segments"])


def measured_traffic(profile, files, **match):
    """HBM bytes per launch from a committed FETCH_SIZE/WRITE_SIZE summary, while the kernel sources (and
    the fields in `match`) are those the counters were taken with; else None."""
    try:
        text = open(os.path.join(PROFILES, profile)).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^- (\w+): `([^`]*)`", text, re.M))
    if fields.get("source_sha1") != source_sha1(files):
        return None
    for k, v in match.items():
        if fields.get(k) != str(v):
            return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_info():
    return {"nproc": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "OPENBLAS_NUM_THREADS": os.environ.get("OPENBLAS_NUM_THREADS")}


# ------------------------------------------------------------------ headline: n = 210
def c4_plans(tuning):
    from paper_2012_02430_amd import api
    from paper_2012_02430_amd import network as N
    from workloads import regular_graph

    n, p, k = 210, 1, 8
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_degree")
    fused = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32")
    if tuning:
        fused.set_tuning(*tuning)
    return net, sch, fused, edges


def time_amplitudes(plan, gd, bd, od, steps, warmup):
    import torch

    from paper_2012_02430_amd import _lib as L

    lib = L.load()
    s = torch.cuda.current_stream().cuda_stream
    for _ in range(warmup):
        L.check(lib.qt_contract_amplitude(plan.handle, gd.data_ptr(), bd.data_ptr(), od.data_ptr(), s))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        L.check(lib.qt_contract_amplitude(plan.handle, gd.data_ptr(), bd.data_ptr(), od.data_ptr(), s))
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def op_roofline(plan, ops, n_steps):
    """Roofline of the operation with the largest summed kernel time over the timed region."""
    desc = plan.describe()
    by_step = {s["step"]: s for s in desc["stream_steps"]}
    live = [o for o in ops if o["op"] >= 0]
    dom = max(live, key=lambda o: o["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    per_launch_bytes = dom["bytes"] / dom["launches"]
    per_launch_flops = dom["flops"] / dom["launches"]
    info = {"kclass": dom["kclass"], "op": dom["op"], "launches_per_step": dom["launches"] / n_steps,
            "avg_launch_ms": avg_ms, "share_of_kernel_time": dom["ms"] / sum(o["ms"] for o in ops)}
    if dom["kclass"] == "gemm":
        st = by_step[dom["op"]]
        kb = st["gemm"]["k_bits"]
        tile = st["gemm"]["tile"]
        mode = 1 if st["gemm"]["mode"].startswith("bf16") else 0
        name = f"k_gemm<{tile[0]}, {tile[1]}, {tile[2]}, {tile[3]}, {mode}>"
        traffic = measured_traffic(f"gemm_k{1 << kb}_qaoa_n210_p1.md", ["gemm.hip", "qt_internal.h:DevGemm"],
                                   kernel=name)
        achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": name, "achieved": achieved, "peak": MFMA_FP32_PEAK_TF,
                "unit": "TFLOP/s", "frac": achieved / MFMA_FP32_PEAK_TF, "traffic": traffic,
                "algorithmic_flops_per_launch": per_launch_flops,
                "algorithmic_bytes_per_launch": per_launch_bytes,
                "hbm_GB/s_algorithmic": per_launch_bytes / (avg_ms * 1e-3) / 1e9, "K": 1 << kb}
    else:
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": f"{dom['kclass']} op {dom['op']}", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": per_launch_bytes}
    roof.update(info)
    return roof


def c4_headline(args):
    import numpy as np
    import torch

    from paper_2012_02430_amd import api
    from workloads import qaoa_params

    net, sch, fused, edges = c4_plans(None)
    inf = fused.info()
    g, b = qaoa_params(1, 1, seed=1)
    log(f"n=210 plan: width {inf.width} fused (unfused {sch.width}), slice step {sch.step}, "
        f"{inf.n_slices} slices")
    gd = torch.tensor(g, dtype=torch.float64, device="cuda")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    od = torch.zeros(3, dtype=torch.float64, device="cuda")
    fused.profile_enable(True)
    time_amplitudes(fused, gd, bd, od, 0, args.warmup)
    fused.profile_read_ops(reset=True)  # drop the warm-up launches
    el = time_amplitudes(fused, gd, bd, od, args.steps, 0)
    ops = fused.profile_read_ops(reset=True)
    fused.profile_enable(False)
    value = args.steps / el
    got = api.amp_to_complex(*od.tolist())
    log(f"n=210 amplitude: {value:.3f} amplitudes/s ({1e3 * el / args.steps:.1f} ms each, "
        f"{value * inf.n_slices:.0f} slices/s)")
    roof = op_roofline(fused, ops, args.steps)
    log(f"dominant kernel {roof['kernel']}: {roof['avg_launch_ms']:.2f} ms per launch, {roof['achieved']:.1f} "
        f"{roof['unit']} ({100 * roof['frac']:.1f}% of {roof['peak']}), traffic {roof['traffic']}")
    kinds = {}
    for o in ops:
        k = kinds.setdefault(o["kclass"], {"launches_per_step": 0.0, "ms_per_step": 0.0, "bytes": 0.0,
                                           "flops": 0.0})
        k["launches_per_step"] += o["launches"] / args.steps
        k["ms_per_step"] += o["ms"] / args.steps
        k["bytes"] += o["bytes"]
        k["flops"] += o["flops"]
    for k in kinds.values():
        ms = k["ms_per_step"] * args.steps
        k["GB/s"] = k.pop("bytes") / ms / 1e6 if ms else 0.0
        k["TFLOP/s"] = k.pop("flops") / ms / 1e9 if ms else 0.0
    # error against the plain complex128 path (one launch per step per slice) over all 256 slices
    plain = api.Plan(net, sch.order, sch.groups, precision="c128", plain=True, slice_batch=1)
    t0 = time.perf_counter()
    want, per_plain = plain.contract_batch(g, b, per_slice=True)
    el_plain = time.perf_counter() - t0
    _, per_f = fused.contract_batch(g, b, per_slice=True)
    want = complex(want[0])
    err = abs(got - want) / abs(want)
    slice_err = float(np.abs(per_f[0] - per_plain[0]).max() / np.abs(per_plain[0]).max())
    cond = float(np.abs(per_plain[0]).sum() / abs(per_plain[0].sum()))
    log(f"rel err vs plain c128 path {err:.2e} (per slice {slice_err:.2e}, condition {cond:.2f}); "
        f"plain c128 {1 / el_plain:.4f} amplitudes/s")
    # the same plan unfused (complex64, no GEMM buckets)
    unfused = api.Plan(net, sch.order, sch.groups, precision="c64")
    unfused.contract_batch(g, b, 0, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    unfused.contract_batch(g, b)
    el_u = time.perf_counter() - t0
    return {
        "value": value, "el": el, "roofline": roof, "kernels": kinds, "amplitude": [got.real, got.imag],
        "rel_err_vs_plain_c128": err, "per_slice_rel_err_vs_plain_c128": slice_err, "condition_estimate": cond,
        "plain_c128": {"value": 1 / el_plain, "unit": "amplitudes/s",
                       "launches_per_amplitude": plain.info().n_launches},
        "speedup_vs_plain_c128": value * el_plain,
        "unfused_c64": {"value": 1 / el_u, "unit": "amplitudes/s", "width": sch.width},
        "launches_per_amplitude": fused.info().n_launches,
        "width": inf.width, "unsliced_width": sch.unsliced_width, "slice_step": sch.step,
        "slices": inf.n_slices,
        "gemm_buckets": [{"step": s["step"], "rank": s["rank"], "K": 1 << s["gemm"]["k_bits"],
                          "tile": s["gemm"]["tile"], "gflop_per_slice": s["gemm"]["flops"] / 1e9}
                         for s in fused.describe()["stream_steps"] if "gemm" in s],
        "edges": edges, "sch": sch, "g": g, "b": b,
    }


def c4_cpu_baseline(edges, g, b, sch):
    """The oracle on the host, on a bounded sample of the headline workload: the serial prefix and slice 0
    of the same plan (one slice takes about a minute and ~27 GB in numpy complex128), extrapolated to all
    of its slices."""
    import oracle
    from oracle.bucket import bucket_elimination, fix

    n = 210
    k = len(sch.slice_vars)
    T = oracle.amplitude_network(n, edges, g[0], b[0])
    t0 = time.perf_counter()
    rem, _ = bucket_elimination(T, sch.order[:sch.step])
    t_prefix = time.perf_counter() - t0
    t1 = time.perf_counter()
    sub = [fix(t, dict(zip(sch.slice_vars, [0] * k))) for t in rem]
    bucket_elimination(sub, sch.order[sch.step:])
    t_slice = time.perf_counter() - t1
    total = t_prefix + t_slice * (1 << k)
    return {"value": 1.0 / total, "unit": "amplitudes/s", "cores": 1, "kind": "oracle",
            "sample": f"extrapolated: serial prefix ({t_prefix:.2f} s) plus slice 0 of the same plan "
                      f"({t_slice:.1f} s, per-slice width {sch.slice_width}) times {1 << k} slices; "
                      "numpy complex128 on the host",
            "threads": cpu_info()}


# ------------------------------------------------------------------ 60-qubit amplitude
def c2_section(args):
    import numpy as np
    import torch

    import oracle
    from paper_2012_02430_amd import api, autotune
    from paper_2012_02430_amd import network as N
    from workloads import qaoa_params, regular_graph

    n, p, k = 60, 2, 8
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill")
    plan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=True)
    if args.lds_waves or args.lds_max_rank:
        plan.set_tuning(args.lds_waves, args.lds_max_rank)
        tuning = dict(plan.get_tuning(), cached=False, ms=float("nan"))
    else:
        tuning = autotune.tune_plan(plan, n_points=1, repeats=3)
    g, b = qaoa_params(p, 1, seed=1)
    gd = torch.tensor(g, dtype=torch.float64, device="cuda")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    od = torch.zeros(3, dtype=torch.float64, device="cuda")
    steps = max(20, 5 * args.steps)
    # the rate without per-operation events (a 120 us amplitude of five
    # launches pays for them), then the kernel's own duration from a
    # second, evented pass of as many amplitudes
    time_amplitudes(plan, gd, bd, od, 0, args.warmup)
    el = time_amplitudes(plan, gd, bd, od, steps, 0)
    plan.profile_enable(True)
    time_amplitudes(plan, gd, bd, od, 0, 1)
    plan.profile_read_ops(reset=True)  # drop the warm-up launches
    el_ev = time_amplitudes(plan, gd, bd, od, steps, 0)
    ops = plan.profile_read_ops(reset=True)
    plan.profile_enable(False)
    n_rec = steps
    lds = [o for o in ops if o["kclass"] == "lds"]
    lds_ms = sum(o["ms"] for o in lds) / n_rec
    lds_flops = sum(o["flops"] for o in lds) / n_rec
    lds_bytes = sum(o["bytes"] for o in lds) / n_rec
    value = steps / el
    per = oracle.sliced_values(oracle.amplitude_network(n, edges, g[0], b[0]), sch.order, sch.groups)
    want = complex(per.sum())
    err = abs(api.amp_to_complex(*od.tolist()) - want) / abs(want)
    plain = api.Plan(net, sch.order, sch.groups, precision="c128", plain=True, slice_batch=1)
    plain.contract_amplitude(g[0], b[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got_p = plain.contract_amplitude(g[0], b[0])
    el_p = time.perf_counter() - t0
    # graph replay of the same contraction
    gplan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=True, graph=True)
    gplan.set_tuning(tuning["lds_waves"], tuning["lds_max_rank"])
    o2 = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
    for _ in range(3):
        gplan.contract_device(gd, bd, o2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gplan.contract_device(gd, bd, o2)
    torch.cuda.synchronize()
    graph_value = steps / (time.perf_counter() - t0)
    tf = lds_flops / (lds_ms * 1e-3) / 1e12
    traffic = measured_traffic("lds_exec_qaoa_n60_p2_256slices.md", ["lds_exec.hip", "qt_internal.h"],
                               schedule=lds_schedule(plan))
    log(f"n=60 amplitude: {value:.0f} amplitudes/s ({steps / el_ev:.0f}/s with per-op events), "
        f"k_lds_exec {1e3 * lds_ms:.1f} us ({tf:.2f} TFLOP/s), "
        f"graph {graph_value:.0f}/s, plain c128 {1 / el_p:.1f}/s, rel err {err:.1e}")
    return {
        "metric": "amplitudes/s", "value": value, "ms_per_amplitude": 1e3 * el / steps,
        "with_per_op_events": {"value": steps / el_ev, "unit": "amplitudes/s"},
        "workload": "QAOA p=2 MaxCut single amplitude, seeded random 3-regular graph n=60, step-dependent slicing "
                    "over 8 variables (256 slices, min-fill orders), prefix folded into each slice, complex64 with "
                    "power-of-two scaling",
        "roofline": {"bound": "alu", "kernel": "k_lds_exec", "achieved": tf, "peak": VALU_FP32_TF,
                     "unit": "TFLOP/s", "frac": tf / VALU_FP32_TF, "frac_of_packed_peak": tf / VALU_FP32_PACKED_TF,
                     "avg_launch_us": 1e3 * lds_ms, "algorithmic_flops_per_launch": lds_flops,
                     "algorithmic_bytes_per_launch": lds_bytes, "traffic": traffic},
        "rel_err_vs_oracle": err, "condition_estimate": float(np.abs(per).sum() / abs(per.sum())),
        "plain_c128": {"value": 1 / el_p, "unit": "amplitudes/s", "rel_err_vs_oracle": abs(got_p - want) / abs(want)},
        "speedup_vs_plain_c128": value * el_p,
        "graph_replay": {"value": graph_value, "unit": "amplitudes/s"},
        "launches_per_amplitude": plan.info().n_launches,
        "tuning": {"lds_waves": tuning["lds_waves"], "lds_max_rank": tuning["lds_max_rank"]},
        "batch_of_amplitudes": open_outputs(args, n, p, k, edges),
        "parameter_batch": points_batch(args, plan, p),
    }


def points_batch(args, plan, p):
    """The same amplitude at 32 seeded (gamma, beta) points per call (one launch runs every point and
    slice): throughput once the single amplitude's dependency-chain latency is shared by many items."""
    import torch

    from workloads import qaoa_params

    npt = 32
    g, b = qaoa_params(p, npt, seed=2)
    gd = torch.tensor(g, dtype=torch.float64, device="cuda")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    od = torch.zeros(npt, 3, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup + 1):
        plan.contract_device(gd, bd, od)
    torch.cuda.synchronize()
    steps = max(10, 2 * args.steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.contract_device(gd, bd, od)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    log(f"n=60 amplitude at {npt} parameter points per call: {npt / el:.0f} amplitudes/s ({1e3 * el:.3f} ms per call)")
    return {"metric": "amplitudes/s", "value": npt / el, "points_per_call": npt, "ms_per_call": 1e3 * el}


def open_outputs(args, n, p, k, edges):
    """Several amplitudes from one contraction (Section VII): a qubits left open, 2^a amplitudes per
    contraction of the same 8-variable slicing plan (searched with the open variables excluded)."""
    import numpy as np
    import torch

    from paper_2012_02430_amd import api
    from paper_2012_02430_amd import network as N
    from workloads import qaoa_params

    out = {}
    for a in (4, 8):
        open_q = [int(q) for q in np.random.default_rng(a).choice(n, a, replace=False)]
        net = api.Network(N.amplitude_network(n, edges, p, open_qubits=open_q))
        ov = N.open_vars(n, p, open_q)
        sch = net.plan_slicing(k, algo="min_fill", exclude=ov)
        plan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=True, open_vars=ov)
        g, b = qaoa_params(p, 1, seed=1)
        gd = torch.tensor(g, dtype=torch.float64, device="cuda")
        bd = torch.tensor(b, dtype=torch.float64, device="cuda")
        od = torch.zeros((1 << a) * 3, dtype=torch.float64, device="cuda")
        steps = max(20, 5 * args.steps)
        el = time_amplitudes(plan, gd, bd, od, steps, args.warmup)
        got = od.view(-1, 3).cpu().numpy()
        amps = np.array([api.amp_to_complex(*row) for row in got])
        # one entry against the complex128 single amplitude of that bitstring (a plan of its own)
        j = 5
        z = np.zeros(n, dtype=np.uint8)
        for qi, q in enumerate(open_q):
            z[q] = (j >> (a - 1 - qi)) & 1
        full = api.Network(N.amplitude_network(n, edges, p, z))
        want = api.Plan(full, full.order_greedy("min_fill")[0], precision="c128").contract_amplitude(g[0], b[0])
        err = abs(amps[j] - want) / abs(want)
        rate = (1 << a) * steps / el
        log(f"n=60 batch of 2^{a} amplitudes: {rate:.0f} amplitudes/s ({1e3 * el / steps:.3f} ms per contraction), "
            f"entry {j} rel err {err:.1e}")
        out[f"a={a}"] = {"value": rate, "unit": "amplitudes/s", "ms_per_contraction": 1e3 * el / steps,
                         "amplitudes_per_contraction": 1 << a, "width": plan.info().width,
                         "rel_err_entry5_vs_c128_single_amplitude": err}
    return out


# ------------------------------------------------------------------ energy and gradient
def lightcone_flops(model, grad=False):
    """Algorithmic real flops of one point over every lightcone (forward steps)."""
    return sum(pl.info().prefix_flops for pl in model.plans)


def energy_section(args):
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
    if args.multi_waves:
        model.set_tuning(args.multi_waves, 0)
        waves, cap = args.multi_waves, 0
    else:
        tu = autotune.tune_energy(model, npt, repeats=7)
        waves, cap = tu["waves"], tu["lds_cap"]
    lib = L.load()
    gd = torch.tensor(gs, dtype=torch.float64, device="cuda")
    bd = torch.tensor(bs, dtype=torch.float64, device="cuda")
    Ed = torch.zeros(npt, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream

    def call():
        L.check(lib.qt_energy_grad(model._arr, len(edges), npt, gd.data_ptr(), bd.data_ptr(), Ed.data_ptr(), None,
                                   None, None, s))

    steps = max(10, 2 * args.steps)
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        call()
    ev1.record()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    gpu_ms = ev0.elapsed_time(ev1) / steps
    rate = len(edges) * npt / el
    E, pe = model.energy(gs, bs, per_edge=True)
    i = 7
    want = np.array([oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real for u, v in edges[:300]])
    err = float(np.abs(pe[i, :300] - want).max())
    flops = lightcone_flops(model) * npt
    tf = flops / (gpu_ms * 1e-3) / 1e12
    rng = np.random.default_rng(0)
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
    log(f"energy n=1000 p=3: {rate:.3e} edge-energies/s ({1e3 * el:.2f} ms per evaluation, stream time "
        f"{gpu_ms:.2f} ms, {tf:.2f} TFLOP/s), max abs err {err:.1e} (300 edges)")
    # the same evaluation with lightcones deduplicated up to isomorphism: one contraction per class,
    # weighted by the class size (reported apart: it skips the duplicate contractions)
    dd = api.EnergyModel(n, edges, p, precision="c64", dedup=True)
    dd.set_tuning(waves, 0, cap)
    for _ in range(args.warmup):
        dd.energy_device(gd, bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dd.energy_device(gd, bd)
    torch.cuda.synchronize()
    el_dd = (time.perf_counter() - t0) / steps
    E_dd = dd.energy(gs, bs)
    log(f"energy with dedup: {len(dd.plans)} lightcone classes of {len(edges)}, {npt / el_dd:.0f} energy "
        f"evaluations/s ({1e3 * el_dd:.3f} ms per 32-point evaluation)")
    return {
        "metric": "edge-energies/s", "value": rate, "ms_per_evaluation": 1e3 * el,
        "dedup": {"metric": "full-graph energies/s (points)", "value": npt / el_dd,
                  "ms_per_evaluation": 1e3 * el_dd, "lightcone_classes": len(dd.plans), "edges": len(edges),
                  "max_rel_diff_vs_all_edges": float(np.abs(E_dd - E).max() / np.abs(E).max()),
                  "note": "one contraction per isomorphism class of lightcones, weighted by class size"},
        "workload": "QAOA p=3 MaxCut energy, seeded random 3-regular graph n=1000: 1500 per-edge lightcone "
                    "networks x 32 seeded points per evaluation, complex64, FP64 edge sums",
        "roofline": {"bound": "alu", "kernel": "k_lds_multi (whole evaluation, stream time)", "achieved": tf,
                     "peak": VALU_FP32_TF, "unit": "TFLOP/s", "frac": tf / VALU_FP32_TF,
                     "frac_of_packed_peak": tf / VALU_FP32_PACKED_TF, "algorithmic_flops_per_evaluation": flops,
                     "traffic": None},
        "max_abs_err_vs_oracle": err, "err_sample": "300 edges at point 7",
        "waves": waves, "lds_cap": cap,
        "plain_c128": {"value": plain_rate, "unit": "edge-energies/s",
                       "sample": f"{len(plain)} lightcones, one launch per bucket step"},
        "speedup_vs_plain_c128": rate / plain_rate,
    }


def gradient_section(args):
    import numpy as np
    import torch

    import oracle
    from paper_2012_02430_amd import api, autotune
    from workloads import qaoa_params, regular_graph

    n, p, npt = 200, 2, 64
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, npt, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    if args.grad_waves:
        model.set_tuning(args.multi_waves, args.grad_waves)
        waves, cap = args.grad_waves, 0
    else:
        tu = autotune.tune_energy(model, npt, grad=True, repeats=7)
        waves, cap = tu["waves"], tu["lds_cap"]
        autotune.tune_energy(model, npt, grad=False, repeats=7)
    gd = torch.tensor(gs, dtype=torch.float64, device="cuda")
    bd = torch.tensor(bs, dtype=torch.float64, device="cuda")
    steps = max(10, 2 * args.steps)

    def timed(grad):
        for _ in range(args.warmup):
            model.energy_device(gd, bd, grad=grad)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(steps):
            model.energy_device(gd, bd, grad=grad)
        ev1.record()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, ev0.elapsed_time(ev1) / steps

    el, gpu_ms = timed(True)
    el_fwd, gpu_ms_fwd = timed(False)
    E, dg, db = model.energy(gs, bs, grad=True)
    errs = []
    for i in (0, 21, 42, 63):
        _, dgo, dbo, _, _ = oracle.energy_grad(n, edges, gs[i], bs[i])
        ref = np.concatenate([dgo, dbo])
        errs.append(float(np.linalg.norm(np.concatenate([dg[i], db[i]]) - ref) / np.linalg.norm(ref)))
    flops = lightcone_flops(model) * npt
    tf = flops / (gpu_ms * 1e-3) / 1e12
    log(f"gradient n=200 p=2: {len(edges) * npt / el:.3e} edge-gradients/s ({1e3 * el:.2f} ms per evaluation, "
        f"forward only {1e3 * el_fwd:.2f} ms), normwise err {max(errs):.1e}")
    # the same gradient with lightcones deduplicated up to isomorphism (reported apart: it skips the
    # duplicate contractions)
    dd = api.EnergyModel(n, edges, p, precision="c64", dedup=True)
    dd.set_tuning(0, waves, 0, cap)
    for _ in range(args.warmup):
        dd.energy_device(gd, bd, grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dd.energy_device(gd, bd, grad=True)
    torch.cuda.synchronize()
    el_dd = (time.perf_counter() - t0) / steps
    _, dg_dd, db_dd = dd.energy(gs, bs, grad=True)
    g_all, g_dd = np.concatenate([dg, db], axis=1), np.concatenate([dg_dd, db_dd], axis=1)
    dd_diff = float((np.linalg.norm(g_dd - g_all, axis=1) / np.linalg.norm(g_all, axis=1)).max())
    log(f"gradient with dedup: {len(dd.plans)} lightcone classes of {len(edges)}, {1e3 * el_dd:.3f} ms per "
        f"64-point evaluation, max normwise diff vs all edges {dd_diff:.1e}")
    return {
        "metric": "edge-gradients/s", "value": len(edges) * npt / el, "ms_per_evaluation": 1e3 * el,
        "ms_forward_only": 1e3 * el_fwd, "adjoint_to_forward_ratio": gpu_ms / gpu_ms_fwd,
        "workload": "dE/dgamma, dE/dbeta of QAOA p=2 MaxCut energy, seeded random 3-regular graph n=200: 300 "
                    "lightcone networks x 64 seeded points per evaluation, forward + adjoint in one launch in "
                    "complex128 (forward-only launch complex64), FP64 reductions",
        "roofline": {"bound": "alu", "kernel": "k_lds_grad (whole evaluation, stream time)", "achieved": tf,
                     "peak": VALU_FP64_TF, "unit": "TFLOP/s", "frac": tf / VALU_FP64_TF,
                     "flops": "forward-step flops only (a lower bound of the adjoint's)", "traffic": None},
        "max_normwise_rel_err_vs_oracle": max(errs), "err_sample": "points 0, 21, 42, 63",
        "waves": waves, "lds_cap": cap,
        "dedup": {"metric": "full-graph gradients/s (points)", "value": npt / el_dd, "ms_per_evaluation": 1e3 * el_dd,
                  "lightcone_classes": len(dd.plans), "edges": len(edges),
                  "max_normwise_diff_vs_all_edges": dd_diff,
                  "note": "one contraction per isomorphism class of lightcones, weighted by class size"},
    }


def c1_latency(args):
    import torch

    import oracle
    from paper_2012_02430_amd import api
    from paper_2012_02430_amd import network as N
    from workloads import qaoa_params, regular_graph

    n, p = 16, 1
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    order, _ = net.order_greedy("min_fill")
    plan = api.Plan(net, order, precision="c128")
    g, b = qaoa_params(p, 1, seed=1)
    gd = torch.tensor(g, dtype=torch.float64, device="cuda")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    od = torch.zeros(3, dtype=torch.float64, device="cuda")
    steps = 200
    el = time_amplitudes(plan, gd, bd, od, steps, 10)
    want = oracle.amplitude(n, edges, g[0], b[0])
    err = abs(api.amp_to_complex(*od.tolist()) - want) / abs(want)
    log(f"n=16 latency: {1e6 * el / steps:.1f} us per amplitude, rel err {err:.1e}")
    return {"metric": "us/amplitude", "value": 1e6 * el / steps, "higher_is_better": False,
            "workload": "QAOA p=1 single amplitude, seeded random 3-regular graph n=16, min-fill order, no "
                        "slicing, complex128", "rel_err_vs_oracle": err,
            "launches_per_amplitude": plan.info().n_launches}


def traffic_probe(args):
    """Program for rocprofv3 --pmc: a 256 MiB device copy (counter calibration), then a few amplitudes of
    the headline workload (or of the 60-qubit one with --sections c2)."""
    import torch

    from workloads import qaoa_params

    a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    if args.sections == "c2":
        from paper_2012_02430_amd import api
        from paper_2012_02430_amd import network as N
        from workloads import regular_graph

        edges = regular_graph(60, 3, 0)
        net = api.Network(N.amplitude_network(60, edges, 2))
        sch = net.plan_slicing(8, algo="min_fill")
        plan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=True)
        plan.set_tuning(args.lds_waves, args.lds_max_rank)
        g, b = qaoa_params(2, 1, seed=1)
    else:
        _, _, plan, _ = c4_plans(None)
        g, b = qaoa_params(1, 1, seed=1)
    gd = torch.tensor(g, dtype=torch.float64, device="cuda")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    time_amplitudes(plan, gd, bd, torch.zeros(3, dtype=torch.float64, device="cuda"), 3, 1)
    log("traffic probe done")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sections", default="c2,energy,gradient,c1",
                    help="comma list of side sections: c2, energy, gradient, c1 ('none' for the headline only)")
    ap.add_argument("--lds-waves", type=int, default=0, help="fix the n=60 LDS executor launch shape")
    ap.add_argument("--lds-max-rank", type=int, default=0)
    ap.add_argument("--multi-waves", type=int, default=0, help="fix the lightcone launch shape (skips tuning)")
    ap.add_argument("--grad-waves", type=int, default=0)
    ap.add_argument("--traffic-probe", action="store_true", help=traffic_probe.__doc__)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: this build runs on one GPU "
              "(DESIGN.md describes how the slices and lightcones would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.traffic_probe:
        traffic_probe(args)
        return
    sections = set() if args.sections == "none" else set(args.sections.split(","))
    head = c4_headline(args)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = c4_cpu_baseline(head["edges"], head["g"], head["b"], head["sch"])
        log(f"oracle on host: {cpu['value']:.3e} amplitudes/s ({cpu['sample']})")
    side = {}
    if "c2" in sections:
        side["c2_amplitude_n60"] = c2_section(args)
    if "energy" in sections:
        side["energy_n1000_p3"] = energy_section(args)
    if "gradient" in sections:
        side["gradient_n200_p2"] = gradient_section(args)
    if "c1" in sections:
        side["latency_n16"] = c1_latency(args)
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["el"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "QAOA p=1 MaxCut single amplitude <0|U|+>, seeded random 3-regular graph n=210 (315 "
                        "edges): all 256 slices of a step-dependent slicing plan over 8 variables (min-degree "
                        "orders), fused GEMM buckets on FP32 MFMA, complex64 with power-of-two scaling, FP64 "
                        "slice sum",
            "n": 210, "p": 1, "slice_vars": 8, "slices": head["slices"], "points": 1,
            "width": head["width"], "unsliced_width": head["unsliced_width"], "slice_step": head["slice_step"],
        },
        "rel_err_vs_plain_c128": head["rel_err_vs_plain_c128"],
        "per_slice_rel_err_vs_plain_c128": head["per_slice_rel_err_vs_plain_c128"],
        "condition_estimate": head["condition_estimate"],
        "slices_per_s": head["value"] * head["slices"],
        "plain_c128": head["plain_c128"],
        "speedup_vs_plain_c128": head["speedup_vs_plain_c128"],
        "unfused_c64": head["unfused_c64"],
        "launches_per_amplitude": head["launches_per_amplitude"],
        "gemm_buckets": head["gemm_buckets"],
        "kernels": head["kernels"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "paper_context": "one 210-qubit, 1785-gate amplitude on 1024 nodes of the Cray XC40 Theta (Xeon Phi); "
                         "not comparable hardware or precision",
    }
    line.update(side)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
