"""Parity of the HIP amplitude path with the oracle (through the C-ABI).

Tolerances (relative): 1e-12 for the complex128 path, 1e-5 for complex64
with power-of-two scaling.  Per-slice values are compared one by one.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from paper_2012_02430_amd import network as N
from workloads import generate_regular_graph, qaoa_params, random_bitstring, regular_graph

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def rel(a, b):
    return abs(a - b) / abs(b)


def slice_err(got, want):
    """Max over slices of |got - want| relative to the largest slice value."""
    return np.abs(np.asarray(got) - np.asarray(want)).max() / np.abs(want).max()


def build(n, p, edges, z=None, k=0, algo="min_fill", precision="c64", slice_batch=0, step=None, plain=False,
          fold=False):
    spec = N.amplitude_network(n, edges, p, z)
    net = api.Network(spec)
    if k == 0:
        order, _ = net.order_greedy(algo)
        groups = []
    else:
        sch = net.plan_slicing(k, algo=algo)
        order, groups = sch.order, sch.groups
        if step is not None:
            # force the slice step: prefix = first `step` of the unsliced
            # order, the rest reordered on the sliced graph
            full, _ = net.order_greedy(algo)
            sl = sch.slice_vars
            pre = [v for v in full if v not in sl][:step]
            rest, _ = net.order_greedy(algo, exclude=sl + pre)
            order, groups = pre + rest, [(step, sl)]
    return net, api.Plan(net, order, groups, precision=precision, slice_batch=slice_batch, plain=plain,
                         fold_prefix=fold)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_c1_amplitude(precision):
    # n=16, p=1, min-fill order, no slicing
    n, p = 16, 1
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 4, seed=1)
    for i in range(4):
        z = random_bitstring(n, i) if i else None
        net, plan = build(n, p, edges, z, precision=precision)
        got = plan.contract_amplitude(gs[i], bs[i])
        want = oracle.amplitude(n, edges, gs[i], bs[i], z)
        assert rel(got, want) < TOL[precision], (i, got, want)
        assert rel(got, oracle.amplitude_sv(n, edges, gs[i], bs[i], z)) < TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_c2_per_slice_parity(precision):
    # n=60, p=2, k=8 slice variables (256 slices), min-fill plan
    n, p, k = 60, 2, 8
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=1)
    net, plan = build(n, p, edges, k=k, precision=precision)
    sch_order, groups = plan.order, plan.groups
    total, per = plan.contract_batch(g, b, per_slice=True)
    T = oracle.amplitude_network(n, edges, g[0], b[0])
    want = oracle.sliced_values(T, sch_order, groups)
    assert per.shape == (1, 256)
    assert slice_err(per[0], want) < TOL[precision]
    assert rel(total[0], want.sum()) < TOL[precision]
    assert rel(plan.contract_amplitude(g[0], b[0]), want.sum()) < TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("k,step,slice_batch", [(1, None, 0), (3, 0, 0), (3, 10, 2), (5, "end", 0), (6, None, 1),
                                                (6, None, 16)])
def test_slicing_variants(precision, k, step, slice_batch):
    n, p = 20, 2
    edges = regular_graph(n, 3, 1)
    z = random_bitstring(n, 5)
    g, b = qaoa_params(p, 1, seed=k)
    spec = N.amplitude_network(n, edges, p, z)
    if step == "end":
        step = len(spec.variables()) - k
    net, plan = build(n, p, edges, z, k=k, precision=precision, slice_batch=slice_batch, step=step)
    total, per = plan.contract_batch(g, b, per_slice=True)
    want = oracle.sliced_values(oracle.amplitude_network(n, edges, g[0], b[0], z), plan.order, plan.groups)
    assert slice_err(per[0], want) < TOL[precision]
    assert rel(total[0], oracle.amplitude_sv(n, edges, g[0], b[0], z)) < TOL[precision]
    # a sub-range of slices sums to the oracle's partial sum
    if 2 ** k >= 4:
        lo, hi = 1, 2 ** k - 1
        part, per2 = plan.contract_batch(g, b, lo, hi, per_slice=True)
        assert rel(part[0], want[lo:hi].sum()) < TOL[precision]
        assert slice_err(per2[0], want[lo:hi]) < TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_many_points_batched(precision):
    n, p, k = 14, 3, 4
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 5, seed=9)
    net, plan = build(n, p, edges, k=k, precision=precision)
    vals, per = plan.contract_batch(gs, bs, per_slice=True)
    for i in range(5):
        assert rel(vals[i], oracle.amplitude_sv(n, edges, gs[i], bs[i])) < TOL[precision]


def _random_dense_network(rng, n_vars, n_tensors, max_rank, hub=None):
    spec = N.NetworkSpec(n_vars=n_vars, p=0)
    T = []
    for t in range(n_tensors):
        r = int(rng.integers(1, max_rank + 1))
        va = list(rng.choice(n_vars, r, replace=False))
        if hub is not None and t < 11 and hub not in va:
            va[0] = hub
        vals = (rng.standard_normal((2,) * len(va)) + 1j * rng.standard_normal((2,) * len(va))) * 0.7
        spec.tensors.append((L.QT_T_DENSE, 0, tuple(int(v) for v in va), vals))
        T.append((vals, tuple(int(v) for v in va)))
    used = set(v for _, va in T for v in va)
    return spec, T, used


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_networks(precision, seed):
    # arbitrary dense tensors, a variable shared by 11 tensors (bucket split
    # into product steps), and possibly disconnected pieces
    rng = np.random.default_rng(seed)
    spec, T, used = _random_dense_network(rng, 16, 24, 4, hub=3)
    net = api.Network(spec)
    order, _ = net.order_greedy("min_fill")
    want = oracle.contract(T, order)
    plan = api.Plan(net, order, precision=precision)
    assert rel(plan.contract_amplitude([], []), want) < TOL[precision]
    sch = net.plan_slicing(3, algo="min_degree")
    plan = api.Plan(net, sch.order, sch.groups, precision=precision, slice_batch=2)
    tot, per = plan.contract_batch([], [], per_slice=True)
    assert rel(tot, want) < TOL[precision]
    assert slice_err(per[0], oracle.sliced_values(T, sch.order, sch.groups)) < TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_disconnected_graph(precision):
    # two disjoint K4s: the amplitude factorises; buckets close to scalars
    k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    edges = k4 + [(a + 4, b + 4) for a, b in k4]
    g, b = [0.3, 1.2], [0.7, 0.1]
    want = oracle.amplitude_sv(8, edges, g, b)
    net, plan = build(8, 2, edges, precision=precision)
    assert rel(plan.contract_amplitude(g, b), want) < TOL[precision]
    net, plan = build(8, 2, edges, k=2, precision=precision)
    assert rel(plan.contract_amplitude(g, b), want) < TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("max_rank", ["4", "14"])
def test_fused_segments_match_streaming(precision, max_rank, monkeypatch):
    # LDS segments (steps up to the rank limit fused) against one launch per
    # step; both against the oracle per slice.  A low limit mixes segments
    # and streaming steps; a small LDS budget forces spills to global memory.
    n, p, k = 24, 3, 5
    edges = generate_regular_graph(n, 3, 2)
    g, b = qaoa_params(p, 1, seed=4)
    want = oracle.sliced_values(oracle.amplitude_network(n, edges, g[0], b[0]), *_plan_of(n, p, edges, k))
    monkeypatch.setenv("QT_LDS_MAX_RANK", max_rank)
    for budget in ("163840", "65536", "32768", "4096"):
        monkeypatch.setenv("QT_LDS_BYTES", budget)
        net, plan = build(n, p, edges, k=k, precision=precision)
        _, per = plan.contract_batch(g, b, per_slice=True)
        assert slice_err(per[0], want) < TOL[precision], budget
        _, again = plan.contract_batch(g, b, per_slice=True)
        assert np.array_equal(per, again), budget
    net, plain = build(n, p, edges, k=k, precision=precision, plain=True, slice_batch=1)
    _, per = plain.contract_batch(g, b, per_slice=True)
    assert slice_err(per[0], want) < TOL[precision]


def _plan_of(n, p, edges, k):
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill")
    return sch.order, sch.groups


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_fold_prefix(precision):
    # the prefix run inside every slice with the slice variables fixed gives
    # the same per-slice values as the prefix run once
    n, p, k = 60, 2, 8
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=1)
    net, plan = build(n, p, edges, k=k, precision=precision, fold=True)
    _, per = plan.contract_batch(g, b, per_slice=True)
    want = oracle.sliced_values(oracle.amplitude_network(n, edges, g[0], b[0]), plan.order, plan.groups)
    assert slice_err(per[0], want) < TOL[precision]
    n, p = 20, 3
    edges = regular_graph(n, 3, 1)
    z = random_bitstring(n, 7)
    gs, bs = qaoa_params(p, 3, seed=2)
    net, plan = build(n, p, edges, z, k=4, precision=precision, fold=True, slice_batch=4)
    vals, _ = plan.contract_batch(gs, bs)
    for i in range(3):
        assert rel(vals[i], oracle.amplitude_sv(n, edges, gs[i], bs[i], z)) < TOL[precision]


def test_bitwise_reproducible():
    n, p = 60, 2
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=1)
    net, plan = build(n, p, edges, k=8, precision="c64")
    a1, s1 = plan.contract_batch(g, b, per_slice=True)
    a2, s2 = plan.contract_batch(g, b, per_slice=True)
    assert a1[0] == a2[0] and np.array_equal(s1, s2)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_streaming_tile_groups_bitwise(precision, monkeypatch):
    # streaming steps with 1, 4 or 16 tiles of an item per workgroup run the
    # same arithmetic per element (and the same max per item): per-slice
    # values are bitwise equal, and match the oracle
    n, p, k = 32, 3, 4
    edges = generate_regular_graph(n, 3, 5)
    g, b = qaoa_params(p, 2, seed=6)
    monkeypatch.setenv("QT_LDS_MAX_RANK", "4")  # most steps stream (ranks up to 16)
    res = []
    for lg in ("0", "2", "4"):
        monkeypatch.setenv("QT_STEP_LG_TILES", lg)
        net, plan = build(n, p, edges, k=k, precision=precision)
        st = plan.describe()["stream_steps"]
        assert sum(s["rank"] >= 14 for s in st) >= 4
        # large steps with inputs indexed by no output bit (held on v and
        # slice variables only), which the kernel multiplies in once per item
        assert any(s["rank"] >= 10 and any(r == hv for r, hv in zip(s["in_ranks"], s["in_has_v"])) for s in st)
        res.append(plan.contract_batch(g, b, per_slice=True)[1])
    assert all(np.array_equal(res[0], r) for r in res[1:])
    for i in range(2):
        want = oracle.sliced_values(oracle.amplitude_network(n, edges, g[i], b[i]), plan.order, plan.groups)
        assert slice_err(res[0][i], want) < TOL[precision]


def test_fault_injection_and_resume(monkeypatch):
    n, p = 20, 2
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=2)
    net, plan = build(n, p, edges, k=4, precision="c64", slice_batch=4)
    full, per_full = plan.contract_batch(g, b, per_slice=True)
    monkeypatch.setenv("QT_FAULT_AFTER_SLICE", "6")
    with pytest.raises(L.QTError) as e:
        plan.contract_batch(g, b, per_slice=True)
    assert e.value.status == L.QT_EFAULT_INJECTED
    monkeypatch.delenv("QT_FAULT_AFTER_SLICE")
    # resume the missing range and combine the journal in slice order
    rest, per_rest = plan.contract_batch(g, b, 6, 16, per_slice=True)
    assert np.array_equal(per_rest[0], per_full[0][6:])


def test_invalid_slice_range():
    n, p = 10, 1
    edges = regular_graph(n, 3, 0)
    net, plan = build(n, p, edges, k=2, precision="c64")
    for lo, hi in [(0, 5), (3, 3), (-1, 2)]:
        with pytest.raises(L.QTError) as e:
            plan.contract_batch([0.1], [0.2], lo, hi)
        assert e.value.status == L.QT_EINVAL


@pytest.mark.parametrize("precision", ["c64"])
def test_invariants_210_qubits_full_size(precision):
    # configuration of the 210-qubit p=1 amplitude: min-degree plan, 8 slice
    # variables (256 slices).  beta = 0 gives exactly 2^{-105}; gamma = 0
    # gives e^{-i n beta} 2^{-105}.
    n, p = 210, 1
    edges = regular_graph(n, 3, 0)
    net, plan = build(n, p, edges, k=8, algo="min_degree", precision=precision)
    a = plan.contract_amplitude([0.83], [0.0])
    assert rel(a, 2.0 ** -105) < TOL[precision]
    a = plan.contract_amplitude([0.0], [0.41])
    assert rel(a, np.exp(-1j * n * 0.41) * 2.0 ** -105) < TOL[precision]


@pytest.mark.parametrize("precision", ["c64_mfma_fp32", "c64_mfma_bf16x3"])
def test_c4_fused_gemm_per_slice_parity(precision):
    # the 210-qubit, p = 1 amplitude plan (min-degree order, 8 slice
    # variables, 256 slices) with fused GEMM buckets on the matrix cores:
    # per-slice values of two slice ranges against the plain complex128 path
    # (one launch per step per slice) at random (gamma, beta).  The oracle
    # cannot hold a width-28 slice in host memory within a test's time, so
    # these slices are pinned transitively: the complex128 path is itself
    # pinned to the oracle on the 60-qubit plan and the smaller cases above.
    n, p = 210, 1
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(8, algo="min_degree")
    fused = api.Plan(net, sch.order, sch.groups, precision=precision)
    gem = sorted((s["gemm"]["k_bits"], s["gemm"]["mode"]) for s in fused.describe()["stream_steps"] if "gemm" in s)
    assert [k for k, _ in gem] == [4, 9], gem  # the K = 16 and K = 512 buckets
    if precision == "c64_mfma_bf16x3":
        assert gem[1][1] == "bf16x3_3m" and gem[0][1] == "fp32_4m"
    plain = api.Plan(net, sch.order, sch.groups, precision="c128", slice_batch=1, plain=True)
    g, b = qaoa_params(p, 1, seed=11)
    for lo, hi in ((0, 2), (181, 183)):
        _, got = fused.contract_batch(g, b, lo, hi, per_slice=True)
        _, want = plain.contract_batch(g, b, lo, hi, per_slice=True)
        err = np.abs(got[0] - want[0]).max() / np.abs(want[0]).max()
        print(f"n=210 {precision} slices [{lo},{hi}): max rel err {err:.2e}", flush=True)
        assert err < TOL["c64"], (lo, err)


def _open_case(n, p, a, seed):
    edges = regular_graph(n, 3, 0)
    rng = np.random.default_rng(seed)
    open_q = [int(q) for q in rng.choice(n, a, replace=False)]
    net = api.Network(N.amplitude_network(n, edges, p, open_qubits=open_q))
    return edges, open_q, net, N.open_vars(n, p, open_q)


def _oracle_open_network(n, edges, g, b, open_q, p):
    opened = {oracle.ket_var(n, q, p) for q in open_q}
    return [t for t in oracle.amplitude_network(n, edges, g, b) if not (len(t[1]) == 1 and t[1][0] in opened)]


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("a", [4, 8])
def test_c2_open_outputs_per_slice_parity(precision, a):
    # a batch of 2^a amplitudes (Section VII) from one contraction of the
    # 60-qubit, p = 2 plan with 256 slices: the open qubits' last variables
    # are held; every per-slice output tensor against the oracle's
    n, p, k = 60, 2, 8
    edges, open_q, net, ov = _open_case(n, p, a, seed=a)
    sch = net.plan_slicing(k, algo="min_fill", exclude=ov)
    plan = api.Plan(net, sch.order, sch.groups, precision=precision, open_vars=ov)
    assert plan.info().n_open == a
    g, b = qaoa_params(p, 2, seed=20 + a)
    tot, per = plan.contract_batch(g, b, per_slice=True)
    assert tot.shape == (2, 1 << a) and per.shape == (2, 1 << a, 256)
    for i in range(2):
        T = _oracle_open_network(n, edges, g[i], b[i], open_q, p)
        want = oracle.sliced_values(T, sch.order, sch.groups, open_vars=ov)  # [slice][j]
        assert slice_err(per[i].T, want) < TOL[precision]
        ws = want.sum(axis=0)
        assert np.abs(tot[i] - ws).max() / np.abs(ws).max() < TOL[precision]
    # one entry against a plain amplitude of the same bitstring
    j = 5
    z = np.zeros(n, dtype=np.uint8)
    for q_i, q in enumerate(open_q):
        z[q] = (j >> (a - 1 - q_i)) & 1
    full = api.Network(N.amplitude_network(n, edges, p, z))
    order_z, _ = full.order_greedy("min_fill")
    single = api.Plan(full, order_z, precision="c128").contract_amplitude(g[0], b[0])
    assert abs(tot[0][j] - single) / abs(single) < TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("r", [4, 2])
def test_c2_slice_groups_per_slice_parity(precision, r):
    # Section VI-D with r < n: 8 slice variables in groups of r, each group
    # at its own step; per-slice values against the oracle's branched
    # schedule (group by group, first variable most significant)
    n, p, k = 60, 2, 8
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill", group_size=r)
    assert len(sch.groups) == k // r
    plan = api.Plan(net, sch.order, sch.groups, precision=precision)
    assert plan.info().n_groups == k // r
    g, b = qaoa_params(p, 1, seed=30 + r)
    tot, per = plan.contract_batch(g, b, per_slice=True)
    want = oracle.sliced_values(oracle.amplitude_network(n, edges, g[0], b[0]), sch.order, sch.groups)
    assert slice_err(per[0], want) < TOL[precision]
    assert rel(tot[0], want.sum()) < TOL[precision]


def test_c4_slice_groups_per_slice_parity():
    # the 210-qubit p = 1 amplitude with two groups of 4 slice variables
    # (each at its own step), fused GEMM buckets, against the plain
    # complex128 path on two slice ranges
    n, p = 210, 1
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(8, algo="min_degree", group_size=4)
    assert len(sch.groups) == 2 and sch.groups[0][0] < sch.groups[1][0]
    fused = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32")
    plain = api.Plan(net, sch.order, sch.groups, precision="c128", slice_batch=1, plain=True)
    g, b = qaoa_params(p, 1, seed=13)
    for lo, hi in ((0, 2), (77, 79)):
        _, got = fused.contract_batch(g, b, lo, hi, per_slice=True)
        _, want = plain.contract_batch(g, b, lo, hi, per_slice=True)
        err = np.abs(got[0] - want[0]).max() / np.abs(want[0]).max()
        print(f"n=210 two groups, slices [{lo},{hi}): max rel err {err:.2e}", flush=True)
        assert err < TOL["c64"], (lo, err)


@pytest.mark.parametrize("case", ["unsliced_c128", "sliced_fold_c64", "sliced_c64", "streaming_c64"])
def test_device_parameters_match_host_parameters(case, monkeypatch):
    """Parameters and results in device memory take their own route (the
    segments read device parameters where they are, or the leaf launch lays
    them out; the final or sum launch writes the results in place); every
    value equals the host-array route bit for bit, at several points."""
    import torch

    if case == "streaming_c64":
        monkeypatch.setenv("QT_LDS_MAX_RANK", "4")  # leaves read by streaming steps
    n, p = (16, 1) if case == "unsliced_c128" else (24, 2)
    edges = regular_graph(n, 3, 3)
    net = api.Network(N.amplitude_network(n, edges, p, random_bitstring(n, 4)))
    if case == "unsliced_c128":
        order, _ = net.order_greedy("min_fill")
        plan = api.Plan(net, order, precision="c128")
    else:
        sch = net.plan_slicing(3, algo="min_fill")
        plan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=case == "sliced_fold_c64")
    npt = 3
    gs, bs = qaoa_params(p, npt, seed=11)
    want, want_per = plan.contract_batch(gs, bs, per_slice=True)
    g = torch.tensor(np.asarray(gs).reshape(npt, p), dtype=torch.float64, device="cuda")
    b = torch.tensor(np.asarray(bs).reshape(npt, p), dtype=torch.float64, device="cuda")
    out = torch.zeros(npt, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(npt, plan.n_slices, 3, dtype=torch.float64, device="cuda")
    plan.contract_device(g, b, out, per)
    torch.cuda.synchronize()
    o, ps = out.cpu().numpy(), per.cpu().numpy()
    got = np.array([api.amp_to_complex(*o[i]) for i in range(npt)])
    got_per = np.vectorize(api.amp_to_complex)(ps[..., 0], ps[..., 1], ps[..., 2])
    assert np.array_equal(got, want)
    assert np.array_equal(got_per, want_per)


def test_single_point_sums_match_batched_points():
    """One point without open outputs has its slice sum formed inside the
    final launch (one workgroup), several points by the sum launch: the same
    arithmetic, so each point's amplitude is bit for bit the same either
    way, at one slice and at a range of slices."""
    n, p = 24, 2
    edges = regular_graph(n, 3, 7)
    net = api.Network(N.amplitude_network(n, edges, p, random_bitstring(n, 8)))
    sch = net.plan_slicing(4, algo="min_fill")
    plan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=True)
    gs, bs = qaoa_params(p, 3, seed=21)
    for lo, hi in ((0, plan.n_slices), (3, 4), (2, 11)):
        batch, _ = plan.contract_batch(gs, bs, lo, hi)
        for i in range(3):
            one, _ = plan.contract_batch(np.asarray(gs)[i:i + 1], np.asarray(bs)[i:i + 1], lo, hi)
            assert one[0] == batch[i], (lo, hi, i)
