"""Parity of fused GEMM buckets (QT_C64_SCALED_MFMA_FP32) with the oracle.

Dense random networks put two tensors A(b, m, K) and B(b, n, K) in the
bucket of the first summed variable, with their variables in random key
order (so every bit map of the kernel is exercised), vectors on the summed
variables (folded into A), vectors on the kept variables (so a transposed or
misplaced output element changes the final value) and rank-2 partners that
keep the batch variables out of the sum.  The oracle contracts the same
tensors by plain bucket elimination in complex128.  Tolerance 1e-5 relative
(complex64 path).
"""
import numpy as np
import pytest

import oracle
from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from paper_2012_02430_amd import network as N
from workloads import qaoa_params, regular_graph

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rand(rng, rank):
    return (rng.normal(size=(2,) * rank) + 1j * rng.normal(size=(2,) * rank)) / np.sqrt(2.0)


def dense_case(seed, nb, nm, nn, nk, n_slice=0):
    """(spec, oracle tensors, order, groups, names) of a network with one fusable bucket."""
    rng = np.random.default_rng(seed)
    K = list(range(nk))
    b = list(range(nk, nk + nb))
    m = list(range(nk + nb, nk + nb + nm))
    n = list(range(nk + nb + nm, nk + nb + nm + nn))
    tensors = []
    va = list(rng.permutation(b + m + K))
    vb = list(rng.permutation(b + n + K))
    tensors.append((_rand(rng, len(va)), tuple(int(x) for x in va)))
    tensors.append((_rand(rng, len(vb)), tuple(int(x) for x in vb)))
    for x in K[1:3] + b + m + n:  # vectors: two on summed variables, one on every kept one
        tensors.append((_rand(rng, 1), (x,)))
    for i, x in enumerate(b):  # batch variables stay kept
        tensors.append((_rand(rng, 2), (x, n[i % nn])))
    kept = b + m + n
    sl = [int(x) for x in rng.permutation(m)[:n_slice]]
    rest = [int(x) for x in rng.permutation([x for x in kept if x not in sl])]
    order = [K[0]] + [int(x) for x in rng.permutation(K[1:])] + rest
    spec = N.NetworkSpec(n_vars=nk + nb + nm + nn, p=0)
    for arr, vs in tensors:
        spec.tensors.append((L.QT_T_DENSE, 0, vs, arr))
    return spec, tensors, order, sl


def gemm_steps(plan):
    return [s for s in plan.describe()["stream_steps"] if "gemm" in s]


@pytest.mark.parametrize("seed,nb,nm,nn,nk", [(0, 0, 4, 4, 3), (1, 2, 5, 4, 5), (2, 1, 6, 5, 4), (3, 3, 4, 6, 6),
                                              (4, 2, 5, 5, 8)])
def test_dense_gemm_bucket(monkeypatch, seed, nb, nm, nn, nk):
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(seed, nb, nm, nn, nk)
    net = api.Network(spec)
    plan = api.Plan(net, order, precision="c64_mfma_fp32")
    g = gemm_steps(plan)
    assert len(g) == 1 and g[0]["gemm"]["k_bits"] == nk and g[0]["rank"] == nb + nm + nn
    got = plan.contract_amplitude([], [])
    want = oracle.contract(tensors, order)
    assert abs(got - want) / abs(want) < TOL, (got, want)


@pytest.mark.parametrize("step", [0, 1])
def test_dense_gemm_with_sliced_operands(monkeypatch, step):
    # step 0: the GEMM runs per slice on prefix leaves that hold the slice
    # variables; step 1: it runs in the unsliced prefix, slice variables kept
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, sl = dense_case(11 + step, 2, 6, 5, 5, n_slice=2)
    order = [x for x in order if x not in sl]
    net = api.Network(spec)
    groups = [(step, sl)]
    plan = api.Plan(net, order, groups, precision="c64_mfma_fp32")
    assert len(gemm_steps(plan)) == 1
    vals, per = plan.contract_batch([], [], per_slice=True)
    want = oracle.sliced_values(tensors, order, groups)
    scale = np.abs(want).max()
    assert np.abs(per[0] - want).max() / scale < TOL
    assert abs(vals[0] - want.sum()) / abs(want.sum()) < TOL


def test_qaoa_amplitude_with_gemm_bucket(monkeypatch):
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "8")
    n, p = 30, 2
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    order, _ = net.order_greedy("min_fill")
    plan = api.Plan(net, order, precision="c64_mfma_fp32")
    assert len(gemm_steps(plan)) == 1
    gs, bs = qaoa_params(p, 3, seed=4)
    for i in range(3):
        got = plan.contract_amplitude(gs[i], bs[i])
        want = oracle.amplitude(n, edges, gs[i], bs[i], order=order)
        assert abs(got - want) / abs(want) < TOL, (i, got, want)


def test_gemm_profile_class(monkeypatch):
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(5, 2, 5, 5, 6)
    plan = api.Plan(api.Network(spec), order, precision="c64_mfma_fp32")
    plan.profile_enable(True)
    plan.contract_amplitude([], [])
    prof = plan.profile_read()
    assert prof["gemm"][0] == 1 and prof["gemm"][3] == 8.0 * 2 ** (2 + 5 + 5 + 6)


@pytest.mark.parametrize("nk", [3, 4, 7])
@pytest.mark.parametrize("tiles", ["1", "2", "8", "64"])
def test_gemm_tile_ranges_bitwise(monkeypatch, tiles, nk):
    # a workgroup's range of tiles (n fastest, then m, inside one batch tile)
    # changes only which workgroup computes a tile: results are bitwise equal
    # to one tile per workgroup, on a bucket with several n and m tiles per
    # batch tile, with 8- and 16-deep single-stage tiles and 64-deep tiles of
    # two stages (the cross-tile prefetch path and the stage cursor's wrap)
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(21, 1, 7, 6, nk)
    plan = api.Plan(api.Network(spec), order, precision="c64_mfma_fp32")
    g = gemm_steps(plan)[0]["gemm"]
    assert g["k_bits"] == nk and g["tile"][3] == {3: 8, 4: 16, 7: 64}[nk], g
    monkeypatch.setenv("QT_GEMM_TILES", "1")
    ref = plan.contract_amplitude([], [])
    monkeypatch.setenv("QT_GEMM_TILES", tiles)
    got = plan.contract_amplitude([], [])
    assert got == ref
    want = oracle.contract(tensors, order)
    assert abs(got - want) / abs(want) < TOL


@pytest.mark.parametrize("nb,nm,nn,nk,tile", [(2, 4, 4, 6, [2, 4, 4, 64]), (1, 5, 4, 6, [1, 5, 4, 64]),
                                              (1, 4, 5, 7, [1, 4, 5, 64]), (0, 5, 4, 6, [0, 5, 4, 64]),
                                              (1, 4, 4, 6, [1, 4, 4, 64]), (0, 4, 4, 7, [0, 4, 4, 64]),
                                              (3, 5, 5, 6, [0, 5, 5, 64])])
def test_dense_gemm_every_long_k_tile_shape(monkeypatch, nb, nm, nn, nk, tile):
    # every tile shape the long-K choice can take (the largest m x n tile,
    # then the most sub-tiles), each with 64-deep K stages; the planner picks
    # which of the two tensors is A, so m and n may trade places
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(40 + nb + 3 * nm + 7 * nn + nk, nb, nm, nn, nk)
    plan = api.Plan(api.Network(spec), order, precision="c64_mfma_fp32")
    g = gemm_steps(plan)
    t = g[0]["gemm"]["tile"]
    assert len(g) == 1 and t[0] == tile[0] and sorted(t[1:3]) == sorted(tile[1:3]) and t[3] == tile[3], g
    got = plan.contract_amplitude([], [])
    want = oracle.contract(tensors, order)
    assert abs(got - want) / abs(want) < TOL, (got, want)


@pytest.mark.parametrize("nk,tk", [(3, 8), (4, 16), (5, 16)])
def test_dense_gemm_short_k_stage_depths(monkeypatch, nk, tk):
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(60 + nk, 1, 5, 5, nk)
    plan = api.Plan(api.Network(spec), order, precision="c64_mfma_fp32")
    g = gemm_steps(plan)
    assert len(g) == 1 and g[0]["gemm"]["tile"][3] == tk, g
    got = plan.contract_amplitude([], [])
    want = oracle.contract(tensors, order)
    assert abs(got - want) / abs(want) < TOL, (got, want)


@pytest.mark.parametrize("seed,nb,nm,nn,nk", [(70, 0, 5, 5, 5), (71, 2, 4, 4, 6), (72, 1, 5, 4, 9), (73, 1, 6, 5, 7),
                                              (74, 3, 4, 5, 8)])
def test_dense_gemm_bucket_split_bf16(monkeypatch, seed, nb, nm, nn, nk):
    # K >= 32: products from three BF16 parts per operand on the BF16 matrix
    # cores (3M), FP32 accumulation; the complex64 tolerance holds
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(seed, nb, nm, nn, nk)
    plan = api.Plan(api.Network(spec), order, precision="c64_mfma_bf16x3")
    g = gemm_steps(plan)
    assert len(g) == 1 and g[0]["gemm"]["mode"] == "bf16x3_3m" and g[0]["gemm"]["tile"][3] == 32, g
    got = plan.contract_amplitude([], [])
    want = oracle.contract(tensors, order)
    assert abs(got - want) / abs(want) < TOL, (got, want)
    # and the FP32 products of the same plan agree with it
    ref = api.Plan(api.Network(spec), order, precision="c64_mfma_fp32").contract_amplitude([], [])
    assert abs(got - ref) / abs(ref) < TOL


def test_split_bf16_short_k_keeps_fp32_products(monkeypatch):
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "6")
    spec, tensors, order, _ = dense_case(75, 1, 5, 5, 4)
    plan = api.Plan(api.Network(spec), order, precision="c64_mfma_bf16x3")
    g = gemm_steps(plan)
    assert len(g) == 1 and g[0]["gemm"]["mode"] == "fp32_4m"
    got = plan.contract_amplitude([], [])
    want = oracle.contract(tensors, order)
    assert abs(got - want) / abs(want) < TOL
