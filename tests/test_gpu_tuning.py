"""Autotuner: measured tunables, their JSON cache, and that tuning leaves
results within tolerance (amplitudes) or bitwise unchanged (the lightcone
launches, whose per-item arithmetic does not depend on the wave count)."""
import numpy as np
import pytest

import oracle
from paper_2012_02430_amd import api, autotune
from paper_2012_02430_amd import network as N
from workloads import qaoa_params, random_bitstring, regular_graph

pytestmark = pytest.mark.gpu


def test_tune_plan_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("QT_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, p = 24, 2
    edges = regular_graph(n, 3, 0)
    z = random_bitstring(n, 3)
    net = api.Network(N.amplitude_network(n, edges, p, z))
    sched = net.plan_slicing(n_slice_vars=3, algo="min_fill")
    gs, bs = qaoa_params(p, 1, seed=2)
    want = oracle.amplitude(n, edges, gs[0], bs[0], z)
    plan = api.Plan(net, sched.order, sched.groups, precision="c64")
    a0 = plan.contract_amplitude(gs[0], bs[0])
    res = autotune.tune_plan(plan, repeats=2, max_ranks=(8, 12, 16))
    grid = {f"{w}/{r}/0/0" for w in autotune.PLAN_WAVES for r in (8, 12, 16)}
    assert not res["cached"] and grid <= set(res["measured"])
    assert plan.get_tuning()["lds_waves"] == res["lds_waves"]
    a1 = plan.contract_amplitude(gs[0], bs[0])
    assert abs(a0 - want) / abs(want) < 1e-5 and abs(a1 - want) / abs(want) < 1e-5
    again = api.Plan(net, sched.order, sched.groups, precision="c64")
    hit = autotune.tune_plan(again)
    assert hit["cached"] and again.get_tuning() == plan.get_tuning()


@pytest.mark.parametrize("grad", [False, True])
def test_tune_energy_leaves_results_bitwise(tmp_path, monkeypatch, grad):
    monkeypatch.setenv("QT_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, p = 14, 2
    edges = regular_graph(n, 3, 1)
    gs, bs = qaoa_params(p, 8, seed=3)
    model = api.EnergyModel(n, edges, p, precision="c64")
    before = model.energy(gs, bs, per_edge=True, grad=grad)
    res = autotune.tune_energy(model, 8, grad=grad, repeats=2)
    assert set(res["measured"]) == {f"{w}/{c}" for w in autotune.MULTI_WAVES for c in autotune.MULTI_LDS_CAPS}
    after = model.energy(gs, bs, per_edge=True, grad=grad)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    for w, cap in ((1, 4096), (16, 0), (4, 160 * 1024)):
        model.set_tuning(w, w, cap, cap)
        for x, y in zip(before, model.energy(gs, bs, per_edge=True, grad=grad)):
            assert np.array_equal(x, y)


def test_tune_plan_tile_counts_streaming_and_gemm(tmp_path, monkeypatch):
    # a plan with streaming steps of several tiles per item and fused GEMM
    # buckets: the tuner also times step_tiles and gemm_tiles, and every
    # tile count leaves the amplitude within the complex64 tolerance
    monkeypatch.setenv("QT_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, p = 48, 2
    edges = regular_graph(n, 3, 0)
    z = random_bitstring(n, 5)
    net = api.Network(N.amplitude_network(n, edges, p, z))
    sched = net.plan_slicing(n_slice_vars=4, algo="min_fill")
    gs, bs = qaoa_params(p, 1, seed=4)
    want = oracle.amplitude(n, edges, gs[0], bs[0], z)
    plan = api.Plan(net, sched.order, sched.groups, precision="c64_mfma_fp32", gemm_min_rank=6)
    plan.set_tuning(lds_waves=8, lds_max_rank=10)
    st = plan.describe()["stream_steps"]
    assert any("gemm" in s for s in st) and any("gemm" not in s and s["rank"] > 10 for s in st)
    res = autotune.tune_plan(plan, repeats=1, waves=(8,), max_ranks=(10,))
    keys = set(res["measured"])
    assert {f"8/10/{t}/0" for t in autotune.STEP_TILES} <= keys
    assert any(k.endswith(f"/{t}") for k in keys for t in autotune.GEMM_TILES)
    for t in ({"step_tiles": 1, "gemm_tiles": 64}, {"step_tiles": 16, "gemm_tiles": 1}, res):
        plan.set_tuning(lds_waves=8, lds_max_rank=10, step_tiles=t["step_tiles"], gemm_tiles=t["gemm_tiles"])
        a = plan.contract_amplitude(gs[0], bs[0])
        assert abs(a - want) / abs(want) < 1e-5, t


def test_tune_gemm_min_rank_builds_the_fastest_plan():
    n, p = 48, 2
    edges = regular_graph(n, 3, 0)
    z = random_bitstring(n, 5)
    net = api.Network(N.amplitude_network(n, edges, p, z))
    sched = net.plan_slicing(n_slice_vars=4, algo="min_fill")
    gs, bs = qaoa_params(p, 1, seed=6)
    want = oracle.amplitude(n, edges, gs[0], bs[0], z)
    ranks = (6, 12, 28)  # a GEMM bucket at 6, none at 28
    plan, measured = autotune.tune_gemm_min_rank(net, sched.order, sched.groups, ranks=ranks)
    assert set(measured) == set(ranks) and plan.gemm_min_rank == min(measured, key=measured.get)
    a = plan.contract_amplitude(gs[0], bs[0])
    assert abs(a - want) / abs(want) < 1e-5
