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
    assert not res["cached"] and len(res["measured"]) == 9
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
    assert set(res["measured"]) == {"1", "2", "4", "8", "16"}
    after = model.energy(gs, bs, per_edge=True, grad=grad)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    for w in (1, 16):
        model.set_tuning(w, w)
        for x, y in zip(before, model.energy(gs, bs, per_edge=True, grad=grad)):
            assert np.array_equal(x, y)
