"""Graph capture of a contraction (QT_PLAN_GRAPH): every replay equals the
eager launch sequence bit for bit, with the program's own eager work and
synchronisations between replays, parameters changed in place between
replays, and recapture after a tuning change reallocates the workspace."""
import numpy as np
import pytest
import torch

from paper_2012_02430_amd import api
from paper_2012_02430_amd import network as N
from workloads import qaoa_params, random_bitstring, regular_graph

pytestmark = pytest.mark.gpu


def _plans(precision, fold):
    n, p = 24, 2
    edges = regular_graph(n, 3, 1)
    net = api.Network(N.amplitude_network(n, edges, p, random_bitstring(n, 2)))
    sch = net.plan_slicing(3, algo="min_fill")
    eager = api.Plan(net, sch.order, sch.groups, precision=precision, fold_prefix=fold)
    graph = api.Plan(net, sch.order, sch.groups, precision=precision, fold_prefix=fold, graph=True)
    return eager, graph, p


@pytest.mark.parametrize("precision,fold", [("c64", True), ("c64", False), ("c128", False)])
def test_graph_replays_equal_eager(precision, fold):
    eager, graph, p = _plans(precision, fold)
    npt, ns = 3, eager.n_slices
    gs, bs = qaoa_params(p, 2 * npt, seed=5)
    g = torch.tensor(gs[:npt], dtype=torch.float64, device="cuda")
    b = torch.tensor(bs[:npt], dtype=torch.float64, device="cuda")

    def run(plan):
        out = torch.zeros(npt, 3, dtype=torch.float64, device="cuda")
        per = torch.zeros(npt, ns, 3, dtype=torch.float64, device="cuda")
        plan.contract_device(g, b, out, per)
        torch.cuda.synchronize()
        return out.cpu().numpy(), per.cpu().numpy()

    want = run(eager)
    out = torch.zeros(npt, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(npt, ns, 3, dtype=torch.float64, device="cuda")
    for i in range(5):
        out.fill_(0.0)
        per.fill_(0.0)
        graph.contract_device(g, b, out, per)  # same addresses: capture once, then replay
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want[0]), i
        assert np.array_equal(per.cpu().numpy(), want[1]), i
        # eager work of the program between replays
        x = torch.randn(256, 256, device="cuda")
        (x @ x).sum().item()
        assert np.array_equal(run(eager)[0], want[0])
    # new parameters written in place: the replay reads them
    g.copy_(torch.tensor(gs[npt:], dtype=torch.float64))
    b.copy_(torch.tensor(bs[npt:], dtype=torch.float64))
    want2 = run(eager)
    assert not np.array_equal(want2[0], want[0])
    for i in range(3):
        out.fill_(0.0)
        graph.contract_device(g, b, out, per)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want2[0]), i
        assert np.array_equal(per.cpu().numpy(), want2[1]), i


def test_graph_recaptured_after_tuning_change():
    eager, graph, p = _plans("c64", True)
    gs, bs = qaoa_params(p, 1, seed=6)
    g = torch.tensor(gs, dtype=torch.float64, device="cuda")
    b = torch.tensor(bs, dtype=torch.float64, device="cuda")
    outs = []
    for waves in (16, 8, 16):
        for plan in (eager, graph):
            plan.set_tuning(waves, 0)
        for plan in (eager, graph):
            out = torch.zeros(1, 3, dtype=torch.float64, device="cuda")
            plan.contract_device(g, b, out)
            plan.contract_device(g, b, out)
            torch.cuda.synchronize()
            outs.append(out.cpu().numpy())
    for i in range(0, len(outs), 2):
        assert np.array_equal(outs[i], outs[i + 1])


def test_graph_plan_with_host_arrays_runs_eagerly():
    eager, graph, p = _plans("c64", True)
    gs, bs = qaoa_params(p, 2, seed=7)
    a, pa = eager.contract_batch(gs, bs, per_slice=True)
    c, pc = graph.contract_batch(gs, bs, per_slice=True)
    assert np.array_equal(a, c) and np.array_equal(pa, pc)


@pytest.mark.parametrize("grad,dedup", [(False, False), (True, False), (True, True)])
def test_energy_graph_replays_equal_eager(grad, dedup, capfd, monkeypatch):
    # QT_PLAN_GRAPH on the lightcones: qt_energy_grad captures its device
    # sequence (parameter copy, the batched launch, FP64 sums, result copies)
    # once per argument set and replays it; parameters change in place
    # between replays, with eager work and synchronisations in between.  Some
    # lightcones run from global scratch (LDS cap), so both item kinds are in
    # the graph.
    n, p, npt = 20, 3, 4
    edges = regular_graph(n, 3, 9)
    eager = api.EnergyModel(n, edges, p, precision="c64", dedup=dedup)
    graph = api.EnergyModel(n, edges, p, precision="c64", dedup=dedup, graph=True)
    for m in (eager, graph):
        m.set_tuning(multi_lds_cap=8192, grad_lds_cap=8192)
    monkeypatch.setenv("QT_DEBUG_GRAD_SCHEDULE", "1")
    g = torch.zeros(npt, p, dtype=torch.float64, device="cuda")
    b = torch.zeros(npt, p, dtype=torch.float64, device="cuda")
    n_pl = len(graph.plans)
    E = torch.zeros(npt, dtype=torch.float64, device="cuda")
    pe = torch.zeros(npt, n_pl, dtype=torch.float64, device="cuda")
    dg = torch.zeros(npt, p, dtype=torch.float64, device="cuda")
    db = torch.zeros(npt, p, dtype=torch.float64, device="cuda")
    w = torch.tensor(graph.weights, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for r in range(4):
        gs, bs = qaoa_params(p, npt, seed=40 + r)
        g.copy_(torch.from_numpy(gs))
        b.copy_(torch.from_numpy(bs))
        graph._call(npt, g.data_ptr(), b.data_ptr(), E.data_ptr(), dg.data_ptr() if grad else None,
                    db.data_ptr() if grad else None, pe.data_ptr(), s, w.data_ptr())
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        want = eager.energy(gs, bs, per_edge=True, grad=grad)
        assert np.array_equal(E.cpu().numpy(), want[0]), r
        got_pe = pe.cpu().numpy()
        assert np.array_equal(got_pe[:, eager.class_of] if dedup else got_pe, want[1]), r
        if grad:
            assert np.array_equal(dg.cpu().numpy(), want[2]) and np.array_equal(db.cpu().numpy(), want[3]), r
        del junk
    err = capfd.readouterr().err
    globs = [int(ln.split(",")[2].split()[0]) for ln in err.splitlines() if ln.startswith("[qt grad] job:")]
    assert globs and max(globs) > 0
