"""Parity of the HIP energy path (per-edge lightcones, one batched launch).

Per-edge values <C_e> lie in [0, 1]; they are compared with an absolute
tolerance equal to the relative one (1e-12 for complex128, 1e-5 for
complex64), and the energy with a relative tolerance.
"""
import numpy as np
import pytest

import oracle
from oracle.statevector import edge_energy_sv
from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from workloads import qaoa_params, regular_graph

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n,p", [(10, 1), (12, 2), (14, 3), (8, 3)])
def test_energy_vs_statevector(precision, n, p):
    edges = regular_graph(n, 3, 1)
    gs, bs = qaoa_params(p, 3, seed=n + p)
    model = api.EnergyModel(n, edges, p, precision=precision)
    E, pe = model.energy(gs, bs, per_edge=True)
    for i in range(3):
        want = oracle.energy_sv(n, edges, gs[i], bs[i])
        assert abs(E[i] - want) / abs(want) < TOL[precision]
        for e, (u, v) in enumerate(edges):
            assert abs(pe[i, e] - edge_energy_sv(n, edges, gs[i], bs[i], u, v)) < TOL[precision]


@pytest.mark.parametrize("precision", ["c64"])
def test_energy_p1_closed_form_n1000(precision):
    n = 1000
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(1, 4, seed=2)
    model = api.EnergyModel(n, edges, 1, precision=precision)
    E, pe = model.energy(gs, bs, per_edge=True)
    for i in range(4):
        want = np.array([oracle.edge_energy_p1(edges, u, v, gs[i, 0], bs[i, 0]).real for u, v in edges])
        assert np.abs(pe[i] - want).max() < TOL[precision]
        assert abs(E[i] - want.sum()) / want.sum() < TOL[precision]


def test_energy_p3_n1000_sampled_and_symmetries():
    # the configuration of the headline energy workload: n=1000, p=3,
    # 1500 lightcones, 32 seeded points
    n, p = 1000, 3
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 32, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    E, pe = model.energy(gs, bs, per_edge=True)
    assert pe.shape == (32, 1500)
    rng = np.random.default_rng(0)
    for i in (0, 17, 31):
        for e in rng.choice(len(edges), 6, replace=False):
            u, v = edges[e]
            want = oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real
            assert abs(pe[i, e] - want) < TOL["c64"], (i, e)
        assert abs(E[i] - pe[i].sum()) < 1e-9 * abs(E[i])
    # exact identities at full size: gamma = 0 or beta = 0 gives |E|/2
    z = np.zeros((2, p))
    E0 = model.energy(z, bs[:2])
    E1 = model.energy(gs[:2], z)
    assert np.abs(E0 - 750.0).max() < 1e-5 * 750 and np.abs(E1 - 750.0).max() < 1e-5 * 750
    # E(-gamma, -beta) = E(gamma, beta)
    Em = model.energy(-gs[:4], -bs[:4])
    assert np.abs(Em - E[:4]).max() < 1e-5 * np.abs(E[:4]).max()


def test_energy_reproducible_and_errors():
    n, p = 20, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 5, seed=3)
    model = api.EnergyModel(n, edges, p)
    a = model.energy(gs, bs, per_edge=True)
    b = model.energy(gs, bs, per_edge=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a plan with slicing is not a lightcone plan
    net = model.networks[0]
    sch = net.plan_slicing(1)
    bad = api.Plan(net, sch.order, sch.groups)
    arr = (L.ctypes.c_void_p * 1)(bad.handle.value) if hasattr(L, "ctypes") else None
    import ctypes

    arr = (ctypes.c_void_p * 1)(bad.handle.value)
    E = np.zeros(1)
    st = L.load().qt_energy_grad(arr, 1, 1, gs[:1].ctypes.data, bs[:1].ctypes.data, E.ctypes.data, None, None,
                                 None, 0)
    assert st == L.QT_EINVAL


def test_energy_p3_n1000_all_edges_one_point():
    # every one of the 1500 lightcones of the p = 3 energy workload at one
    # point against the oracle's contraction of the same lightcone network
    n, p = 1000, 3
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 32, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    E, pe = model.energy(gs, bs, per_edge=True)
    i = 5
    want = np.array([oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real for u, v in edges])
    assert np.abs(pe[i] - want).max() < TOL["c64"]
    assert abs(E[i] - want.sum()) / want.sum() < TOL["c64"]


def test_energy_c128_n1000_p3_sampled():
    n, p = 1000, 3
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 4, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c128")
    E, pe = model.energy(gs, bs, per_edge=True)
    rng = np.random.default_rng(3)
    for i in range(4):
        for e in rng.choice(len(edges), 10, replace=False):
            u, v = edges[e]
            want = oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real
            assert abs(pe[i, e] - want) < TOL["c128"], (i, e)


def _job(err):
    """(programs in LDS, programs from global scratch) of the last job built."""
    ln = [ln for ln in err.splitlines() if ln.startswith("[qt grad] job:")][-1]
    return int(ln.split(":")[1].split()[0]), int(ln.split(",")[2].split()[0])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_energy_oversized_lightcones_run_from_global_scratch(precision, capfd, monkeypatch):
    # an LDS budget below what the largest lightcones need sends them to
    # global scratch in the same launch; the others stay in LDS.  The same
    # schedule runs either way, so every value is bitwise that of the run
    # with every lightcone in LDS, and every edge is checked against the oracle.
    n, p = 40, 3
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 3, seed=12)
    monkeypatch.setenv("QT_DEBUG_GRAD_SCHEDULE", "1")
    monkeypatch.setenv("QT_MULTI_LDS_CAP", str(160 * 1024))  # LDS per workgroup up to the budget
    model = api.EnergyModel(n, edges, p, precision=precision)
    E0, pe0 = model.energy(gs, bs, per_edge=True)
    n_fit0, n_glob0 = _job(capfd.readouterr().err)
    assert n_fit0 + n_glob0 == len(edges) and n_fit0 > 0
    n_fit = n_fit0
    budget = 160 * 1024
    while budget > 2048:  # shrink the budget until more lightcones no longer fit
        budget -= 2048
        monkeypatch.setenv("QT_LDS_BYTES", str(budget))
        E, pe = model.energy(gs, bs, per_edge=True)
        n_fit, n_glob = _job(capfd.readouterr().err)
        if n_fit < n_fit0:
            break
    assert 0 < n_fit < n_fit0 and n_fit + n_glob == len(edges), (budget, n_fit, n_glob)
    assert np.array_equal(E, E0) and np.array_equal(pe, pe0)
    for i in range(3):
        want = np.array([oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real for u, v in edges])
        assert np.abs(pe[i] - want).max() < TOL[precision]


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_energy_lds_cap_tunable_moves_lightcones_to_global_scratch(precision, capfd, monkeypatch):
    # the multi_lds_cap tunable: lightcones needing more LDS than the cap run
    # from global scratch in the same launch, bitwise as from LDS
    n, p = 40, 3
    edges = regular_graph(n, 3, 2)
    gs, bs = qaoa_params(p, 5, seed=13)
    monkeypatch.setenv("QT_DEBUG_GRAD_SCHEDULE", "1")
    model = api.EnergyModel(n, edges, p, precision=precision)
    model.set_tuning(multi_lds_cap=160 * 1024)
    ref = model.energy(gs, bs, per_edge=True)
    n_glob0 = _job(capfd.readouterr().err)[1]
    for cap in (16384, 65536):
        model.set_tuning(multi_lds_cap=cap)
        got = model.energy(gs, bs, per_edge=True)
        n_fit, n_glob = _job(capfd.readouterr().err)
        assert n_fit + n_glob == len(edges) and n_glob >= n_glob0
        if cap == 16384:
            assert n_glob > n_glob0
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), cap
    model.set_tuning()


def test_dedup_energy_n1000_p3_matches_all_edges():
    # one lightcone per isomorphism class, weighted by the class size in the
    # FP64 edge sum, against every edge contracted on its own
    n, p = 1000, 3
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 8, seed=21)
    full = api.EnergyModel(n, edges, p, precision="c64")
    dd = api.EnergyModel(n, edges, p, precision="c64", dedup=True)
    assert len(dd.plans) < 50 and dd.weights.sum() == len(edges)
    E0, pe0 = full.energy(gs, bs, per_edge=True)
    E1, pe1 = dd.energy(gs, bs, per_edge=True)
    assert np.abs(pe1 - pe0).max() < TOL["c64"]
    assert np.abs(E1 - E0).max() < TOL["c64"] * np.abs(E0).max()
    # the dedup'd sum against the oracle on one point, class by class
    i = 3
    for c in dd.classes[:6]:
        u, v = edges[c[0]]
        assert abs(pe1[i, c[0]] - oracle.edge_energy(n, edges, gs[i], bs[i], u, v).real) < TOL["c64"]


def test_dedup_gradient_n200_p2_matches_all_edges():
    n, p = 200, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 16, seed=22)
    full = api.EnergyModel(n, edges, p, precision="c64")
    dd = api.EnergyModel(n, edges, p, precision="c64", dedup=True)
    E0, dg0, db0 = full.energy(gs, bs, grad=True)
    E1, dg1, db1 = dd.energy(gs, bs, grad=True)
    g0 = np.concatenate([dg0, db0], axis=1)
    g1 = np.concatenate([dg1, db1], axis=1)
    assert np.abs(E1 - E0).max() < 1e-12 * np.abs(E0).max()
    assert (np.linalg.norm(g1 - g0, axis=1) / np.linalg.norm(g0, axis=1)).max() < 1e-12
    # device-resident call with weights on the GPU
    import torch

    gd = torch.tensor(gs, device="cuda")
    bd = torch.tensor(bs, device="cuda")
    Ed, ped = dd.energy_device(gd, bd, per_edge=True)
    assert np.abs(Ed.cpu().numpy() - E1).max() < TOL["c64"] * np.abs(E1).max()
    assert ped.shape == (16, len(edges))


def test_weighted_energy_rejects_negative_weights():
    import ctypes

    n, p = 12, 1
    edges = regular_graph(n, 3, 0)
    model = api.EnergyModel(n, edges, p)
    gs, bs = qaoa_params(p, 1, seed=1)
    w = np.ones(len(edges))
    w[3] = -1.0
    E = np.zeros(1)
    st = L.load().qt_energy_grad_weighted(model._arr, w.ctypes.data, len(edges), 1, gs.ctypes.data, bs.ctypes.data,
                                          E.ctypes.data, None, None, None, 0)
    assert st == L.QT_EINVAL


def test_energy_job_cache_eviction_and_threads():
    # The library caches one job (uploaded programs and device buffers) per
    # list of lightcones, at most 16, dropping the oldest; a plan's free drops
    # its jobs.  Jobs are shared-owned, so a call that holds one survives an
    # eviction by another thread, and calls on one model are serialised.
    import threading

    n, p = 10, 1
    gs, bs = qaoa_params(p, 3, seed=31)
    models = [api.EnergyModel(n, regular_graph(n, 3, s), p, precision="c128") for s in range(18)]
    first = [m.energy(gs, bs) for m in models]  # 18 jobs: the first two are evicted
    for m, e in zip(models, first):  # rebuilt on demand, same values
        assert np.array_equal(m.energy(gs, bs), e)
    e0 = models[0].edges
    want = [sum(edge_energy_sv(n, e0, gs[i], bs[i], u, v) for u, v in e0) for i in range(3)]
    assert np.abs(first[0] - np.array(want)).max() < 1e-12 * np.abs(want).max()
    del models[5]  # frees its plans and their jobs
    errors = []

    def worker(k):
        try:
            for _ in range(5):
                j = (3 * k) % 8  # threads k and k + 8/gcd share a model
                m = models[j]
                got = m.energy(gs, bs)
                ref = first[j if j < 5 else j + 1]
                if not np.array_equal(got, ref):
                    errors.append(k)
        except Exception as ex:  # noqa: BLE001 - reported below
            errors.append(repr(ex))

    threads = [threading.Thread(target=worker, args=(k % 4,)) for k in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors


@pytest.mark.parametrize("dedup", [False, True])
@pytest.mark.parametrize("grad", [False, True])
def test_device_arguments_match_host_arguments(grad, dedup):
    """With parameters, weights and results in device memory the batched
    launch reads the parameters where they are and the sums write the
    caller's arrays; energies, per-edge values and gradients equal the
    host-array route bit for bit."""
    import torch

    n, p, npt = 30, 2, 5
    edges = regular_graph(n, 3, 4)
    model = api.EnergyModel(n, edges, p, precision="c64", dedup=dedup)
    gs, bs = qaoa_params(p, npt, seed=13)
    host = model.energy(gs, bs, per_edge=True, grad=grad)
    g = torch.tensor(np.asarray(gs).reshape(npt, p), dtype=torch.float64, device="cuda")
    b = torch.tensor(np.asarray(bs).reshape(npt, p), dtype=torch.float64, device="cuda")
    dev = model.energy_device(g, b, grad=grad, per_edge=True)
    torch.cuda.synchronize()
    assert len(host) == len(dev)
    for h, d in zip(host, dev):
        assert np.array_equal(h, d.cpu().numpy())
