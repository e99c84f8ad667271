"""Parity of the HIP adjoint (reverse bucket elimination) gradient.

dE/dgamma and dE/dbeta from ``qt_energy_grad`` against the oracle's
forward-mode tangents, central finite differences of the GPU energy, and
the complex step of the p = 1 closed form.  The gradient of one point is
compared normwise: ||g - g_ref||_2 / ||g_ref||_2, absolute when
||g_ref||_2 < 1e-8.  The gradient pass runs in complex128 for every plan
precision (a derivative is a cancellation of per-gate terms of the size of
the edge energy, which complex64 arithmetic does not resolve to 1e-5 near
stationary points), so the bound is the complex128 one, 1e-12, for both.
"""

import numpy as np
import pytest

import oracle
from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from workloads import qaoa_params, regular_graph

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}  # energies from the forward-only launch
GRAD_TOL = 1e-12  # gradients (and the energies of a gradient call): complex128 for every precision


def oracle_grad(n, edges, g, b):
    E, dg, db, pe, peg = oracle.energy_grad(n, edges, g, b)
    return E, np.concatenate([dg, db])


def normwise(got, want):
    d = np.linalg.norm(np.asarray(got) - np.asarray(want))
    w = np.linalg.norm(want)
    return d / w if w >= 1e-8 else d


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n,p", [(8, 1), (10, 2), (12, 3), (14, 2)])
def test_grad_vs_oracle(precision, n, p):
    edges = regular_graph(n, 3, 1)
    gs, bs = qaoa_params(p, 3, seed=10 * n + p)
    model = api.EnergyModel(n, edges, p, precision=precision)
    E, dg, db = model.energy(gs, bs, grad=True)
    for i in range(3):
        Eo, go = oracle_grad(n, edges, gs[i], bs[i])
        got = np.concatenate([dg[i], db[i]])
        assert abs(E[i] - Eo) / abs(Eo) < GRAD_TOL
        assert normwise(got, go) <= GRAD_TOL, (got, go)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_grad_call_returns_forward_energies_bitwise(precision):
    # a gradient call's energies are those of the complex128 forward-only
    # launch, bitwise (same order, same arithmetic); for a complex64 model
    # they agree with its own forward launch to the complex64 tolerance
    n, p = 12, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 5, seed=3)
    model = api.EnergyModel(n, edges, p, precision=precision)
    wide = model if precision == "c128" else api.EnergyModel(n, edges, p, precision="c128")
    E0, pe0 = wide.energy(gs, bs, per_edge=True)
    E1, pe1, _, _ = model.energy(gs, bs, per_edge=True, grad=True)
    assert np.array_equal(E0, E1)
    assert np.array_equal(pe0, pe1)
    E2, pe2 = model.energy(gs, bs, per_edge=True)
    assert np.abs(E2 - E1).max() < TOL[precision] * np.abs(E1).max()
    assert np.abs(pe2 - pe1).max() < TOL[precision]


def test_grad_vs_central_differences():
    n, p = 12, 3
    edges = regular_graph(n, 3, 2)
    gs, bs = qaoa_params(p, 2, seed=4)
    model = api.EnergyModel(n, edges, p, precision="c128")
    _, dg, db = model.energy(gs, bs, grad=True)
    h = 1e-5
    for k in range(p):
        for which, d in (("g", dg), ("b", db)):
            gp, gm, bp, bm = gs.copy(), gs.copy(), bs.copy(), bs.copy()
            if which == "g":
                gp[:, k] += h
                gm[:, k] -= h
            else:
                bp[:, k] += h
                bm[:, k] -= h
            fd = (model.energy(gp, bp) - model.energy(gm, bm)) / (2 * h)
            assert np.all(np.abs(fd - d[:, k]) < 1e-7 * (1 + np.abs(fd))), (which, k, fd, d[:, k])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_grad_p1_closed_form_n1000(precision):
    n = 1000
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(1, 3, seed=5)
    model = api.EnergyModel(n, edges, 1, precision=precision)
    _, dg, db = model.energy(gs, bs, grad=True)
    h = 1e-20
    for i in range(3):
        g, b = gs[i, 0], bs[i, 0]
        e_g = np.array([oracle.edge_energy_p1(edges, u, v, g + 1j * h, b) for u, v in edges])
        e_b = np.array([oracle.edge_energy_p1(edges, u, v, g, b + 1j * h) for u, v in edges])
        want = np.array([(e_g.imag / h).sum(), (e_b.imag / h).sum()])
        assert normwise([dg[i, 0], db[i, 0]], want) <= GRAD_TOL, (i, dg[i, 0], db[i, 0], want)


def test_grad_n200_p2_64_points_sampled_and_antisymmetry():
    # the configuration of the gradient workload: n=200, p=2, 300 lightcones,
    # 64 seeded points in one launch; 16 of them against the oracle,
    # including point 0, the one with the smallest gradient (|g| = 2.2, where
    # the per-gate terms cancel most)
    n, p = 200, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 64, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    E, dg, db = model.energy(gs, bs, grad=True)
    assert dg.shape == (64, 2) and db.shape == (64, 2)
    for i in range(0, 64, 4):
        Eo, go = oracle_grad(n, edges, gs[i], bs[i])
        assert abs(E[i] - Eo) / abs(Eo) < GRAD_TOL
        got = np.concatenate([dg[i], db[i]])
        assert normwise(got, go) <= GRAD_TOL, (i, got, go)
    # E(-gamma, -beta) = E(gamma, beta) (complex conjugation of the circuit),
    # so the gradient is odd
    E2, dg2, db2 = model.energy(-gs, -bs, grad=True)
    assert np.abs(E2 - E).max() < GRAD_TOL * np.abs(E).max()
    for i in range(64):
        assert normwise(-np.concatenate([dg2[i], db2[i]]), np.concatenate([dg[i], db[i]])) <= GRAD_TOL


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_grad_reproducible(precision):
    n, p = 14, 3
    edges = regular_graph(n, 3, 3)
    gs, bs = qaoa_params(p, 6, seed=6)
    model = api.EnergyModel(n, edges, p, precision=precision)
    a = model.energy(gs, bs, grad=True)
    b = model.energy(gs, bs, grad=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def _job_line(err):
    """(LDS bytes per point of the largest program in LDS, programs from global scratch) of the last job."""
    lines = [ln for ln in err.splitlines() if ln.startswith("[qt grad] job:")]
    assert lines, err
    ln = lines[-1]
    return int(ln.split(",")[-1].split()[0]), int(ln.split(",")[2].split()[0])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_checkpoint_recompute_under_forced_budget(precision, capfd, monkeypatch):
    # budgets below what keeps every intermediate force dropped checkpoints
    # that are recomputed in the reverse schedule, and below what any
    # recomputation reaches, programs that run from global scratch in the
    # same launch; all run the same arithmetic, so the results are bitwise
    # equal
    n, p = 10, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 4, seed=7)
    model = api.EnergyModel(n, edges, p, precision=precision)
    monkeypatch.setenv("QT_DEBUG_GRAD_SCHEDULE", "1")
    monkeypatch.setenv("QT_GRAD_LDS_CAP", str(160 * 1024))  # LDS per workgroup up to the budget
    full = model.energy(gs, bs, grad=True)
    need, n_global = _job_line(capfd.readouterr().err)
    assert n_global == 0
    elt = 16  # the gradient pass runs in complex128 for both precisions
    dropped_any = global_any = False
    for k in range(1, 400):
        budget = need - elt * 4 * k
        if budget <= 0:
            break
        monkeypatch.setenv("QT_GRAD_LDS_BYTES", str(budget))
        got = model.energy(gs, bs, grad=True)
        err = capfd.readouterr().err
        drops = [int(ln.split(" dropped")[0].split(",")[-1]) for ln in err.splitlines() if " dropped" in ln]
        dropped_any = dropped_any or any(d > 0 for d in drops)
        global_any = global_any or _job_line(err)[1] > 0
        for x, y in zip(full, got):
            assert np.array_equal(x, y), budget
        if dropped_any and global_any:
            break
    assert dropped_any and global_any


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_global_scratch_path_matches_lds(precision, capfd, monkeypatch):
    n, p = 12, 2
    edges = regular_graph(n, 3, 5)
    gs, bs = qaoa_params(p, 3, seed=8)
    model = api.EnergyModel(n, edges, p, precision=precision)
    monkeypatch.setenv("QT_GRAD_LDS_CAP", str(160 * 1024))
    lds = model.energy(gs, bs, per_edge=True, grad=True)
    monkeypatch.setenv("QT_DEBUG_GRAD_SCHEDULE", "1")
    monkeypatch.setenv("QT_GRAD_LDS_BYTES", "1024")
    glob = model.energy(gs, bs, per_edge=True, grad=True)
    assert _job_line(capfd.readouterr().err)[1] == len(edges)
    for x, y in zip(lds, glob):
        assert np.array_equal(x, y)


def test_autograd_function():
    import torch

    n, p = 12, 2
    edges = regular_graph(n, 3, 4)
    gs, bs = qaoa_params(p, 4, seed=9)
    model = api.EnergyModel(n, edges, p, precision="c128")
    g = torch.tensor(gs, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(bs, dtype=torch.float64, device="cuda", requires_grad=True)
    E = api.qaoa_energy(model, g, b)
    w = torch.arange(1, 5, dtype=torch.float64, device="cuda")
    (w * E).sum().backward()
    _, dg, db = model.energy(gs, bs, grad=True)
    wn = np.arange(1, 5, dtype=np.float64)[:, None]
    assert np.allclose(g.grad.cpu().numpy(), wn * dg, rtol=1e-13, atol=1e-13)
    assert np.allclose(b.grad.cpu().numpy(), wn * db, rtol=1e-13, atol=1e-13)
    # no gradient requested: the forward-only launch, same energies
    with torch.no_grad():
        E2 = api.qaoa_energy(model, g, b)
    assert torch.equal(E.detach(), E2)
