"""Parity of the HIP adjoint (reverse bucket elimination) gradient.

dE/dgamma and dE/dbeta from ``qt_energy_grad`` against the oracle's
forward-mode tangents, central finite differences of the GPU energy, and
the complex step of the p = 1 closed form.  A gradient component is a sum
over edges of per-edge derivatives; every edge's contraction uses the same
gate entries, rounded once per point, so rounding errors are correlated
across edges and add up linearly, and each per-edge derivative is itself a
cancellation of terms of the size of the edge's energy.  Its error is
therefore measured against the size of the terms that enter it,
sum_e (|<C_e>| + |d<C_e>/dtheta|), times 1e-12 for complex128 and 1e-5 for
complex64.
"""

import numpy as np
import pytest

import oracle
from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from workloads import qaoa_params, regular_graph

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def oracle_grad(n, edges, g, b):
    E, dg, db, pe, peg = oracle.energy_grad(n, edges, g, b)
    scale = np.abs(pe).sum() + np.abs(peg).sum(axis=0)  # per parameter: gamma_1..p, beta_1..p
    return E, np.concatenate([dg, db]), scale


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n,p", [(8, 1), (10, 2), (12, 3), (14, 2)])
def test_grad_vs_oracle(precision, n, p):
    edges = regular_graph(n, 3, 1)
    gs, bs = qaoa_params(p, 3, seed=10 * n + p)
    model = api.EnergyModel(n, edges, p, precision=precision)
    E, dg, db = model.energy(gs, bs, grad=True)
    for i in range(3):
        Eo, go, scale = oracle_grad(n, edges, gs[i], bs[i])
        got = np.concatenate([dg[i], db[i]])
        assert abs(E[i] - Eo) / abs(Eo) < TOL[precision]
        assert np.all(np.abs(got - go) <= TOL[precision] * scale), (got, go)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_grad_call_returns_forward_energies_bitwise(precision):
    n, p = 12, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 5, seed=3)
    model = api.EnergyModel(n, edges, p, precision=precision)
    E0, pe0 = model.energy(gs, bs, per_edge=True)
    E1, pe1, _, _ = model.energy(gs, bs, per_edge=True, grad=True)
    assert np.array_equal(E0, E1)
    assert np.array_equal(pe0, pe1)


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


def test_grad_p1_closed_form_n1000():
    n = 1000
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(1, 3, seed=5)
    model = api.EnergyModel(n, edges, 1, precision="c64")
    _, dg, db = model.energy(gs, bs, grad=True)
    h = 1e-20
    for i in range(3):
        g, b = gs[i, 0], bs[i, 0]
        e_g = np.array([oracle.edge_energy_p1(edges, u, v, g + 1j * h, b) for u, v in edges])
        e_b = np.array([oracle.edge_energy_p1(edges, u, v, g, b + 1j * h) for u, v in edges])
        size = np.abs(e_g.real).sum()
        assert abs(dg[i, 0] - (e_g.imag / h).sum()) <= 1e-5 * (size + np.abs(e_g.imag / h).sum())
        assert abs(db[i, 0] - (e_b.imag / h).sum()) <= 1e-5 * (size + np.abs(e_b.imag / h).sum())


def test_grad_n200_p2_64_points_sampled_and_antisymmetry():
    # the configuration of the gradient workload: n=200, p=2, 300 lightcones,
    # 64 seeded points in one launch
    n, p = 200, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 64, seed=1)
    model = api.EnergyModel(n, edges, p, precision="c64")
    E, dg, db = model.energy(gs, bs, grad=True)
    assert dg.shape == (64, 2) and db.shape == (64, 2)
    for i in (0, 9, 21, 30, 38, 47, 55, 63):
        Eo, go, scale = oracle_grad(n, edges, gs[i], bs[i])
        assert abs(E[i] - Eo) / abs(Eo) < TOL["c64"]
        got = np.concatenate([dg[i], db[i]])
        assert np.all(np.abs(got - go) <= TOL["c64"] * scale), (i, got, go)
    # E(-gamma, -beta) = E(gamma, beta) (complex conjugation of the circuit),
    # so the gradient is odd
    E2, dg2, db2 = model.energy(-gs, -bs, grad=True)
    assert np.abs(E2 - E).max() < 1e-5 * np.abs(E).max()
    assert np.abs(dg2 + dg).max() < 1e-5 * max(1.0, np.abs(dg).max())
    assert np.abs(db2 + db).max() < 1e-5 * max(1.0, np.abs(db).max())


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
    lines = [ln for ln in err.splitlines() if ln.startswith("[qt grad] job:")]
    assert lines, err
    ln = lines[-1]
    return int(ln.split(",")[1].split()[0]), int(ln.split(",")[2].split()[0])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_checkpoint_recompute_under_forced_budget(precision, capfd, monkeypatch):
    # budgets below what keeps every intermediate force dropped checkpoints
    # that are recomputed in the reverse schedule, and below what any
    # recomputation reaches, the level-per-launch path from global scratch;
    # both run the same arithmetic, so the results are bitwise equal
    n, p = 10, 2
    edges = regular_graph(n, 3, 0)
    gs, bs = qaoa_params(p, 4, seed=7)
    model = api.EnergyModel(n, edges, p, precision=precision)
    monkeypatch.setenv("QT_DEBUG_GRAD_SCHEDULE", "1")
    full = model.energy(gs, bs, grad=True)
    need, n_global = _job_line(capfd.readouterr().err)
    assert n_global == 0
    elt = 16 if precision == "c128" else 8
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
