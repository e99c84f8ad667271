"""Lightcone deduplication (host side): classes of edges with isomorphic
lightcones, checked against the oracle's per-edge contractions and the p = 1
closed form (whose value depends on the edge only through its endpoints'
degrees and its triangle count)."""
import numpy as np
import pytest

import oracle
from paper_2012_02430_amd.lightcones import lightcone_classes
from workloads import qaoa_params, regular_graph


def _partition_ok(classes, n_edges):
    seen = sorted(i for c in classes for i in c)
    return seen == list(range(n_edges)) and all(c == sorted(c) for c in classes)


@pytest.mark.parametrize("n,p", [(40, 2), (24, 3), (80, 3)])
def test_members_have_the_representatives_energy(n, p):
    edges = regular_graph(n, 3, 0)
    classes = lightcone_classes(edges, p)
    assert _partition_ok(classes, len(edges))
    if n >= 40:  # small graphs at depth 3: every lightcone covers most of the graph
        assert len(classes) < len(edges)
    g, b = qaoa_params(p, 1, seed=n + p)
    vals = np.array([oracle.edge_energy(n, edges, g[0], b[0], u, v).real for u, v in edges])
    for c in classes:
        assert np.abs(vals[c] - vals[c[0]]).max() < 1e-12, c
    # classes are not merged too far: distinct classes differ at a random point
    reps = np.array([vals[c[0]] for c in classes])
    assert len(np.unique(np.round(reps, 10))) == len(classes)


def test_p1_classes_follow_the_triangle_count():
    n = 1000
    edges = regular_graph(n, 3, 0)
    classes = lightcone_classes(edges, 1)
    nb = {}
    for a, b in edges:
        nb.setdefault(a, set()).add(b)
        nb.setdefault(b, set()).add(a)
    lam = [len(nb[u] & nb[v]) for u, v in edges]
    assert _partition_ok(classes, len(edges))
    for c in classes:
        assert len({lam[i] for i in c}) == 1
    assert len(classes) == len(set(lam))


def test_n1000_p3_has_few_classes():
    edges = regular_graph(1000, 3, 0)
    classes = lightcone_classes(edges, 3)
    assert _partition_ok(classes, len(edges))
    assert len(classes) <= 40 and max(len(c) for c in classes) > 1000
