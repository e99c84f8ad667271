"""Seeded synthetic inputs for the QAOA MaxCut workloads.

This module is the only code shared by the oracle and the HIP path.  It holds
no tensor-network arithmetic: it produces problem graphs (edge lists) and
variational parameter vectors, nothing else.

Workload family (Section III-B): QAOA MaxCut circuits on random 3-regular
graphs.  The paper publishes no instances, so seeded instances stand in for
them: graphs come from networkx's random regular generator with a fixed seed
and are frozen to edge-list files under ``fixtures/`` so that a change in the
generator cannot change the instances.  Parameters gamma and beta are drawn
uniformly from [0, pi) by numpy's PCG64 generator, gamma before beta for each
point.
"""
from __future__ import annotations

from pathlib import Path

import numpy as np

FIXTURES = Path(__file__).resolve().parent / "fixtures"


def _fixture_path(n: int, d: int, seed: int) -> Path:
    return FIXTURES / f"rr{d}_n{n}_s{seed}.edges"


def regular_graph(n: int, d: int = 3, seed: int = 0) -> list[tuple[int, int]]:
    """Edge list of a seeded random d-regular graph on vertices 0..n-1.

    Edges are (a, b) with a < b, sorted.  A frozen fixture is used when one
    exists; otherwise the graph is generated with networkx.
    """
    path = _fixture_path(n, d, seed)
    if path.exists():
        edges = []
        for line in path.read_text().split("\n"):
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b = line.split()
            edges.append((int(a), int(b)))
        return edges
    return generate_regular_graph(n, d, seed)


def generate_regular_graph(n: int, d: int = 3, seed: int = 0) -> list[tuple[int, int]]:
    import networkx as nx

    g = nx.random_regular_graph(d, n, seed=seed)
    return sorted(tuple(sorted((int(a), int(b)))) for a, b in g.edges())


def freeze_regular_graph(n: int, d: int = 3, seed: int = 0) -> Path:
    """Write the generated graph to its fixture file (used by ``freeze.py``)."""
    edges = generate_regular_graph(n, d, seed)
    path = _fixture_path(n, d, seed)
    path.parent.mkdir(parents=True, exist_ok=True)
    lines = [f"# random {d}-regular graph, n={n}, networkx seed={seed}"]
    lines += [f"{a} {b}" for a, b in edges]
    path.write_text("\n".join(lines) + "\n")
    return path


def qaoa_params(p: int, n_points: int = 1, seed: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """(gammas, betas), each of shape (n_points, p), uniform on [0, pi).

    For each point, the p gammas are drawn first, then the p betas.
    """
    rng = np.random.default_rng(seed)
    gammas = np.empty((n_points, p), dtype=np.float64)
    betas = np.empty((n_points, p), dtype=np.float64)
    for i in range(n_points):
        gammas[i] = rng.uniform(0.0, np.pi, p)
        betas[i] = rng.uniform(0.0, np.pi, p)
    return gammas, betas


def random_bitstring(n: int, seed: int) -> np.ndarray:
    """A seeded output bitstring z (uint8 array of length n)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, n).astype(np.uint8)


# The five workloads the method is measured on (n, p and the size of each
# batch).  Graph seed 0 and parameter seed 1 throughout.
CONFIGS = {
    "C1": dict(kind="amplitude", n=16, p=1, n_points=1, slice_vars=0, order="min_fill"),
    "C2": dict(kind="amplitude", n=60, p=2, n_points=1, slice_vars=8),
    "C3": dict(kind="energy", n=1000, p=3, n_points=32),
    "C4": dict(kind="amplitude", n=210, p=1, n_points=1, slices_run=256),
    "C5": dict(kind="gradient", n=200, p=2, n_points=64),
}
