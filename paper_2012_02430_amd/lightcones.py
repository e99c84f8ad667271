"""Deduplication of per-edge lightcones up to isomorphism (host side).

The energy term of edge (u, v) at depth p depends only on the gates of its
backward lightcone (Section III-A): the ZZ gates of layer k are the graph
edges with an endpoint within distance p - k of {u, v}, so the whole
network is fixed by the subgraph H_uv of edges with an endpoint within
distance p - 1 of {u, v}, with u and v marked.  An isomorphism of H_uv onto
H_u'v' that maps {u, v} onto {u', v'} preserves those distances and so maps
one lightcone network onto the other, tensor by tensor (every gate of the
ansatz is symmetric in its two variables), and the two contractions have
the same value: symmetric lightcones are contracted once (the symmetry
acceleration the paper cites for QAOA energies).  Classes are found exactly:
a Weisfeiler-Lehman hash of H_uv buckets candidates, and a VF2 isomorphism
test (networkx) against each class representative in the bucket decides.
"""
from __future__ import annotations

import networkx as nx


def cone_graph(nbrs: dict, u: int, v: int, p: int) -> nx.Graph:
    """H_uv: the edges with an endpoint within distance p - 1 of {u, v}; node
    attribute ``root`` marks u and v."""
    dist = {u: 0, v: 0}
    frontier = [u, v]
    for d in range(1, p):
        nxt = []
        for q in frontier:
            for w in nbrs.get(q, ()):
                if w not in dist:
                    dist[w] = d
                    nxt.append(w)
        frontier = nxt
    H = nx.Graph()
    for q in dist:
        H.add_node(q)
        for w in nbrs.get(q, ()):
            H.add_edge(q, w)
    for q in H.nodes:
        H.nodes[q]["root"] = 1 if q in (u, v) else 0
    return H


def lightcone_classes(edges, p: int) -> list:
    """Classes of edges with isomorphic lightcones, in order of first
    appearance: a list of lists of edge indices, the first of each class its
    representative."""
    nbrs: dict = {}
    for a, b in edges:
        nbrs.setdefault(a, []).append(b)
        nbrs.setdefault(b, []).append(a)
    same = lambda x, y: x["root"] == y["root"]  # noqa: E731
    graphs, classes, buckets = [], [], {}
    for i, (u, v) in enumerate(edges):
        H = cone_graph(nbrs, int(u), int(v), p)
        graphs.append(H)
        h = nx.weisfeiler_lehman_graph_hash(H, node_attr="root", iterations=3)
        for c in buckets.get(h, ()):
            if nx.is_isomorphic(H, graphs[classes[c][0]], node_match=same):
                classes[c].append(i)
                break
        else:
            buckets.setdefault(h, []).append(len(classes))
            classes.append([i])
    return classes
