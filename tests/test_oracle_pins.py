"""Pins of the oracle against facts that do not go through its tensor-network code.

* hand-derived two-qubit amplitudes (closed form),
* brute-force state vectors (independent phase/mixer application),
* the p=1 partition-sum amplitude and the p=1 per-edge energy closed form,
* exact invariants of the ansatz,
* the slicing identity of Eq. (2) (sum over slices = unsliced contraction),
* gradients: the oracle's tangent-mode derivatives vs central differences of
  the state-vector energy, and vs the complex step of the p=1 closed form.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
from oracle import bucket, networks
from workloads import qaoa_params, random_bitstring, regular_graph

RNG = np.random.default_rng(1234)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("g,b", [(0.3, 0.7), (2.1, 1.3), (0.0, 0.4), (1.0, 0.0)])
def test_two_qubit_hand_derivation(g, b):
    # One edge (0,1), p=1.  Summing the four input bits of |++> by hand:
    # <00|U|++> = <11|U|++> = (cos 2b - i sin 2b e^{-ig}) / 2
    # <01|U|++> = <10|U|++> = (e^{-ig} cos 2b - i sin 2b) / 2
    e = cmath.exp(-1j * g)
    same = 0.5 * (math.cos(2 * b) - 1j * math.sin(2 * b) * e)
    diff = 0.5 * (e * math.cos(2 * b) - 1j * math.sin(2 * b))
    edges = [(0, 1)]
    for z, want in [((0, 0), same), ((1, 1), same), ((1, 0), diff), ((0, 1), diff)]:
        z = np.array(z, dtype=np.uint8)
        assert abs(oracle.amplitude(2, edges, [g], [b], z) - want) < 1e-15
        assert abs(oracle.amplitude_sv(2, edges, [g], [b], z) - want) < 1e-15


def test_single_edge_energy_closed_form():
    # Two qubits, one edge: <C> = 1/2 + 1/2 sin(4b) sin(g) (degrees 1, no triangle).
    for g, b in [(0.3, 0.7), (2.1, 1.3)]:
        want = 0.5 + 0.5 * math.sin(4 * b) * math.sin(g)
        assert abs(oracle.edge_energy(2, [(0, 1)], [g], [b], 0, 1) - want) < 1e-15
        assert abs(oracle.energy_sv(2, [(0, 1)], [g], [b]) - want) < 1e-15


# ------------------------------------------------------ brute force vs network
@pytest.mark.parametrize("n", [4, 6, 8, 10, 12, 14])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_amplitude_vs_statevector(n, p):
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 2, seed=n + 10 * p)
    psi = oracle.qaoa_state(n, edges, g[0], b[0])
    for s in range(3):
        z = random_bitstring(n, seed=s) if s else np.zeros(n, np.uint8)
        want = psi[int(sum(int(x) << q for q, x in enumerate(z)))]
        tensors = oracle.amplitude_network(n, edges, g[0], b[0], z)
        got = oracle.contract(tensors)
        assert rel(got, want) < 1e-12
        # plan independence: a random order gives the same value
        vs = sorted(bucket.variables(tensors))
        order = list(RNG.permutation(vs)) if n <= 8 else None
        if order is not None:
            assert rel(oracle.contract(tensors, order), want) < 1e-12


@pytest.mark.parametrize("n,p", [(16, 1), (18, 1), (20, 1)])
def test_amplitude_p1_partition_sum(n, p):
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(1, 1)
    for s in range(2):
        z = random_bitstring(n, seed=s) if s else None
        want = oracle.amplitude_p1(n, edges, g[0, 0], b[0, 0], z)
        got = oracle.amplitude(n, edges, g[0], b[0], z)
        assert rel(got, want) < 1e-12


def test_norm_over_all_bitstrings():
    n = 8
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(2, 1)
    total = 0.0
    for zi in range(2 ** n):
        z = np.array([(zi >> q) & 1 for q in range(n)], dtype=np.uint8)
        total += abs(oracle.amplitude(n, edges, g[0], b[0], z)) ** 2
    assert abs(total - 1.0) < 1e-12


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("n,p", [(16, 2), (24, 1), (20, 3)])
def test_invariants(n, p):
    edges = _rr(24) if n == 24 else regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=7)
    g, b = g[0], b[0]
    base = 2.0 ** (-n / 2)
    # beta = 0: U is diagonal, <0|U|+> = 2^{-n/2} exactly
    assert rel(oracle.amplitude(n, edges, g, np.zeros(p)), base) < 1e-12
    # gamma = 0: |+> is a +1 eigenvector of every X, <0|U|+> = e^{-i n sum(beta)} 2^{-n/2}
    want = cmath.exp(-1j * n * b.sum()) * base
    assert rel(oracle.amplitude(n, edges, np.zeros(p), b), want) < 1e-12
    a = oracle.amplitude(n, edges, g, b)
    # beta_k -> beta_k + pi/2 multiplies by (-i)^n (X^n commutes with U, fixes |+>)
    b2 = b.copy()
    b2[p - 1] += math.pi / 2
    assert rel(oracle.amplitude(n, edges, g, b2), (-1j) ** n * a) < 1e-12
    # C is integer valued: gamma is 2 pi periodic
    assert rel(oracle.amplitude(n, edges, g + 2 * math.pi, b), a) < 1e-11


def _rr(n):
    from workloads import generate_regular_graph

    return generate_regular_graph(n, 3, 0)


# --------------------------------------------------------------------- energy
@pytest.mark.parametrize("n", [6, 8, 10, 12])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_energy_vs_statevector(n, p):
    edges = regular_graph(n, 3, 1)
    g, b = qaoa_params(p, 1, seed=n * p)
    E, per_edge = oracle.energy(n, edges, g[0], b[0])
    assert abs(E - oracle.energy_sv(n, edges, g[0], b[0])) < 1e-11
    assert np.abs(per_edge.imag).max() < 1e-13
    from oracle.statevector import edge_energy_sv

    for (u, v), val in list(zip(edges, per_edge))[:4]:
        assert abs(val - edge_energy_sv(n, edges, g[0], b[0], u, v)) < 1e-12


def test_energy_p1_closed_form_with_triangles():
    # K4 is 3-regular and every edge lies in two triangles.
    k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for g, b in [(0.4, 1.1), (2.7, 0.3)]:
        for u, v in k4:
            assert abs(oracle.edge_energy(4, k4, [g], [b], u, v) - oracle.edge_energy_p1(k4, u, v, g, b)) < 1e-14


def test_energy_p1_closed_form_n1000():
    n = 1000
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(1, 1)
    for i in range(0, len(edges), 97):
        u, v = edges[i]
        got = oracle.edge_energy(n, edges, g[0], b[0], u, v)
        assert abs(got - oracle.edge_energy_p1(edges, u, v, g[0, 0], b[0, 0])) < 1e-13


def test_energy_symmetries():
    n = 10
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(2, 1, seed=5)
    g, b = g[0], b[0]
    E = oracle.energy(n, edges, g, b)[0].real
    assert abs(oracle.energy(n, edges, np.zeros(2), b)[0] - len(edges) / 2) < 1e-12
    assert abs(oracle.energy(n, edges, g, np.zeros(2))[0] - len(edges) / 2) < 1e-12
    assert abs(oracle.energy(n, edges, -g, -b)[0] - E) < 1e-12
    assert 0 <= E <= len(edges)


def test_lightcone_radius():
    # every qubit of the lightcone is within p of the edge; the edge's own qubits enter at layer p
    n = 60
    edges = regular_graph(n, 3, 0)
    entry, layer_edges = networks.lightcone(n, edges, *edges[0], 2)
    assert entry[edges[0][0]] == 2 and entry[edges[0][1]] == 2
    assert len(entry) <= 2 + 4 + 8
    assert all(0 <= k <= 2 for k in entry.values())


# -------------------------------------------------------------------- slicing
@pytest.mark.parametrize("seed", range(4))
def test_slicing_identity(seed):
    rng = np.random.default_rng(seed)
    n, p = 10, 2
    edges = regular_graph(n, 3, seed % 2)
    g, b = qaoa_params(p, 1, seed=seed)
    z = random_bitstring(n, seed)
    tensors = oracle.amplitude_network(n, edges, g[0], b[0], z)
    full = oracle.contract(tensors)
    assert rel(full, oracle.amplitude_sv(n, edges, g[0], b[0], z)) < 1e-12
    vs = sorted(bucket.variables(tensors))
    k1, k2 = 2, 1 + seed % 2
    sl = list(rng.choice(vs, k1 + k2, replace=False))
    rest = [v for v in vs if v not in sl]
    order = oracle.min_degree_order(tensors, exclude=sl)
    assert sorted(order) == sorted(rest)
    s1 = int(rng.integers(0, len(order) // 2))
    s2 = int(rng.integers(s1, len(order)))
    one = oracle.sliced_values(tensors, order, [(s1, sl)])
    assert one.shape == (2 ** (k1 + k2),)
    assert rel(one.sum(), full) < 1e-12
    two = oracle.sliced_values(tensors, order, [(s1, sl[:k1]), (s2, sl[k1:])])
    assert rel(two.sum(), full) < 1e-12
    # a slice's value is the network with those bits fixed, whatever the step
    assert np.abs(one - two).max() < 1e-13 * np.abs(one).max()
    # slice id bit order: the first slice variable is the most significant bit
    # fixing a variable to bit c = attaching the unit vector e_c to it
    e = [np.array([1.0, 0.0], complex), np.array([0.0, 1.0], complex)]
    bits = [1] + [0] * (len(sl) - 1)
    want = oracle.contract(tensors + [(e[c], (v,)) for v, c in zip(sl, bits)])
    assert rel(one[2 ** (len(sl) - 1)], want) < 1e-12


# ------------------------------------------------------------------- gradient
def test_gradient_vs_finite_differences():
    n, p = 8, 2
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=3)
    E, dg, db, _, _ = oracle.energy_grad(n, edges, g[0], b[0])
    theta = np.concatenate([g[0], b[0]])
    h = 1e-5
    for i in range(2 * p):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (oracle.energy_sv(n, edges, tp[:p], tp[p:]) - oracle.energy_sv(n, edges, tm[:p], tm[p:])) / (2 * h)
        got = dg[i] if i < p else db[i - p]
        assert abs(got - fd) < 1e-7


def test_gradient_p1_closed_form():
    n = 200
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(1, 1, seed=9)
    sub = edges[:12]
    E, dg, db, pe, peg = oracle.energy_grad(n, edges, g[0], b[0], edge_list=sub)
    # the closed form evaluates to an exactly real number at real arguments,
    # so its complex step is exact
    h = 1e-20
    for (u, v), row in zip(sub, peg):
        cg = oracle.edge_energy_p1(edges, u, v, g[0, 0] + 1j * h, b[0, 0]).imag / h
        cb = oracle.edge_energy_p1(edges, u, v, g[0, 0], b[0, 0] + 1j * h).imag / h
        assert abs(row[0] - cg) < 1e-13 and abs(row[1] - cb) < 1e-13


# -------------------------------------------------------- batch of amplitudes
@pytest.mark.parametrize("n,p,open_q", [(10, 2, [3, 7, 0]), (12, 1, [11, 2, 5, 8]), (8, 3, [6])])
def test_open_amplitudes_vs_statevector(n, p, open_q):
    # a contraction with the open qubits' last variables held gives, at
    # index j, the amplitude of the bitstring whose open qubit open_q[i] is
    # bit a-1-i of j (others 0): checked against the state vector for every j
    edges = regular_graph(n, 3, 1)
    g, b = qaoa_params(p, 1, seed=n + p)
    got = oracle.amplitudes_open(n, edges, g[0], b[0], open_q)
    a = len(open_q)
    assert got.shape == (1 << a,)
    for j in range(1 << a):
        z = np.zeros(n, dtype=np.uint8)
        for i, q in enumerate(open_q):
            z[q] = (j >> (a - 1 - i)) & 1
        assert abs(got[j] - oracle.amplitude_sv(n, edges, g[0], b[0], z)) < 1e-12 * 2.0 ** (-n / 2) * 8, j


def test_open_amplitudes_sliced_sum():
    # per-slice open tensors of a slicing schedule add up to the unsliced one
    n, p = 10, 2
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 1, seed=4)
    open_q = [1, 4]
    opened = {oracle.ket_var(n, q, p) for q in open_q}
    T = [t for t in oracle.amplitude_network(n, edges, g[0], b[0]) if not (len(t[1]) == 1 and t[1][0] in opened)]
    ov = [oracle.ket_var(n, q, p) for q in open_q]
    order = oracle.min_degree_order(T, exclude=ov)
    sl = order[4:7]
    rest = [v for v in order if v not in sl]
    per = oracle.sliced_values(T, rest, [(4, sl)], open_vars=ov)
    assert per.shape == (8, 4)
    want = oracle.amplitudes_open(n, edges, g[0], b[0], open_q)
    assert np.abs(per.sum(axis=0) - want).max() < 1e-12 * np.abs(want).max()
