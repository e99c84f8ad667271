"""The oracle's pins have teeth: each planted mistake makes one of them fail.

Every mutation below is monkeypatched into the oracle (CPU only) and the
compact pin suite ``_pins_hold`` must then report a failure.  The pins use
only the state-vector simulator, closed forms and exact identities.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import bucket, gates, networks
from oracle.statevector import edge_energy_sv
from workloads import qaoa_params, random_bitstring, regular_graph


def _pins_hold():
    try:
        n, p = 6, 2
        edges = regular_graph(n, 3, 0)
        g, b = qaoa_params(p, 1, seed=11)
        g, b = g[0], b[0]
        z = random_bitstring(n, 2)
        a = oracle.amplitude(n, edges, g, b, z)
        if abs(a - oracle.amplitude_sv(n, edges, g, b, z)) > 1e-12 * abs(a):
            return False
        for u, v in edges[:3]:
            if abs(oracle.edge_energy(n, edges, g, b, u, v) - edge_energy_sv(n, edges, g, b, u, v)) > 1e-12:
                return False
        k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
        if abs(oracle.edge_energy(4, k4, [0.4], [1.1], 0, 1) - oracle.edge_energy_p1(k4, 0, 1, 0.4, 1.1)) > 1e-13:
            return False
        # gradient vs central differences
        _, dg, db, _, _ = oracle.energy_grad(n, edges, g, b)
        th = np.concatenate([g, b])
        for i in range(2 * p):
            tp, tm = th.copy(), th.copy()
            tp[i] += 1e-5
            tm[i] -= 1e-5
            fd = (oracle.energy_sv(n, edges, tp[:p], tp[p:]) - oracle.energy_sv(n, edges, tm[:p], tm[p:])) / 2e-5
            if abs((dg[i] if i < p else db[i - p]) - fd) > 1e-7:
                return False
        # slicing: sum identity and first-variable-most-significant bit order
        T = oracle.amplitude_network(n, edges, g, b, z)
        sl = [3, 8]
        order = oracle.min_degree_order(T, exclude=sl)
        vals = oracle.sliced_values(T, order, [(4, sl)])
        if abs(vals.sum() - a) > 1e-12 * abs(a):
            return False
        # fixing a variable to bit c = attaching the unit vector e_c to it
        e0, e1 = np.array([1.0, 0.0], complex), np.array([0.0, 1.0], complex)
        want = oracle.contract(T + [(e1, (3,)), (e0, (8,))])
        if abs(vals[2] - want) > 1e-12 * abs(want):
            return False
        # batch of amplitudes: index bit a-1-i is the value of open qubit i;
        # a second component (a K4 with no open qubit) closes to a scalar
        e2 = edges + [(6, 7), (6, 8), (6, 9), (7, 8), (7, 9), (8, 9)]
        z2 = random_bitstring(10, 5)
        oq = [4, 1]
        amps = oracle.amplitudes_open(10, e2, g, b, oq, z2)
        for j in range(4):
            zz = z2.copy()
            zz[4], zz[1] = (j >> 1) & 1, j & 1
            if abs(amps[j] - oracle.amplitude_sv(10, e2, g, b, zz)) > 1e-12 * 2.0 ** -5 * 8:
                return False
        return True
    except Exception:
        return False


def test_pins_hold_unmutated():
    assert _pins_hold()


def _rx_wrong_sign(beta):
    c, s = np.cos(np.complex128(beta)), np.sin(np.complex128(beta))
    return np.array([[c, 1j * s], [1j * s, c]])


def _zz_wrong_sign(gamma):
    e = np.exp(1j * np.complex128(gamma))
    return np.array([[1.0, e], [e, 1.0]])


def _zz_on_diagonal(gamma):
    e = np.exp(-1j * np.complex128(gamma))
    return np.array([[e, 1.0], [1.0, e]])


def _plus_unnormalised():
    return np.array([1.0, 1.0], dtype=np.complex128)


def _obs_wrong():
    return np.array([[1.0, 0.0], [0.0, 0.0]], dtype=np.complex128)


def _d_rx_wrong(beta):
    c, s = np.cos(np.complex128(beta)), np.sin(np.complex128(beta))
    return np.array([[s, -1j * c], [-1j * c, s]])


def _lightcone_one_layer_short(n, edges, u, v, p):
    entry, layer_edges = _orig_lightcone(n, edges, u, v, p)
    if p >= 2:
        # plausible slip: only edges with both ends already inside the set
        S = {q for q, k in entry.items() if k >= 1}
        layer_edges = dict(layer_edges)
        layer_edges[1] = [(a, b) for a, b in layer_edges[1] if a in S and b in S]
    return entry, layer_edges


_orig_lightcone = networks.lightcone
_orig_fix = bucket.fix
_orig_product = bucket._product
_orig_sum_out = bucket._sum_out


def _fix_lsb_first(T, values, tangent=False):
    keys = list(values)
    flipped = dict(zip(keys, [values[k] for k in reversed(keys)]))
    return _orig_fix(T, flipped, tangent)


def _product_leibniz_half(A, B, tangent=False):
    if not tangent:
        return _orig_product(A, B)
    c, u = _orig_product(A, B, True)
    a, va = A
    b, vb = B
    union = list(va) + [x for x in vb if x not in va]
    lab = {x: chr(98 + i) for i, x in enumerate(union)}
    sa = "".join(lab[x] for x in va)
    sb = "".join(lab[x] for x in vb)
    su = "".join(lab[x] for x in union)
    c[1:] = np.einsum(f"a{sa},{sb}->a{su}", a[1:], b[0])
    return c, u


def _sum_out_first_axis(R, v, tangent=False):
    r, vr = R
    return r.sum(axis=int(tangent)), vr[1:]


_orig_open_tensor = bucket.open_tensor


def _open_tensor_lsb_first(remaining, scalar, open_vars):
    return _orig_open_tensor(remaining, scalar, list(reversed(open_vars)))


def _open_tensor_drops_scalar(remaining, scalar, open_vars):
    return _orig_open_tensor(remaining, 1.0, open_vars)


MUTATIONS = [
    ("gates.rx sign", gates, "rx", _rx_wrong_sign),
    ("gates.zz sign", gates, "zz", _zz_wrong_sign),
    ("gates.zz phase on equal bits", gates, "zz", _zz_on_diagonal),
    ("gates.plus normalisation", gates, "plus", _plus_unnormalised),
    ("gates.obs_cut wrong diagonal", gates, "obs_cut", _obs_wrong),
    ("gates.d_rx sign", gates, "d_rx", _d_rx_wrong),
    ("lightcone drops layer-1 gates", networks, "lightcone", _lightcone_one_layer_short),
    ("slice bits least significant first", bucket, "fix", _fix_lsb_first),
    ("Leibniz rule drops a term", bucket, "_product", _product_leibniz_half),
    ("sum over the wrong variable", bucket, "_sum_out", _sum_out_first_axis),
    ("open outputs least significant first", bucket, "open_tensor", _open_tensor_lsb_first),
    ("open outputs drop the closed scalars", bucket, "open_tensor", _open_tensor_drops_scalar),
]


@pytest.mark.parametrize("name,mod,attr,fn", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(monkeypatch, name, mod, attr, fn):
    monkeypatch.setattr(mod, attr, fn)
    assert not _pins_hold(), f"planted mistake not caught: {name}"
