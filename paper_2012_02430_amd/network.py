"""QAOA MaxCut circuits as tensor expressions (Section IV-A, IV-B), host side.

Produces the tensor lists handed to ``qt_load_network``: kinds, layers and
variable ids only -- the gate values are materialised on the GPU from
(gamma, beta) at contraction time.

Variable numbering (the same convention the plans and tests use):
ket variable "qubit q after layer k" is ``k*n + q`` (k = 0 is the input);
the bra variables of the energy network's adjoint half are
``(p + 1 + k)*n + q``.  Diagonal gates (ZZ, the edge observable) add no
variables; each RX opens a new one on its wire.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from paper_2012_02430_amd import _lib as L


@dataclass
class NetworkSpec:
    n_vars: int
    p: int
    # (kind, layer, vars); layer is the bit z for BRA_BIT
    tensors: list = field(default_factory=list)

    def add(self, kind, layer, *vars_):
        self.tensors.append((kind, layer, tuple(int(v) for v in vars_)))

    def variables(self):
        vs = set()
        for _, _, va in self.tensors:
            vs.update(va)
        return vs


def amplitude_network(n: int, edges, p: int, z=None, open_qubits=()) -> NetworkSpec:
    """<z| U(gamma, beta) |+^n>: |+> on layer-0 variables, per layer one ZZ
    per edge and one RX per qubit, <z_q| on the last variable of each wire.

    Qubits in ``open_qubits`` get no <z_q|: their last variables
    (``open_vars(n, p, open_qubits)``) stay open, and a plan that leaves them
    open gives the amplitudes of all 2^a values of those qubits at once (a
    batch of amplitudes, Section VII)."""
    spec = NetworkSpec(n_vars=(p + 1) * n, p=p)
    opened = set(int(q) for q in open_qubits)
    for q in range(n):
        spec.add(L.QT_T_VEC_PLUS, 0, q)
    for k in range(1, p + 1):
        lo = (k - 1) * n
        for a, b in edges:
            spec.add(L.QT_T_ZZ, k, lo + a, lo + b)
        for q in range(n):
            spec.add(L.QT_T_RX, k, lo + q, lo + n + q)
    for q in range(n):
        if q in opened:
            continue
        bit = 0 if z is None else int(z[q])
        spec.add(L.QT_T_BRA_BIT, bit, p * n + q)
    return spec


def open_vars(n: int, p: int, open_qubits) -> list:
    """Variables of the open qubits' last layer, in the order given (the
    first is the most significant bit of the output index)."""
    return [p * n + int(q) for q in open_qubits]


def edge_lightcone(n: int, edges, u: int, v: int, p: int):
    """Qubits and gates of the backward lightcone of the edge term C_uv.

    Walking the layers from p down to 1: the current qubit set gets that
    layer's RX; the layer's ZZ gates touching the set survive (all others
    cancel against their adjoints) and their endpoints join the set.
    Returns (top, zz): ``top[q]`` is the last layer whose RX acts on q (0 for
    qubits reached only by layer-1 ZZ gates), ``zz[k]`` the surviving edges
    of layer k.
    """
    nbrs = {}
    for a, b in edges:
        nbrs.setdefault(a, []).append(b)
        nbrs.setdefault(b, []).append(a)
    inside = {u: p, v: p}
    zz = {}
    for k in range(p, 0, -1):
        cur = set(inside)
        layer = set()
        for q in cur:
            for w in nbrs.get(q, ()):
                layer.add((min(q, w), max(q, w)))
        zz[k] = sorted(layer)
        for a, b in zz[k]:
            for q in (a, b):
                if q not in inside:
                    inside[q] = k - 1
    return inside, zz


def energy_network(n: int, edges, p: int, u: int, v: int) -> NetworkSpec:
    """<+| U^dagger C_uv U |+> over the lightcone of (u, v) (Section III-B).

    Qubit q with top layer t has ket variables for layers 0..t and bra
    variables for layers 0..t-1; its layer-t variable is shared between the
    two halves (only diagonal gates act after it).
    """
    top, zz = edge_lightcone(n, edges, u, v, p)
    spec = NetworkSpec(n_vars=(2 * p + 1) * n, p=p)

    def ket(q, k):
        return min(k, top[q]) * n + q

    def bra(q, k):
        return ket(q, k) if k >= top[q] else (p + 1 + k) * n + q

    qubits = sorted(top)
    for q in qubits:
        spec.add(L.QT_T_VEC_PLUS, 0, ket(q, 0))
        spec.add(L.QT_T_VEC_PLUS, 0, bra(q, 0))
    for k in range(1, p + 1):
        for a, b in zz[k]:
            spec.add(L.QT_T_ZZ, k, ket(a, k - 1), ket(b, k - 1))
            spec.add(L.QT_T_ZZ_DAG, k, bra(a, k - 1), bra(b, k - 1))
        for q in qubits:
            if top[q] >= k:
                spec.add(L.QT_T_RX, k, ket(q, k - 1), ket(q, k))
                spec.add(L.QT_T_RX_DAG, k, bra(q, k - 1), bra(q, k))
    spec.add(L.QT_T_OBS_CUT, 0, ket(u, p), ket(v, p))
    return spec
