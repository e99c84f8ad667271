"""Circuit -> tensor expression for QAOA MaxCut (Section IV-A, IV-B).

A tensor is a pair (array, vars): ``array`` has one axis of length 2 per
variable, in the order of ``vars``.  Diagonal gates (the ZZ phase, the edge
observable) are written on the variables they share with their wires, which
is the line-graph simplification of Section IV-B: they add no variables.
Each non-diagonal one-qubit gate (RX) ends its wire's current variable and
starts a new one.

Canonical variable numbering (an interface shared, by convention only, with
the plans the tests pass in):

* ket variable x_q^(k), the value of qubit q after layer k (k = 0 is the
  input), has id ``k*n + q``;
* bra variable y_q^(k) of the energy network has id ``(p + 1 + k)*n + q``.
"""
import numpy as np

from oracle import gates


def ket_var(n, q, k):
    return k * n + q


def bra_var(n, p, q, k):
    return (p + 1 + k) * n + q


def amplitude_network(n, edges, gammas, betas, z=None):
    """Tensors of <z| U |+^n> (Section V; the paper's amplitude).

    Variables x_q^(0..p).  |+> on x_q^(0); for k = 1..p one ZZ(gamma_k) per
    edge on (x_a^(k-1), x_b^(k-1)) and one RX(beta_k) per qubit from
    x_q^(k-1) to x_q^(k); <z_q| on x_q^(p).
    """
    p = len(gammas)
    assert len(betas) == p
    if z is None:
        z = np.zeros(n, dtype=np.uint8)
    T = []
    for q in range(n):
        T.append((gates.plus(), (ket_var(n, q, 0),)))
    for k in range(1, p + 1):
        for a, b in edges:
            T.append((gates.zz(gammas[k - 1]), (ket_var(n, a, k - 1), ket_var(n, b, k - 1))))
        for q in range(n):
            T.append((gates.rx(betas[k - 1]), (ket_var(n, q, k - 1), ket_var(n, q, k))))
    for q in range(n):
        T.append((gates.bra_bit(z[q]), (ket_var(n, q, p),)))
    return T


def lightcone(n, edges, u, v, p):
    """Backward lightcone of the edge term C_uv through p layers.

    Returns (entry, layer_edges): ``entry[q]`` is the last layer whose RX acts
    on qubit q inside the lightcone (0 if only ZZ gates of layer 1 reach it);
    ``layer_edges[k]`` lists the ZZ gates of layer k that do not cancel
    between U and U^dagger, i.e. those touching a qubit that layer k's RX
    acts on.  Every gate outside commutes through the observable and cancels
    with its adjoint (Section III-A, lightcone optimisation).
    """
    S = {u, v}
    entry = {u: p, v: p}
    layer_edges = {}
    for k in range(p, 0, -1):
        Ek = [(a, b) for a, b in edges if a in S or b in S]
        layer_edges[k] = Ek
        grown = set(S)
        for a, b in Ek:
            grown.add(a)
            grown.add(b)
        for q in grown - S:
            entry[q] = k - 1
        S = grown
    return entry, layer_edges


def energy_network(n, edges, gammas, betas, u, v, tangents=False):
    """Tensors of <+| U^dagger C_uv U |+> restricted to the lightcone of (u, v).

    This is the duplicated expression of Section III-B: the ket circuit, the
    diagonal edge observable (1 - Z_u Z_v)/2 on the top variables of u and v,
    and the adjoint circuit.  A qubit whose last RX is at layer e shares its
    top variable x^(e) between ket and bra (no non-diagonal gate follows it).

    With ``tangents`` every array gets a leading axis of length 1 + 2p:
    entry 0 is the tensor, entry 1 + i its derivative with respect to
    parameter i of (gamma_1..gamma_p, beta_1..beta_p).
    """
    p = len(gammas)
    D = 1 + 2 * p

    def tag(value, param=None, deriv=None):
        if not tangents:
            return value
        out = np.zeros((D,) + value.shape, dtype=np.complex128)
        out[0] = value
        if param is not None:
            out[1 + param] = deriv
        return out

    entry, layer_edges = lightcone(n, edges, u, v, p)

    def xv(q, k):
        return ket_var(n, q, min(k, entry[q]))

    def yv(q, k):
        if k >= entry[q]:
            return ket_var(n, q, entry[q])
        return bra_var(n, p, q, k)

    T = []
    for q in sorted(entry):
        T.append((tag(gates.plus()), (xv(q, 0),)))
        T.append((tag(gates.plus()), (yv(q, 0),)))
    for k in range(1, p + 1):
        g, b = gammas[k - 1], betas[k - 1]
        for a, c in layer_edges[k]:
            T.append((tag(gates.zz(g), k - 1, gates.d_zz(g)), (xv(a, k - 1), xv(c, k - 1))))
            T.append((tag(gates.zz_dag(g), k - 1, gates.d_zz_dag(g)), (yv(a, k - 1), yv(c, k - 1))))
        for q in sorted(entry):
            if entry[q] >= k:
                T.append((tag(gates.rx(b), p + k - 1, gates.d_rx(b)), (xv(q, k - 1), xv(q, k))))
                T.append((tag(gates.rx_dag(b), p + k - 1, gates.d_rx_dag(b)), (yv(q, k - 1), yv(q, k))))
    T.append((tag(gates.obs_cut()), (xv(u, p), xv(v, p))))
    return T
