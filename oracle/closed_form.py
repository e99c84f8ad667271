"""Closed forms at p = 1, used as pins that do not go through tensor networks.

* Amplitude: with U = RX(beta)^{(x)n} e^{-i gamma C}, the matrix element
  <z|RX^{(x)n}|x> is cos(beta)^(n-d) (-i sin beta)^d with d the Hamming
  distance of x and z, so
  <z|U|+^n> = 2^{-n/2} sum_x e^{-i gamma C(x)} cos(beta)^(n-d) (-i sin beta)^d.
* Per-edge energy: the p = 1 MaxCut edge expectation of Wang, Hadfield, Jiang
  and Rieffel (2018), the reference the paper gives for the MaxCut
  formulation (Section III-A).  For edge (u, v) with degrees d_u, d_v and
  lam common neighbours (triangles through the edge):
  <C_uv> = 1/2 + 1/4 sin(4b) sin(g) (cos(g)^(d_u-1) + cos(g)^(d_v-1))
             - 1/4 sin(2b)^2 cos(g)^(d_u+d_v-2-2 lam) (1 - cos(2g)^lam).
  Both are analytic in (g, b), so a complex step through them is exact.
"""
import numpy as np

from oracle.statevector import cut_values


def amplitude_p1(n, edges, gamma, beta, z=None):
    zi = 0 if z is None else int(sum(int(bit) << q for q, bit in enumerate(z)))
    idx = np.arange(2 ** n, dtype=np.int64)
    d = np.zeros(2 ** n, dtype=np.int64)
    x = idx ^ zi
    for q in range(n):
        d += (x >> q) & 1
    g = np.complex128(gamma)
    b = np.complex128(beta)
    terms = np.exp(-1j * g * cut_values(n, edges)) * np.cos(b) ** (n - d) * (-1j * np.sin(b)) ** d
    return complex(2.0 ** (-n / 2) * terms.sum())


def edge_energy_p1(edges, u, v, gamma, beta):
    nb = {}
    for a, b in edges:
        nb.setdefault(a, set()).add(b)
        nb.setdefault(b, set()).add(a)
    du, dv = len(nb[u]), len(nb[v])
    lam = len(nb[u] & nb[v])
    g = np.complex128(gamma)
    b = np.complex128(beta)
    cg = np.cos(g)
    return complex(
        0.5
        + 0.25 * np.sin(4 * b) * np.sin(g) * (cg ** (du - 1) + cg ** (dv - 1))
        - 0.25 * np.sin(2 * b) ** 2 * cg ** (du + dv - 2 - 2 * lam) * (1 - np.cos(2 * g) ** lam)
    )
