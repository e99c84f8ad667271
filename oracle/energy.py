"""QAOA MaxCut energy and its gradient from per-edge lightcone networks.

E(gamma, beta) = sum over edges of <C_e>, each <C_e> the full contraction of
the edge's duplicated lightcone network (Section III-B; lightcone
optimisation, Section III-A).  The gradient is forward-mode differentiation
of the same contraction (tangent mode of the bucket elimination: every gate
tensor carries its analytic derivative with respect to its layer's gamma or
beta, and products follow the Leibniz rule), exact up to rounding.
"""
import numpy as np

from oracle.bucket import contract, contract_tangent
from oracle.networks import energy_network


def edge_energy(n, edges, gammas, betas, u, v, order=None):
    """<C_uv> as a complex number (real up to rounding for real parameters)."""
    return contract(energy_network(n, edges, gammas, betas, u, v), order)


def edge_energy_grad(n, edges, gammas, betas, u, v, order=None):
    """(<C_uv>, d<C_uv>/d(gamma_1..gamma_p, beta_1..beta_p)) as complex numbers."""
    return contract_tangent(energy_network(n, edges, gammas, betas, u, v, tangents=True), order)


def energy(n, edges, gammas, betas, edge_list=None):
    """(E, per_edge): the sum in edge order and the per-edge values."""
    edge_list = edges if edge_list is None else edge_list
    per_edge = np.array([edge_energy(n, edges, gammas, betas, u, v) for u, v in edge_list])
    return complex(per_edge.sum()), per_edge


def energy_grad(n, edges, gammas, betas, edge_list=None):
    """(E, dE/dgamma, dE/dbeta, per_edge, per_edge_grad) at real parameters.

    ``per_edge_grad`` has shape (n_edges, 2p): gamma derivatives then beta.
    Values are real parts (the imaginary parts vanish up to rounding).
    """
    p = len(gammas)
    edge_list = edges if edge_list is None else edge_list
    per_edge = []
    per_edge_grad = []
    for u, v in edge_list:
        val, g = edge_energy_grad(n, edges, gammas, betas, u, v)
        per_edge.append(val.real)
        per_edge_grad.append(g.real)
    per_edge = np.array(per_edge)
    per_edge_grad = np.array(per_edge_grad).reshape(len(edge_list), 2 * p)
    grad = per_edge_grad.sum(axis=0)
    return float(per_edge.sum()), grad[:p], grad[p:], per_edge, per_edge_grad
