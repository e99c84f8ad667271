"""Brute-force state-vector simulation of the QAOA ansatz (n <= 20).

Independent of the tensor-network code: the state is a length-2^n vector
indexed by z = sum_q z_q 2^q, the phase layer multiplies entry z by
exp(-i gamma C(z)) with C(z) the number of cut edges, and the mixer applies
exp(-i beta X_q) = cos(beta) I - i sin(beta) X_q qubit by qubit (X_q flips
bit q of the index).  Complex gamma and beta are accepted.
"""
import numpy as np


def cut_values(n, edges):
    idx = np.arange(2 ** n, dtype=np.int64)
    cut = np.zeros(2 ** n, dtype=np.int64)
    for a, b in edges:
        cut += ((idx >> a) ^ (idx >> b)) & 1
    return cut


def qaoa_state(n, edges, gammas, betas):
    """|psi_p(gamma, beta)> = prod_k e^{-i beta_k H_B} e^{-i gamma_k C} |+^n>."""
    assert n <= 22
    cut = cut_values(n, edges)
    idx = np.arange(2 ** n, dtype=np.int64)
    psi = np.full(2 ** n, 2.0 ** (-n / 2), dtype=np.complex128)
    for g, b in zip(gammas, betas):
        psi = psi * np.exp(-1j * np.complex128(g) * cut)
        c, s = np.cos(np.complex128(b)), np.sin(np.complex128(b))
        for q in range(n):
            psi = c * psi - 1j * s * psi[idx ^ (1 << q)]
    return psi


def amplitude_sv(n, edges, gammas, betas, z=None):
    psi = qaoa_state(n, edges, gammas, betas)
    if z is None:
        return complex(psi[0])
    return complex(psi[int(sum(int(bit) << q for q, bit in enumerate(z)))])


def energy_sv(n, edges, gammas, betas):
    """<psi| C |psi> = sum_z |psi(z)|^2 C(z) (expected cut size); real inputs only."""
    psi = qaoa_state(n, edges, gammas, betas)
    return float(np.sum(np.abs(psi) ** 2 * cut_values(n, edges)))


def edge_energy_sv(n, edges, gammas, betas, u, v):
    psi = qaoa_state(n, edges, gammas, betas)
    idx = np.arange(2 ** n, dtype=np.int64)
    return float(np.sum(np.abs(psi) ** 2 * (((idx >> u) ^ (idx >> v)) & 1)))
