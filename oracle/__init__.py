"""Oracle for the QAOA tensor-network contraction -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation, in complex128, of what
the MI355X path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call it; the product
package never does, and this package imports nothing from the product.  It
shares no code with the HIP path: the only common module is ``workloads``
(seeded graphs and parameters, no tensor arithmetic).

Contents
--------
gates        gate tensors of the QAOA MaxCut ansatz (Section III-A)
networks     circuit -> tensor expression, amplitude and per-edge energy
             networks with the canonical variable numbering (Section IV-A,
             Section IV-B, Section III-B's duplicated expression for the energy)
bucket       bucket elimination with a serial prefix and step-dependent slicing
             (Algorithm 1 without processes or threads, Section VI-C/VI-D)
statevector  brute-force state-vector simulation (independent pin, n <= 20)
closed_form  p=1 closed forms (amplitude partition sum, per-edge energy)
energy       energy and its gradient (forward-mode tangents through the same
             elimination) from lightcone networks

Every function is pinned by tests under ``tests/test_oracle_*.py`` against
brute force, closed forms and invariants, none of which goes through the
tensor network code being pinned.
"""
from oracle.gates import plus, zz, zz_dag, rx, rx_dag, bra_bit, obs_cut, d_zz, d_zz_dag, d_rx, d_rx_dag  # noqa: F401
from oracle.networks import (  # noqa: F401
    amplitude_network,
    energy_network,
    lightcone,
    ket_var,
    bra_var,
)
from oracle.bucket import (  # noqa: F401
    bucket_elimination,
    contract,
    contract_open,
    sliced_values,
    min_degree_order,
)
from oracle.energy import edge_energy, edge_energy_grad, energy, energy_grad  # noqa: F401
from oracle.statevector import qaoa_state, amplitude_sv, energy_sv  # noqa: F401
from oracle.closed_form import amplitude_p1, edge_energy_p1  # noqa: F401


def amplitudes_open(n, edges, gammas, betas, open_qubits, z=None, order=None):
    """<z'| U |+^n> for every value of the qubits in ``open_qubits`` (the
    other qubits at z, default 0), in one contraction with their last
    variables held (a batch of amplitudes, Section VII).  Index bit a-1-q of
    the returned 2^a array is the value of open_qubits[q]."""
    p = len(gammas)
    opened = set(int(q) for q in open_qubits)
    tensors = [t for t in amplitude_network(n, edges, gammas, betas, z)
               if not (len(t[1]) == 1 and t[1][0] >= p * n and t[1][0] - p * n in opened)]
    return contract_open(tensors, [ket_var(n, int(q), p) for q in open_qubits], order)


def amplitude(n, edges, gammas, betas, z=None, order=None):
    """<z| U(gamma, beta) |+^n> by plain bucket elimination (Section V).

    ``z`` defaults to the all-zero bitstring.  ``order`` is an elimination
    order over the network's variables (any permutation gives the same value;
    default: the oracle's own min-degree greedy).
    """
    tensors = amplitude_network(n, edges, gammas, betas, z)
    return contract(tensors, order)
