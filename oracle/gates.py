"""Gate tensors of the QAOA MaxCut ansatz, complex128 (Section III-A).

Conventions (the paper leaves signs and factors unstated; this is the reading
used throughout, and the p=1 closed form of Wang et al. holds under it):

* initial state |+> on every qubit (H applied to |0>),
* layer k applies exp(-i gamma_k C) with C = sum over edges of (1 - Z_a Z_b)/2,
  i.e. one diagonal two-variable tensor per edge whose entry is 1 when the
  two bits agree and exp(-i gamma_k) when they differ,
* then exp(-i beta_k X) on every qubit (H_B is the sum of X's), k = 1 first.

A one-qubit gate tensor on variables (in, out) has entry [a, b] = <b|G|a>;
RX is symmetric so the orientation never matters for it.  Adjoint gates used
on the bra side of the energy network are written as analytic functions of
the parameter (never as complex conjugates), so the energy stays holomorphic
in (gamma, beta) and the complex-step derivative applies.
"""
import numpy as np

SQRT1_2 = 1.0 / np.sqrt(2.0)


def plus():
    """|+> = (|0> + |1>)/sqrt(2) as a vector on one variable."""
    return np.array([SQRT1_2, SQRT1_2], dtype=np.complex128)


def zz(gamma):
    """exp(-i gamma (1 - Z_a Z_b)/2) as a diagonal tensor on (x_a, x_b)."""
    e = np.exp(-1j * np.asarray(gamma, dtype=np.complex128))
    return np.array([[1.0, e], [e, 1.0]], dtype=np.complex128)


def zz_dag(gamma):
    """Adjoint of ``zz`` for real gamma: exp(+i gamma (1 - Z_a Z_b)/2)."""
    e = np.exp(1j * np.asarray(gamma, dtype=np.complex128))
    return np.array([[1.0, e], [e, 1.0]], dtype=np.complex128)


def rx(beta):
    """exp(-i beta X) = [[cos b, -i sin b], [-i sin b, cos b]] on (in, out)."""
    b = np.asarray(beta, dtype=np.complex128)
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def rx_dag(beta):
    """Adjoint of ``rx`` for real beta: exp(+i beta X)."""
    b = np.asarray(beta, dtype=np.complex128)
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, 1j * s], [1j * s, c]], dtype=np.complex128)


def d_zz(gamma):
    """d zz / d gamma = -i e^{-i gamma} on the off-diagonal (bits differ)."""
    e = -1j * np.exp(-1j * np.asarray(gamma, dtype=np.complex128))
    return np.array([[0.0, e], [e, 0.0]], dtype=np.complex128)


def d_zz_dag(gamma):
    e = 1j * np.exp(1j * np.asarray(gamma, dtype=np.complex128))
    return np.array([[0.0, e], [e, 0.0]], dtype=np.complex128)


def d_rx(beta):
    """d rx / d beta = [[-sin b, -i cos b], [-i cos b, -sin b]]."""
    b = np.asarray(beta, dtype=np.complex128)
    c, s = np.cos(b), np.sin(b)
    return np.array([[-s, -1j * c], [-1j * c, -s]], dtype=np.complex128)


def d_rx_dag(beta):
    b = np.asarray(beta, dtype=np.complex128)
    c, s = np.cos(b), np.sin(b)
    return np.array([[-s, 1j * c], [1j * c, -s]], dtype=np.complex128)


def bra_bit(z):
    """<z| on one output variable: the unit vector e_z."""
    v = np.zeros(2, dtype=np.complex128)
    v[int(z)] = 1.0
    return v


def obs_cut():
    """Diagonal of the edge term (1 - Z_u Z_v)/2 on (x_u, x_v): 1 iff bits differ."""
    return np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
