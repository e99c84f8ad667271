"""Bucket elimination with step-dependent slicing, complex128.

Follows Algorithm 1 (parallel bucket elimination) with its process and thread
levels taken out: the slices are run one after another and their values
summed at the end, which is what the final reduction over ranks computes.

* Each tensor goes to the bucket of its earliest variable under the order pi.
* For each variable v in pi: multiply the bucket's tensors pairwise into R
  (the product's variables are the union of the factors'), sum R over v, and
  put R in the bucket of its earliest remaining variable, or multiply it into
  the scalar result when no variable is left.
* Step-dependent slicing (Section VI-C, VI-D): the first s buckets are
  eliminated once, unsliced (the serial prefix); then the slice variables are
  fixed to the bits of the slice id (binary representation, first slice
  variable = most significant bit) in every remaining tensor and the rest of
  the order is run per slice.  The amplitude is the sum over slice ids of
  the per-slice values (Eq. (2), the sum over the sliced indices m_i).

The library primitive used for a step is numpy's einsum for the broadcast
product of two tensors (no summation inside it); the sum over v is a plain
``ndarray.sum``.

Tangent mode (for gradients): every array carries a leading axis of length D,
entry 0 the value and entries 1.. first-order derivatives.  The pairwise
product then follows the Leibniz rule, C' = A' B + A B', and the sum over v
and slicing act on every entry alike.  This is forward-mode differentiation
of the same elimination, exact up to rounding.
"""
import itertools
import string

import numpy as np

_LETTERS = string.ascii_letters


def _product(A, B, tangent=False):
    """Broadcast product of two tensors: C[union] = A[vars_A] * B[vars_B]."""
    a, va = A
    b, vb = B
    union = list(va) + [x for x in vb if x not in va]
    lab = {x: _LETTERS[i + 1] for i, x in enumerate(union)}
    sa = "".join(lab[x] for x in va)
    sb = "".join(lab[x] for x in vb)
    su = "".join(lab[x] for x in union)
    if not tangent:
        return np.einsum(f"{sa},{sb}->{su}", a, b), tuple(union)
    c = np.empty((a.shape[0],) + (2,) * len(union), dtype=np.complex128)
    c[0] = np.einsum(f"{sa},{sb}->{su}", a[0], b[0])
    c[1:] = np.einsum(f"a{sa},{sb}->a{su}", a[1:], b[0]) + np.einsum(f"{sa},a{sb}->a{su}", a[0], b[1:])
    return c, tuple(union)


def _sum_out(R, v, tangent=False):
    r, vr = R
    i = vr.index(v)
    return r.sum(axis=i + int(tangent)), vr[:i] + vr[i + 1:]


def _scalar_mul(x, y, tangent=False):
    if not tangent:
        return x * y
    out = np.empty_like(x)
    out[0] = x[0] * y[0]
    out[1:] = x[1:] * y[0] + x[0] * y[1:]
    return out


def fix(T, values, tangent=False):
    """Slice a tensor: index every variable in ``values`` at its fixed bit."""
    a, va = T
    keep = []
    idx = [slice(None)] if tangent else []
    for x in va:
        if x in values:
            idx.append(int(values[x]))
        else:
            idx.append(slice(None))
            keep.append(x)
    return a[tuple(idx)], tuple(keep)


def bucket_elimination(tensors, order, tangent=False, D=1):
    """Eliminate the variables of ``order`` in turn.

    Variables not in ``order`` are held (never summed).  Returns
    (remaining, scalar): the tensors left over (those whose variables are all
    held) and the product of the scalars met on the way.  In tangent mode the
    scalar is a length-D vector (value, derivatives).
    """
    pos = {v: i for i, v in enumerate(order)}
    held = len(order)
    buckets = {}
    remaining = []
    if tangent:
        scalar = np.zeros(D, dtype=np.complex128)
        scalar[0] = 1.0
    else:
        scalar = np.complex128(1.0)

    def place(T):
        nonlocal scalar
        a, va = T
        if len(va) == 0:
            scalar = _scalar_mul(scalar, np.asarray(a, dtype=np.complex128), tangent)
            return
        first = min(pos.get(x, held) for x in va)
        if first == held:
            remaining.append(T)
        else:
            buckets.setdefault(first, []).append(T)

    for T in tensors:
        place(T)
    for i, v in enumerate(order):
        bucket = buckets.pop(i, [])
        if not bucket:
            continue
        R = bucket[0]
        for T in bucket[1:]:
            R = _product(R, T, tangent)
        if v in R[1]:
            R = _sum_out(R, v, tangent)
        place(R)
    assert not buckets
    return remaining, scalar


def contract(tensors, order=None):
    """Full contraction of a closed network to a scalar."""
    if order is None:
        order = min_degree_order(tensors)
    rem, s = bucket_elimination(tensors, order)
    assert not rem, "order does not cover every variable"
    return complex(s)


def open_tensor(remaining, scalar, open_vars):
    """The tensor over ``open_vars`` that a contraction with those variables
    held leaves: the outer product of the remaining tensors (each over a
    subset of them) times the scalar, flattened with open_vars[0] as the most
    significant index bit (a batch of amplitudes, Section VII)."""
    a = len(open_vars)
    res = np.full((2,) * a, scalar, dtype=np.complex128)
    for arr, vs in remaining:
        pos = [open_vars.index(x) for x in vs]
        perm = sorted(range(len(vs)), key=lambda i: pos[i])
        shape = [1] * a
        for i in perm:
            shape[pos[i]] = 2
        res = res * np.transpose(arr, perm).reshape(shape)
    return res.reshape(-1)


def contract_open(tensors, open_vars, order=None):
    """Contraction with ``open_vars`` held: 2^a values (open_vars[0] most significant)."""
    open_vars = list(open_vars)
    if order is None:
        order = min_degree_order(tensors, exclude=open_vars)
    rem, s = bucket_elimination(tensors, order)
    return open_tensor(rem, s, open_vars)


def contract_tangent(tensors, order=None):
    """Full contraction in tangent mode: returns (value, derivatives)."""
    if order is None:
        order = min_degree_order(tensors)
    D = tensors[0][0].shape[0]
    rem, s = bucket_elimination(tensors, order, tangent=True, D=D)
    assert not rem, "order does not cover every variable"
    return complex(s[0]), np.array(s[1:])


def sliced_values(tensors, order, groups, open_vars=None):
    """Per-slice values of a step-dependent slicing schedule.

    ``order`` is the elimination order of the unsliced variables; ``groups``
    is a list of (step, slice_vars) with non-decreasing steps: the variables
    of a group are fixed after ``step`` variables of ``order`` have been
    eliminated.  The slice id's bits are the slice variables' values, group
    by group, first variable most significant.  Returns a complex128 array of
    length 2**(total slice variables); its sum is the contraction.  With
    ``open_vars`` (held, never eliminated) each slice gives the 2^a values of
    ``open_tensor`` and the array has shape (2**k, 2**a).
    """
    groups = [(int(s), list(vs)) for s, vs in groups]
    steps = [s for s, _ in groups]
    assert steps == sorted(steps)
    out = []

    def run(tensors, start, g, scalar):
        if g == len(groups):
            rem, s = bucket_elimination(tensors, order[start:])
            if open_vars is None:
                assert not rem
                out.append(scalar * s)
            else:
                out.append(open_tensor(rem, scalar * s, list(open_vars)))
            return
        step, vs = groups[g]
        rem, s = bucket_elimination(tensors, order[start:step])
        for bits in itertools.product((0, 1), repeat=len(vs)):
            values = dict(zip(vs, bits))
            run([fix(T, values) for T in rem], step, g + 1, scalar * s)

    run(list(tensors), 0, 0, np.complex128(1.0))
    return np.array(out, dtype=np.complex128)


def variables(tensors):
    vs = set()
    for _, va in tensors:
        vs.update(va)
    return vs


def min_degree_order(tensors, exclude=()):
    """The oracle's own elimination order: greedy lowest degree (Section V-A1).

    Degree = number of neighbours in the line graph (variables sharing a
    tensor); ties go to the smallest variable id.  Only efficiency depends on
    the order; the contraction value does not.
    """
    exclude = set(exclude)
    adj = {v: set() for v in variables(tensors) if v not in exclude}
    for _, va in tensors:
        va = [x for x in va if x not in exclude]
        for x in va:
            adj[x].update(y for y in va if y != x)
    order = []
    while adj:
        v = min(adj, key=lambda x: (len(adj[x]), x))
        nb = adj.pop(v)
        for x in nb:
            adj[x].discard(v)
            adj[x].update(y for y in nb if y != x)
        order.append(v)
    return order
