"""qt_contract_batch_noalloc (workspace in the library's static scratch
array, no device allocation) against qt_contract_batch through the C-ABI.

Both paths run the same kernels with the same launch shapes per slice, so
per-slice values agree to the complex64 tolerance (and in practice bitwise
where the slice batch is the same).  Calls run in a row on one GPU: the
second with a smaller input (another plan, fewer points, a slice sub-range)
lays out the array afresh, and a third returns to the first plan.
"""
import numpy as np
import pytest

from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from paper_2012_02430_amd import network as N
from workloads import qaoa_params, regular_graph

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def _plan(n, p, k, precision, **kw):
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill")
    return api.Plan(net, sch.order, sch.groups, precision=precision, **kw)


def _err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_noalloc_matches_contract_batch_on_calls_in_a_row(precision):
    big = _plan(60, 2, 8, precision)          # 256 slices
    small = _plan(20, 2, 4, precision)        # 16 slices
    gb, bb = qaoa_params(2, 3, seed=41)
    gs, bs = qaoa_params(2, 1, seed=42)
    # first call: the 60-qubit plan at three points, all slices, with the journal
    v1, p1 = api.contract_batch_noalloc(big, gb, bb, per_slice=True)
    w1, q1 = big.contract_batch(gb, bb, per_slice=True)
    assert v1.shape == (3,) and p1.shape == (3, 256)
    assert _err(p1, q1) < TOL[precision] and _err(v1, w1) < TOL[precision]
    # second call, smaller: another plan, one point, a slice sub-range
    v2, p2 = api.contract_batch_noalloc(small, gs, bs, 3, 11, per_slice=True)
    w2, q2 = small.contract_batch(gs, bs, 3, 11, per_slice=True)
    assert p2.shape == (1, 8)
    assert _err(p2, q2) < TOL[precision] and _err(v2, w2) < TOL[precision]
    # back to the first plan: the array is laid out for it again
    v3, p3 = api.contract_batch_noalloc(big, gb[:1], bb[:1], per_slice=True)
    assert _err(p3[0], q1[0]) < TOL[precision]
    # and repeating a call on the current layout gives the same values bitwise
    v4, p4 = api.contract_batch_noalloc(big, gb[:1], bb[:1], per_slice=True)
    assert np.array_equal(p3, p4) and np.array_equal(v3, v4)


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    # the 210-qubit plan needs far more than the static array at one slice
    # per launch (per-slice intermediates of 2^25 complex64 values)
    edges = regular_graph(210, 3, 0)
    net = api.Network(N.amplitude_network(210, edges, 1))
    sch = net.plan_slicing(8, algo="min_degree")
    plan = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32")
    g, b = qaoa_params(1, 1, seed=1)
    with pytest.raises(L.QTError) as e:
        api.contract_batch_noalloc(plan, g, b, 0, 2)
    assert e.value.status == L.QT_EINVAL and "static scratch" in str(e.value)
    # a later call that fits still works
    small = _plan(16, 1, 2, "c64")
    v, _ = api.contract_batch_noalloc(small, g, b)
    w, _ = small.contract_batch(g, b)
    assert _err(v, w) < TOL["c64"]
