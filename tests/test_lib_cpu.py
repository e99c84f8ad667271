"""Host-only checks of the C-ABI library (no GPU): exports, planner, plan validation."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd import api
from paper_2012_02430_amd import network as N
from workloads import regular_graph

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    names = set()
    for h in (ROOT / "include").glob("*.h"):
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names.update(re.findall(r"\b(qt_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "qt_contract_amplitude" in names and "qt_plan_slicing" in names
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) <= set(L.SIGNATURES)


def _width_of(spec, order, removed=()):
    """Contraction width of an order by plain vertex elimination (Section IV-B)."""
    removed = set(removed)
    adj = {v: set() for v in spec.variables() if v not in removed}
    for _, _, va in spec.tensors:
        va = [x for x in va if x not in removed]
        for a in va:
            adj[a].update(x for x in va if x != a)
    w = 0
    for v in order:
        nb = adj.pop(v)
        w = max(w, len(nb))
        for a in nb:
            adj[a].discard(v)
            adj[a].update(x for x in nb if x != a)
    assert not adj
    return w


@pytest.mark.parametrize("algo", ["min_degree", "min_fill", "rgreedy"])
def test_greedy_order_width(algo):
    n, p = 30, 2
    spec = N.amplitude_network(n, regular_graph(n, 3, 0) if n in (4, 6, 8, 10, 12, 14, 16, 18, 20) else
                               __import__("workloads").generate_regular_graph(n, 3, 0), p)
    net = api.Network(spec)
    order, w = net.order_greedy(algo, tau=0.5, repeats=4, seed=3)
    assert sorted(order) == sorted(spec.variables())
    assert w == _width_of(spec, order)


def test_greedy_tie_break_smallest_id():
    # a 4-cycle of ZZ-like rank-2 tensors: every vertex has degree 2; the
    # smallest id goes first
    spec = N.NetworkSpec(n_vars=4, p=1)
    for a, b in [(0, 1), (1, 2), (2, 3), (3, 0)]:
        spec.add(L.QT_T_ZZ, 1, a, b)
    order, w = api.Network(spec).order_greedy("min_degree")
    assert order[0] == 0 and w == 2


@pytest.mark.parametrize("algo", ["min_degree", "min_fill"])
@pytest.mark.parametrize("k", [1, 4, 8])
def test_step_dependent_slicing(algo, k):
    n, p = 60, 2
    spec = N.amplitude_network(n, regular_graph(n, 3, 0), p)
    net = api.Network(spec)
    sch = net.plan_slicing(k, algo=algo)
    assert len(sch.slice_vars) == k and not set(sch.slice_vars) & set(sch.order)
    assert sorted(sch.order + sch.slice_vars) == sorted(spec.variables())
    assert sch.width == max(sch.prefix_width, sch.slice_width)
    assert sch.width <= sch.unsliced_width
    assert 0 <= sch.step <= sch.peak_step
    # widths recomputed independently: prefix on the full graph, the rest on
    # the graph with the slice variables deleted after the prefix
    assert sch.width_by_step[sch.step] == sch.width
    assert min(sch.width_by_step.values()) == sch.width
    # the symbolic compile of the plan reaches the same widths
    pl = api.Plan(net, sch.order, sch.groups, precision="c64")
    inf = pl.info()
    assert (inf.prefix_width, inf.slice_width) == (sch.prefix_width, sch.slice_width)
    assert inf.n_slices == 2 ** k


def test_slicing_reduces_width_on_210_qubits():
    # Section VIII: greedy width about 44 on the 210-qubit p=1 circuit, and
    # slicing lowers it; here min-degree on the seeded instance
    spec = N.amplitude_network(210, regular_graph(210, 3, 0), 1)
    net = api.Network(spec)
    one = net.plan_slicing(1, algo="min_degree")
    eight = net.plan_slicing(8, algo="min_degree")
    assert 40 <= one.unsliced_width <= 46
    assert one.width <= one.unsliced_width - 1
    assert eight.width <= one.width - 4


def _plan_status(net, order, groups=(), precision="c64"):
    try:
        api.Plan(net, order, groups, precision=precision)
        return L.QT_OK
    except L.QTError as e:
        return e.status


def test_plan_validation():
    spec = N.amplitude_network(8, regular_graph(8, 3, 0), 1)
    net = api.Network(spec)
    order, _ = net.order_greedy("min_fill")
    assert _plan_status(net, order) == L.QT_OK
    assert _plan_status(net, order[:-1]) == L.QT_EPLAN                 # a variable left out
    assert _plan_status(net, order + [order[0]]) == L.QT_EPLAN         # repeated
    assert _plan_status(net, order[1:], [(0, [order[0], order[0]])]) == L.QT_EPLAN
    assert _plan_status(net, order, [(0, [order[0]])]) == L.QT_EPLAN    # sliced and ordered
    assert _plan_status(net, order[1:], [(len(order), [order[0]])]) == L.QT_EPLAN  # step > n_order
    assert _plan_status(net, order[2:], [(0, [order[0]]), (1, [order[1]])]) == L.QT_OK  # two groups (r < n)
    assert _plan_status(net, order[2:], [(2, [order[0]]), (1, [order[1]])]) == L.QT_EPLAN  # steps decrease
    assert _plan_status(net, order + [999]) == L.QT_EPLAN
    assert _plan_status(net, order[1:], [(3, [order[0]])]) == L.QT_OK


def test_open_variable_validation():
    n, p = 8, 1
    edges = regular_graph(n, 3, 0)
    spec = N.amplitude_network(n, edges, p, open_qubits=[2, 5])
    net = api.Network(spec)
    ov = N.open_vars(n, p, [2, 5])
    order, _ = net.order_greedy("min_fill", exclude=ov)
    pl = api.Plan(net, order, open_vars=ov)
    assert pl.info().n_open == 2 and pl.describe()["n_open"] == 2
    with pytest.raises(L.QTError) as e:  # open variables left out of the plan
        api.Plan(net, order)
    assert e.value.status == L.QT_EPLAN
    with pytest.raises(L.QTError) as e:  # an open variable also in the order
        api.Plan(net, order + [ov[0]], open_vars=ov)
    assert e.value.status == L.QT_EPLAN
    with pytest.raises(L.QTError) as e:
        api.Plan(net, order, open_vars=[ov[0], ov[0]])
    assert e.value.status == L.QT_EPLAN


@pytest.mark.parametrize("r", [2, 3])
def test_slicing_groups_r_less_than_n(r):
    # Section VI-D with r < n: groups of r variables, each at its own step of
    # the already-sliced expression; steps non-decreasing, all variables
    # distinct, the order covers every other variable
    n, p, k = 60, 2, 6
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(k, algo="min_fill", group_size=r)
    one = net.plan_slicing(k, algo="min_fill")
    assert len(sch.groups) == (k + r - 1) // r
    assert [len(v) for _, v in sch.groups] == [min(r, k - i * r) for i in range(len(sch.groups))]
    steps = [s for s, _ in sch.groups]
    assert steps == sorted(steps) and steps[0] == sch.step
    sl = [v for _, vs in sch.groups for v in vs]
    assert len(set(sl)) == k and not set(sl) & set(sch.order)
    assert set(sl) | set(sch.order) == net.spec.variables()
    assert sch.width <= one.unsliced_width
    api.Plan(net, sch.order, sch.groups)  # accepted


def test_network_validation():
    lib = L.load()
    spec = N.NetworkSpec(n_vars=4, p=1)
    spec.add(L.QT_T_ZZ, 2, 0, 1)  # layer > p
    with pytest.raises(L.QTError) as e:
        api.Network(spec)
    assert e.value.status == L.QT_EINVAL
    spec = N.NetworkSpec(n_vars=4, p=1)
    spec.add(L.QT_T_RX, 1, 0, 0)  # repeated variable
    with pytest.raises(L.QTError):
        api.Network(spec)
    spec = N.NetworkSpec(n_vars=4, p=1)
    spec.add(L.QT_T_VEC_PLUS, 0, 7)  # out of range
    with pytest.raises(L.QTError):
        api.Network(spec)
    assert lib.qt_load_network(None, ctypes.byref(ctypes.c_void_p())) == L.QT_EINVAL


def test_energy_network_matches_lightcone_convention():
    # same variables and tensor count as the oracle's independent builder
    import oracle

    n, p = 60, 2
    edges = regular_graph(n, 3, 0)
    for u, v in edges[:5]:
        spec = N.energy_network(n, edges, p, u, v)
        T = oracle.energy_network(n, edges, np.zeros(p), np.zeros(p), u, v)
        assert sorted(tuple(sorted(t[2])) for t in spec.tensors) == sorted(tuple(sorted(t[1])) for t in T)


def test_plan_tuning_roundtrip_and_validation(lib):
    from paper_2012_02430_amd import api

    edges = regular_graph(16, 3, 0)
    net = api.Network(N.amplitude_network(16, edges, 2))
    plan = api.Plan(net, net.order_greedy("min_fill")[0], precision="c64")
    names = ("lds_waves", "lds_max_rank", "multi_waves", "grad_waves", "step_tiles", "gemm_tiles", "multi_lds_cap",
             "grad_lds_cap")
    assert plan.get_tuning() == dict.fromkeys(names, 0)
    plan.set_tuning(8, 12, 2, 4, 4, 32, 65536, 8192)
    assert plan.get_tuning() == dict(zip(names, (8, 12, 2, 4, 4, 32, 65536, 8192)))
    for bad in ((17, 0, 0, 0), (0, 5, 0, 0), (0, 17, 0, 0), (0, 0, -1, 0), (0, 0, 0, 99), (0, 0, 0, 0, 3),
                (0, 0, 0, 0, 32), (0, 0, 0, 0, 0, 128), (0, 0, 0, 0, 0, 6), (0, 0, 0, 0, 0, 0, 4095),
                (0, 0, 0, 0, 0, 0, 160 * 1024 + 1), (0, 0, 0, 0, 0, 0, 0, 100)):
        with pytest.raises(L.QTError) as ex:
            plan.set_tuning(*bad)
        assert ex.value.status == L.QT_EINVAL
    assert plan.get_tuning()["lds_max_rank"] == 12  # a rejected call changes nothing
    # the schedule follows the rank threshold (host-only description): at
    # width 9, a threshold of 6 streams the larger steps, 16 keeps all in LDS
    assert plan.info().width >= 8
    plan.set_tuning(0, 6)
    d6 = plan.describe()
    plan.set_tuning(0, 16)
    d16 = plan.describe()
    assert len(d6["stream_steps"]) > 0 and len(d16["stream_steps"]) == 0


def test_plan_signature_is_a_shape_key(lib):
    from paper_2012_02430_amd import api

    edges = regular_graph(8, 3, 0)
    net = api.Network(N.amplitude_network(8, edges, 1))
    order = net.order_greedy("min_fill")[0]
    a = api.Plan(net, order, precision="c64")
    b = api.Plan(net, order, precision="c64")
    c = api.Plan(net, order, precision="c128")
    assert a.signature() == b.signature() != c.signature()


def test_gemm_fusion_only_for_mfma_precision_and_above_threshold(monkeypatch):
    from paper_2012_02430_amd import api

    n, p = 30, 2
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    order, _ = net.order_greedy("min_fill")

    def n_gemm(prec):
        return sum("gemm" in s for s in api.Plan(net, order, precision=prec).describe()["stream_steps"])

    monkeypatch.setenv("QT_GEMM_MIN_RANK", "8")
    assert n_gemm("c64_mfma_fp32") == 1
    assert n_gemm("c64") == 0 and n_gemm("c128") == 0
    monkeypatch.setenv("QT_GEMM_MIN_RANK", "40")
    assert n_gemm("c64_mfma_fp32") == 0
    # the split-BF16 precision fuses the same buckets
    monkeypatch.delenv("QT_GEMM_MIN_RANK", raising=False)
    assert n_gemm("c64_mfma_bf16x3") == n_gemm("c64_mfma_fp32")


def test_gemm_fusion_shrinks_the_n210_plan():
    # the n=210, p=1 min-degree plan with 8 slice variables: two buckets are
    # fused and the largest per-slice intermediate shrinks from 2^29 to 2^25
    from paper_2012_02430_amd import api

    edges = regular_graph(210, 3, 0)
    net = api.Network(N.amplitude_network(210, edges, 1))
    sch = net.plan_slicing(8, algo="min_degree")
    fused = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32")
    plain = api.Plan(net, sch.order, sch.groups, precision="c64")
    g = [s for s in fused.describe()["stream_steps"] if "gemm" in s]
    assert len(g) >= 1
    assert fused.info().width < plain.info().width


def test_product_steps_merged_into_their_producers(lib):
    # The 210-qubit plan with fused GEMM buckets: the product steps that fold
    # a bucket's small tensors into a GEMM operand are merged with the step
    # producing that operand (an extra input without the summed variable);
    # the plain plan keeps them as steps of their own.
    from paper_2012_02430_amd import api

    n, p = 210, 1
    edges = regular_graph(n, 3, 0)
    net = api.Network(N.amplitude_network(n, edges, p))
    sch = net.plan_slicing(8, algo="min_degree")

    def products(plan):  # streaming steps with no summed variable whose first input covers the output
        st = plan.describe()["stream_steps"]
        return [s for s in st if "gemm" not in s and not any(s["in_has_v"]) and s["in_ranks"][0] == s["rank"]]

    fused = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32")
    plain = api.Plan(net, sch.order, sch.groups, precision="c64_mfma_fp32", plain=True)
    assert products(fused) == [] and len(products(plain)) >= 2
    merged = [s for s in fused.describe()["stream_steps"] if "gemm" not in s and s["in_has_v"][-1] == 0
              and any(s["in_has_v"])]
    assert len(merged) >= 2
    assert fused.info().n_steps == plain.info().n_steps - len(products(plain))


def test_describe_lists_segment_steps_by_level(lib):
    """Each LDS segment lists its steps: dependency level, rank, summed flag
    and per input (rank within a slice, holds v, leaf).  Levels are
    consistent with the segment's level count, a summed step has an input
    holding the summed variable (Algorithm 1: a bucket holds the tensors that
    contain its variable; a merged product's inputs may not), and a step's
    output rank never exceeds the sum of its inputs' ranks less v."""
    n, p = 40, 2
    net = api.Network(N.amplitude_network(n, regular_graph(n, 3, 0), p))
    sch = net.plan_slicing(4, algo="min_fill")
    plan = api.Plan(net, sch.order, sch.groups, precision="c64", fold_prefix=True)
    d = plan.describe()
    assert d["segments"]
    for s in d["segments"]:
        steps = s["step_list"]
        assert len(steps) == s["steps"]
        assert max(st[0] for st in steps) == s["levels"] - 1
        for level, rank, summed, ins in steps:
            assert 0 <= level < s["levels"] and ins
            if summed:
                assert any(hv == 1 for _, hv, _ in ins)
            assert rank <= sum(r - hv for r, hv, _ in ins)
