"""Python face of the C-ABI: networks, plans, contractions.

Thin wrappers over ``_lib`` (ctypes).  Names follow the C entry points;
objects own their C handles and free them on garbage collection.  Streams
are HIP streams given as integers (``torch.cuda.current_stream().cuda_stream``)
or None for the default stream.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from paper_2012_02430_amd import _lib as L
from paper_2012_02430_amd.network import NetworkSpec

PRECISIONS = {"c128": L.QT_C128, "c64": L.QT_C64_SCALED, "c64_mfma_fp32": L.QT_C64_SCALED_MFMA_FP32,
              "c64_mfma_bf16x3": L.QT_C64_SCALED_MFMA_BF16X3}
ORDER_ALGOS = {"min_degree": L.QT_ORDER_MIN_DEGREE, "min_fill": L.QT_ORDER_MIN_FILL, "rgreedy": L.QT_ORDER_RGREEDY}


def amp_to_complex(re: float, im: float, log2_scale: float) -> complex:
    """(re + i im) * 2^log2_scale in FP64."""
    e = math.floor(log2_scale)
    f = 2.0 ** (log2_scale - e)
    return complex(math.ldexp(re * f, e), math.ldexp(im * f, e))


class Network:
    """A loaded tensor network (``qt_load_network``)."""

    def __init__(self, spec: NetworkSpec):
        lib = L.load()
        self.spec = spec
        self._keep = []
        descs = (L.qt_tensor_desc * max(1, len(spec.tensors)))()
        for i, t in enumerate(spec.tensors):
            kind, layer, va = t[0], t[1], t[2]
            arr = L.int32_array(va)
            self._keep.append(arr)
            descs[i].kind = kind
            descs[i].rank = len(va)
            descs[i].layer = layer
            descs[i].vars = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
            if kind == L.QT_T_DENSE:
                vals = np.asarray(t[3], dtype=np.complex128).reshape(-1)
                dense = L.double_array(np.stack([vals.real, vals.imag], axis=1).reshape(-1))
                self._keep.append(dense)
                descs[i].dense = ctypes.cast(dense, ctypes.POINTER(ctypes.c_double))
        nd = L.qt_network_desc(spec.n_vars, len(spec.tensors), spec.p, descs)
        h = ctypes.c_void_p()
        L.check(lib.qt_load_network(ctypes.byref(nd), ctypes.byref(h)))
        self.handle = h
        self._keep = None

    def __del__(self):
        if getattr(self, "handle", None) and L is not None and L._LIB is not None:
            L._LIB.qt_free_network(self.handle)
            self.handle = None

    # ---- planning (host only, Section V-A / VI-C / VI-D)
    def order_greedy(self, algo="min_fill", exclude=(), tau=1.0, repeats=1, seed=0):
        lib = L.load()
        cap = self.spec.n_vars
        out = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        w = ctypes.c_int32()
        ex = L.int32_array(exclude)
        L.check(lib.qt_order_greedy(self.handle, ORDER_ALGOS[algo], ex, len(exclude), float(tau), int(repeats),
                                    int(seed), out, ctypes.byref(n), ctypes.byref(w)))
        return [out[i] for i in range(n.value)], w.value

    def plan_slicing(self, n_slice_vars, algo="min_fill", max_candidates=0, threads=0, tau=1.0, repeats=1, seed=0,
                     group_size=0, exclude=()):
        """Step-dependent slicing search; ``group_size`` r < n slices r variables per group, each group at
        its own step (Section VI-D); ``exclude`` holds variables (open outputs) out of the search."""
        lib = L.load()
        cap = self.spec.n_vars
        order = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        sl = (ctypes.c_int32 * max(1, n_slice_vars))()
        res = L.qt_slicing_result()
        wbs = (ctypes.c_int32 * (cap + 1))()
        ex = L.int32_array(exclude)
        opts = L.qt_slicing_opts(ORDER_ALGOS[algo], n_slice_vars, max_candidates, threads, tau, repeats, seed,
                                 int(group_size), ctypes.cast(ex, ctypes.POINTER(ctypes.c_int32)), len(exclude))
        L.check(lib.qt_plan_slicing(self.handle, ctypes.byref(opts), order, ctypes.byref(n), sl,
                                    ctypes.byref(res), wbs))
        slice_vars = [sl[i] for i in range(n_slice_vars)]
        groups, at = [], 0
        for gi in range(res.n_groups):
            ln = res.group_len[gi]
            groups.append((res.group_step[gi], slice_vars[at:at + ln]))
            at += ln
        return SlicingSchedule(
            order=[order[i] for i in range(n.value)],
            step=res.step,
            slice_vars=slice_vars,
            slice_groups=groups,
            width=res.width,
            prefix_width=res.prefix_width,
            slice_width=res.slice_width,
            unsliced_width=res.unsliced_width,
            peak_step=res.peak_step,
            cost=res.cost,
            width_by_step={s: wbs[s] for s in range(cap + 1) if wbs[s] >= 0},
        )


@dataclass
class SlicingSchedule:
    order: list
    step: int
    slice_vars: list
    slice_groups: list = None
    width: int = 0
    prefix_width: int = 0
    slice_width: int = 0
    unsliced_width: int = 0
    peak_step: int = 0
    cost: float = 0.0
    width_by_step: dict = None

    @property
    def groups(self):
        """[(step, variables)] per slice group, in slice-id bit order."""
        if self.slice_groups:
            return [(s, list(v)) for s, v in self.slice_groups]
        return [(self.step, list(self.slice_vars))] if self.slice_vars else []


class Plan:
    """A compiled plan (``qt_load_plan``) over a loaded network."""

    def __init__(self, network: Network, order, groups=(), precision="c64", slice_batch=0, plain=False,
                 fold_prefix=False, graph=False, open_vars=(), gemm_min_rank=0):
        lib = L.load()
        self.network = network
        groups = list(groups)
        self.order = list(order)
        self.groups = groups
        self.open_vars = [int(v) for v in open_vars]
        self.precision = precision
        o = L.int32_array(self.order)
        steps = L.int32_array([g[0] for g in groups])
        lens = L.int32_array([len(g[1]) for g in groups])
        sv = L.int32_array([v for g in groups for v in g[1]])
        ov = L.int32_array(self.open_vars)
        d = L.qt_plan_desc(ctypes.cast(o, ctypes.POINTER(ctypes.c_int32)), len(self.order), len(groups),
                           ctypes.cast(steps, ctypes.POINTER(ctypes.c_int32)),
                           ctypes.cast(lens, ctypes.POINTER(ctypes.c_int32)),
                           ctypes.cast(sv, ctypes.POINTER(ctypes.c_int32)),
                           PRECISIONS[precision], int(slice_batch),
                           (L.QT_PLAN_PLAIN if plain else 0) | (L.QT_PLAN_FOLD_PREFIX if fold_prefix else 0)
                           | (L.QT_PLAN_GRAPH if graph else 0), len(self.open_vars),
                           ctypes.cast(ov, ctypes.POINTER(ctypes.c_int32)), int(gemm_min_rank))
        h = ctypes.c_void_p()
        L.check(lib.qt_load_plan(network.handle, ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.p = network.spec.p
        self.slice_batch, self.plain, self.fold_prefix = int(slice_batch), bool(plain), bool(fold_prefix)
        self.graph = bool(graph)
        self.gemm_min_rank = int(gemm_min_rank)

    def signature(self) -> str:
        """Shape signature (network structure, order, slicing, precision, flags): the autotuner's cache key."""
        import hashlib
        import json

        spec = self.network.spec
        blob = json.dumps({"n_vars": spec.n_vars, "p": spec.p,
                           "tensors": [[int(t[0]), int(t[1]), [int(v) for v in t[2]]]
                                       + ([np.asarray(t[3], dtype=np.complex128).reshape(-1).view(np.float64).tolist()]
                                          if len(t) > 3 else [])
                                       for t in spec.tensors],
                           "order": self.order, "groups": [[int(g[0]), [int(v) for v in g[1]]] for g in self.groups],
                           "open_vars": self.open_vars,
                           "precision": self.precision, "slice_batch": self.slice_batch, "plain": self.plain,
                           "fold_prefix": self.fold_prefix, "gemm_min_rank": self.gemm_min_rank}, sort_keys=True)
        return hashlib.sha1(blob.encode()).hexdigest()

    def set_tuning(self, lds_waves=0, lds_max_rank=0, multi_waves=0, grad_waves=0, step_tiles=0, gemm_tiles=0,
                   multi_lds_cap=0, grad_lds_cap=0):
        """Sets every tunable (0: the library default); ``qt_plan_set_tuning``."""
        t = L.qt_tuning(int(lds_waves), int(lds_max_rank), int(multi_waves), int(grad_waves), int(step_tiles),
                        int(gemm_tiles), int(multi_lds_cap), int(grad_lds_cap))
        L.check(L.load().qt_plan_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = L.qt_tuning()
        L.check(L.load().qt_plan_get_tuning(self.handle, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in L.qt_tuning._fields_}

    def __del__(self):
        if getattr(self, "handle", None) and L is not None and L._LIB is not None:
            L._LIB.qt_free_plan(self.handle)
            self.handle = None

    def info(self) -> L.qt_plan_info:
        inf = L.qt_plan_info()
        L.check(L.load().qt_plan_get_info(self.handle, ctypes.byref(inf)))
        return inf

    @property
    def n_slices(self) -> int:
        return self.info().n_slices

    def describe(self) -> dict:
        """Launch schedule (segments, levels, LDS bytes, streaming steps); host only."""
        import json

        need = ctypes.c_int64()
        L.load().qt_plan_describe(self.handle, None, 0, ctypes.byref(need))
        buf = ctypes.create_string_buffer(need.value)
        L.check(L.load().qt_plan_describe(self.handle, buf, need.value, ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def profile_enable(self, on=True):
        L.check(L.load().qt_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self, reset=True):
        """{kernel class: (launches, ms, bytes, flops)} from HIP events."""
        arr = (L.qt_kernel_stats * L.QT_KCLASS_COUNT)()
        L.check(L.load().qt_profile_read(self.handle, arr, 1 if reset else 0))
        return {name: (arr[i].launches, arr[i].ms, arr[i].bytes, arr[i].flops)
                for i, name in L.QT_KCLASS_NAMES.items() if arr[i].launches}

    def profile_read_ops(self, reset=True) -> list:
        """Per operation of the schedule: dicts with kclass, op (step or segment index, -1 for other
        kernels), launches, ms, bytes, flops, in order of first launch."""
        n = ctypes.c_int32()
        L.check(L.load().qt_profile_read_ops(self.handle, None, 0, ctypes.byref(n), 0))
        arr = (L.qt_op_stats * max(1, n.value))()
        L.check(L.load().qt_profile_read_ops(self.handle, arr, n.value, ctypes.byref(n), 1 if reset else 0))
        return [{"kclass": L.QT_KCLASS_NAMES.get(arr[i].kclass, arr[i].kclass), "op": arr[i].op,
                 "launches": arr[i].launches, "ms": arr[i].ms, "bytes": arr[i].bytes, "flops": arr[i].flops}
                for i in range(n.value)]

    def contract_amplitude(self, gammas, betas, stream=None):
        """The amplitude (complex), or with open variables the 2^a amplitudes (complex array, index bit
        a-1-q = value of open_vars[q])."""
        g = np.ascontiguousarray(gammas, dtype=np.float64).reshape(-1)
        b = np.ascontiguousarray(betas, dtype=np.float64).reshape(-1)
        if g.size != self.p or b.size != self.p:
            raise ValueError("gammas and betas need p values each")
        na = 1 << len(self.open_vars)
        out = (L.qt_amp * na)()
        L.check(L.load().qt_contract_amplitude(self.handle, g.ctypes.data, b.ctypes.data,
                                               ctypes.cast(out, ctypes.c_void_p), stream or 0))
        vals = np.array([amp_to_complex(o.re, o.im, o.log2_scale) for o in out])
        return complex(vals[0]) if not self.open_vars else vals

    def contract_device(self, gammas, betas, out, per_slice=None, slice_begin=0, slice_end=None, stream=None):
        """Device-resident call: gammas/betas float64 GPU tensors [n_points, p]; out a float64 GPU tensor
        [n_points, 3] (re, im, log2 scale); per_slice optional [n_points, n_range, 3].  With graph=True the
        launch sequence is captured on the first call and replayed on later ones."""
        import torch

        n_points = out.shape[0]
        end = self.n_slices if slice_end is None else slice_end
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        arr = (ctypes.c_void_p * 1)(self.handle.value)
        L.check(L.load().qt_contract_batch(arr, 1, n_points, gammas.data_ptr() if self.p else None,
                                           betas.data_ptr() if self.p else None, slice_begin, end,
                                           ctypes.c_void_p(out.data_ptr()),
                                           per_slice.data_ptr() if per_slice is not None else None, s))

    def contract_batch(self, gammas, betas, slice_begin=0, slice_end=None, per_slice=False, stream=None):
        """Partial sums over a slice range at every point; optional per-slice values.

        Returns (values[n_points] complex, per_slice[n_points, n_range] complex or None); with open
        variables values[n_points, 2^a] and per_slice[n_points, 2^a, n_range].
        """
        return contract_batch([self], gammas, betas, slice_begin, slice_end, per_slice, stream)


def contract_batch_noalloc(plan, gammas, betas, slice_begin=0, slice_end=None, per_slice=False, stream=None):
    """``qt_contract_batch_noalloc``: one plan, with its device workspace in the library's static scratch
    array (no device allocation).  Same results as ``contract_batch([plan], ...)``."""
    lib = L.load()
    p = plan.p
    g = np.ascontiguousarray(gammas, dtype=np.float64).reshape(-1, p) if p else np.zeros((1, 0))
    b = np.ascontiguousarray(betas, dtype=np.float64).reshape(-1, p) if p else np.zeros((1, 0))
    n_points = g.shape[0]
    if slice_end is None:
        slice_end = plan.n_slices
    n_range = slice_end - slice_begin
    a = len(plan.open_vars)
    out = (L.qt_amp * (n_points << a))()
    ps = np.zeros((n_points << a, n_range, 3)) if per_slice else None
    L.check(lib.qt_contract_batch_noalloc(plan.handle, n_points, g.ctypes.data, b.ctypes.data, slice_begin, slice_end,
                                          ctypes.cast(out, ctypes.c_void_p), ps.ctypes.data if per_slice else None,
                                          stream or 0))
    shape = (n_points,) + ((1 << a,) if a else ())
    vals = np.array([amp_to_complex(o.re, o.im, o.log2_scale) for o in out]).reshape(shape)
    slices = None
    if per_slice:
        slices = np.vectorize(amp_to_complex)(ps[..., 0], ps[..., 1], ps[..., 2]).reshape(shape + (n_range,))
    return vals, slices


def contract_batch(plans, gammas, betas, slice_begin=0, slice_end=None, per_slice=False, stream=None):
    lib = L.load()
    p = plans[0].p
    g = np.ascontiguousarray(gammas, dtype=np.float64).reshape(-1, p) if p else np.zeros((1, 0))
    b = np.ascontiguousarray(betas, dtype=np.float64).reshape(-1, p) if p else np.zeros((1, 0))
    n_points = g.shape[0]
    if slice_end is None:
        slice_end = plans[0].n_slices
    n_range = slice_end - slice_begin
    a = len(plans[0].open_vars)
    arr = (ctypes.c_void_p * len(plans))(*[pl.handle.value for pl in plans])
    out = (L.qt_amp * (len(plans) * (n_points << a)))()
    ps = np.zeros((len(plans), n_points << a, n_range, 3)) if per_slice else None
    st = lib.qt_contract_batch(arr, len(plans), n_points, g.ctypes.data, b.ctypes.data, slice_begin, slice_end,
                               ctypes.cast(out, ctypes.c_void_p), ps.ctypes.data if per_slice else None,
                               stream or 0)
    L.check(st)
    shape = (len(plans), n_points) + ((1 << a,) if a else ())
    vals = np.array([amp_to_complex(o.re, o.im, o.log2_scale) for o in out]).reshape(shape)
    slices = None
    if per_slice:
        slices = np.vectorize(amp_to_complex)(ps[..., 0], ps[..., 1], ps[..., 2])
        slices = slices.reshape(shape + (n_range,))
    if len(plans) == 1:
        return vals[0], (slices[0] if per_slice else None)
    return vals, slices


class SliceJournal:
    """Journal of per-slice results: the resumable unit of work.

    Slices of a step-dependent slicing plan are independent and their values
    add up to the amplitude (Eq. (2)), so a contraction interrupted partway
    can be resumed by running only the slices it has not recorded.  A work
    unit is (plan signature, point, slice id); ``record`` stores the FP64
    per-slice values of a slice range for every point, ``missing`` lists the
    ranges still to run, and ``total`` sums the recorded values of each point
    in slice-id order, so a resumed run gives bitwise the same total as an
    uninterrupted one.  ``save``/``load`` keep the journal in an .npz file
    (plain arrays, no pickled objects).
    """

    def __init__(self, key: str, n_points: int, n_slices: int):
        self.key = str(key)
        self.values = np.zeros((n_points, n_slices), dtype=np.complex128)
        self.done = np.zeros(n_slices, dtype=bool)

    @property
    def n_slices(self) -> int:
        return self.done.size

    def record(self, begin: int, per_slice) -> None:
        per = np.asarray(per_slice, dtype=np.complex128).reshape(self.values.shape[0], -1)
        end = begin + per.shape[1]
        if begin < 0 or end > self.n_slices:
            raise ValueError("slice range outside the journal")
        self.values[:, begin:end] = per
        self.done[begin:end] = True

    def missing(self, max_len: int = 0) -> list:
        """Ranges [begin, end) of unrecorded slices, cut to at most ``max_len`` slices (0: uncut)."""
        out = []
        i = 0
        while i < self.n_slices:
            if self.done[i]:
                i += 1
                continue
            j = i
            while j < self.n_slices and not self.done[j] and (max_len <= 0 or j - i < max_len):
                j += 1
            out.append((i, j))
            i = j
        return out

    def complete(self) -> bool:
        return bool(self.done.all())

    def total(self) -> np.ndarray:
        if not self.complete():
            raise ValueError("journal has unrecorded slices")
        tot = np.zeros(self.values.shape[0], dtype=np.complex128)
        for s in range(self.n_slices):  # slice-id order, FP64
            tot += self.values[:, s]
        return tot

    def save(self, path) -> None:
        np.savez(path, key=np.array(self.key), values=self.values, done=self.done)

    @classmethod
    def load(cls, path, key: str):
        with np.load(path, allow_pickle=False) as z:
            if str(z["key"]) != str(key):
                raise ValueError("journal belongs to another contraction")
            j = cls(key, z["values"].shape[0], z["values"].shape[1])
            j.values[...] = z["values"]
            j.done[...] = z["done"]
        return j


def run_resumable(contract, journal: SliceJournal, max_len: int = 0, path=None) -> np.ndarray:
    """Runs the journal's missing slice ranges through ``contract(begin, end)``
    (per-slice values [n_points][end - begin]), recording (and saving, when
    ``path`` is given) after every range; returns the totals per point."""
    for begin, end in journal.missing(max_len):
        journal.record(begin, contract(begin, end))
        if path is not None:
            journal.save(path)
    return journal.total()


class EnergyModel:
    """QAOA MaxCut energy from per-edge lightcone networks (``qt_energy_grad``).

    One network and one plan per edge (greedy order, no slicing); every edge
    and point runs in one batched launch.  With ``dedup`` the edges are
    grouped by lightcone isomorphism (``lightcones.lightcone_classes``): one
    network and plan per class, each weighted by its size in the FP64 sums
    (``qt_energy_grad_weighted``); per-edge values are those of the edge's
    class representative.
    """

    def __init__(self, n, edges, p, precision="c64", algo="min_fill", dedup=False, graph=False):
        from paper_2012_02430_amd import network as N

        self.n, self.p = n, p
        self.edges = [tuple(e) for e in edges]
        if dedup:
            from paper_2012_02430_amd.lightcones import lightcone_classes

            self.classes = lightcone_classes(self.edges, p)
        else:
            self.classes = [[e] for e in range(len(self.edges))]
        self.dedup = bool(dedup)
        self.class_of = np.zeros(len(self.edges), dtype=np.int64)
        for c, members in enumerate(self.classes):
            self.class_of[members] = c
        self.weights = np.array([float(len(m)) for m in self.classes])
        reps = [self.edges[m[0]] for m in self.classes]
        self.networks = [Network(N.energy_network(n, self.edges, p, u, v)) for u, v in reps]
        self.plans = [Plan(net, net.order_greedy(algo)[0], precision=precision, graph=graph) for net in self.networks]
        self._arr = (ctypes.c_void_p * len(self.plans))(*[pl.handle.value for pl in self.plans])

    def _call(self, npt, g_ptr, b_ptr, E_ptr, dg_ptr, db_ptr, pe_ptr, stream, w_ptr=None):
        lib = L.load()
        if self.dedup:
            w = w_ptr if w_ptr is not None else self.weights.ctypes.data
            L.check(lib.qt_energy_grad_weighted(self._arr, w, len(self.plans), npt, g_ptr, b_ptr, E_ptr, dg_ptr,
                                                db_ptr, pe_ptr, stream))
        else:
            L.check(lib.qt_energy_grad(self._arr, len(self.plans), npt, g_ptr, b_ptr, E_ptr, dg_ptr, db_ptr,
                                       pe_ptr, stream))

    def energy(self, gammas, betas, per_edge=False, grad=False, stream=None):
        """E per point (and per-edge values [n_points, n_edges], and (dE/dgamma, dE/dbeta))."""
        p = self.p
        g = np.ascontiguousarray(gammas, dtype=np.float64).reshape(-1, p)
        b = np.ascontiguousarray(betas, dtype=np.float64).reshape(-1, p)
        npt = g.shape[0]
        E = np.zeros(npt)
        pc = np.zeros((npt, len(self.plans))) if per_edge else None
        dg = np.zeros((npt, p)) if grad else None
        db = np.zeros((npt, p)) if grad else None
        self._call(npt, g.ctypes.data, b.ctypes.data, E.ctypes.data, dg.ctypes.data if grad else None,
                   db.ctypes.data if grad else None, pc.ctypes.data if per_edge else None, stream or 0)
        out = [E]
        if per_edge:
            out.append(pc[:, self.class_of] if self.dedup else pc)
        if grad:
            out += [dg, db]
        return out[0] if len(out) == 1 else tuple(out)

    def signature(self) -> str:
        import hashlib

        return hashlib.sha1(":".join(pl.signature() for pl in self.plans).encode()).hexdigest()

    def set_tuning(self, multi_waves=0, grad_waves=0, multi_lds_cap=0, grad_lds_cap=0):
        """Launch shapes of the batched lightcone launches (read from the first plan): wavefronts
        per workgroup and LDS bytes per workgroup of the energy and of the gradient launch."""
        for pl in self.plans:
            pl.set_tuning(**dict(pl.get_tuning(), multi_waves=multi_waves, grad_waves=grad_waves,
                                 multi_lds_cap=multi_lds_cap, grad_lds_cap=grad_lds_cap))

    def energy_device(self, gammas, betas, grad=False, per_edge=False, stream=None):
        """Device-resident call: gammas/betas are float64 torch tensors [n_points, p] on the GPU.

        Returns torch tensors (E, and per-edge values, and dE/dgamma, dE/dbeta)
        written by the library on ``stream`` (default: torch's current stream).
        """
        import torch

        lib = L.load()
        g = gammas.detach().to(torch.float64).contiguous()
        b = betas.detach().to(torch.float64).contiguous()
        npt = g.shape[0]
        dev = g.device
        E = torch.empty(npt, dtype=torch.float64, device=dev)
        pe = torch.empty(npt, len(self.plans), dtype=torch.float64, device=dev) if per_edge else None
        dg = torch.empty(npt, self.p, dtype=torch.float64, device=dev) if grad else None
        db = torch.empty(npt, self.p, dtype=torch.float64, device=dev) if grad else None
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        if self.dedup and not hasattr(self, "_wdev"):
            self._wdev = torch.tensor(self.weights, dtype=torch.float64, device=dev)
        self._call(npt, g.data_ptr(), b.data_ptr(), E.data_ptr(), dg.data_ptr() if grad else None,
                   db.data_ptr() if grad else None, pe.data_ptr() if per_edge else None, s,
                   self._wdev.data_ptr() if self.dedup else None)
        out = [E]
        if per_edge:
            out.append(pe[:, torch.as_tensor(self.class_of, device=dev)] if self.dedup else pe)
        if grad:
            out += [dg, db]
        return out[0] if len(out) == 1 else tuple(out)


def _energy_function():
    import torch

    class QAOAEnergy(torch.autograd.Function):
        """E(gamma, beta) per point; backward uses the adjoint gradient that
        the same ``qt_energy_grad`` launch computes (reverse bucket
        elimination), so no second contraction runs."""

        @staticmethod
        def forward(ctx, model, gammas, betas):
            need = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
            if need:
                E, dg, db = model.energy_device(gammas, betas, grad=True)
                ctx.save_for_backward(dg, db)
            else:
                E = model.energy_device(gammas, betas)
            return E

        @staticmethod
        def backward(ctx, gE):
            dg, db = ctx.saved_tensors
            w = gE.to(torch.float64).unsqueeze(1)
            return None, w * dg, w * db

    return QAOAEnergy


_QAOA_ENERGY = None


def qaoa_energy(model: EnergyModel, gammas, betas):
    """Differentiable E per point: gammas, betas are float64 GPU tensors [n_points, p]."""
    global _QAOA_ENERGY
    if _QAOA_ENERGY is None:
        _QAOA_ENERGY = _energy_function()
    return _QAOA_ENERGY.apply(model, gammas, betas)
