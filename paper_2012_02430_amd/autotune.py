"""Autotuner of the execution tunables (``qt_plan_set_tuning``).

Eq. (1) of the paper fixes the thread count of a pairwise product by a
formula calibrated on one machine.  Here the corresponding choices are
measured: wavefronts per workgroup of the LDS and lightcone launches, the
largest step rank run from LDS rather than streamed, output tiles per
workgroup of the streaming step and fused GEMM kernels, the LDS bytes per
workgroup of the batched lightcone launch (lightcones needing more run from
global scratch), and, at plan build time, the smallest bucket rank fused into
an MFMA GEMM.  Every candidate is timed with HIP events on the caller's
stream over device-resident inputs, the fastest is kept, and the winner is
cached in a JSON file keyed by device architecture, the kind of call and the
shape signature (network structure, order, slicing, precision), so a later
process applies it without measuring.  Grids are searched one coordinate
group at a time (launch shape and rank threshold jointly, then each tile
count with the others fixed).

Cache file: ``$QT_TUNE_CACHE``, else ``$XDG_CACHE_HOME/qtensor_hip/tune.json``
(``~/.cache/...``).  Tuning changes speed only; results stay within the
stated tolerances.
"""
from __future__ import annotations

import json
import os
import time
from pathlib import Path

PLAN_WAVES = (4, 8, 16)
PLAN_MAX_RANK = (10, 12, 14, 16)
STEP_TILES = (1, 2, 4, 8, 16)
GEMM_TILES = (1, 2, 4, 8, 16, 32)
MULTI_WAVES = (1, 2, 4, 8)
MULTI_LDS_CAPS = (4096, 8192, 12288, 16384, 24576, 32768, 49152, 65536, 163840)
GEMM_MIN_RANKS = (8, 10, 12, 14, 16)


def cache_path() -> Path:
    if os.environ.get("QT_TUNE_CACHE"):
        return Path(os.environ["QT_TUNE_CACHE"])
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return Path(base) / "qtensor_hip" / "tune.json"


def _load(path: Path) -> dict:
    try:
        return json.loads(path.read_text())
    except (OSError, ValueError):
        return {}


def _store(path: Path, key: str, value: dict) -> None:
    try:
        path.parent.mkdir(parents=True, exist_ok=True)
        data = _load(path)
        data[key] = value
        tmp = path.with_suffix(".tmp")
        tmp.write_text(json.dumps(data, indent=1, sort_keys=True))
        tmp.replace(path)
    except OSError:
        pass  # a read-only cache location only costs re-measuring


def _arch() -> str:
    import torch

    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu").split(":")[0]


def _time_ms(fn, repeats: int) -> float:
    """Milliseconds per call in steady state: the median over three runs of `repeats` back-to-back calls
    (HIP events on torch's current stream around each run), after two untimed calls (the first may build
    the call's device state).  Back-to-back calls are how the work is used; a call timed alone after an
    idle GPU can rank launch shapes differently."""
    import torch

    fn()
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(repeats):
            fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / repeats)
    times.sort()
    return times[1]


def _plan_caller(plan, n_points):
    import numpy as np
    import torch

    from paper_2012_02430_amd import _lib as L

    lib = L.load()
    p = max(1, plan.p)
    rng = np.random.default_rng(0)
    g = torch.tensor(rng.uniform(0, np.pi, (n_points, p)), dtype=torch.float64, device="cuda")
    b = torch.tensor(rng.uniform(0, np.pi, (n_points, p)), dtype=torch.float64, device="cuda")
    arr = (L.ctypes.c_void_p * 1)(plan.handle.value)
    n_slices = plan.n_slices
    stream = torch.cuda.current_stream().cuda_stream
    outd = torch.empty((n_points << len(plan.open_vars)) * 3, dtype=torch.float64, device="cuda")

    def call():
        L.check(lib.qt_contract_batch(arr, 1, n_points, g.data_ptr(), b.data_ptr(), 0, n_slices,
                                      L.ctypes.cast(outd.data_ptr(), L.ctypes.POINTER(L.qt_amp)), None, stream))

    return call


def tune_plan(plan, n_points: int = 1, repeats: int = 5, cache: bool = True, waves=PLAN_WAVES,
              max_ranks=PLAN_MAX_RANK, step_tiles=STEP_TILES, gemm_tiles=GEMM_TILES) -> dict:
    """Picks lds_waves, lds_max_rank, step_tiles and gemm_tiles for ``qt_contract_batch`` over all
    slices at n_points points: (lds_waves, lds_max_rank) on their grid, then step_tiles, then
    gemm_tiles (skipped when the plan has no step or GEMM launch to time).

    Returns the chosen tunables with "ms" and "measured" ({candidate: ms}) and applies them.
    """
    names = ("lds_waves", "lds_max_rank", "step_tiles", "gemm_tiles")
    key = f"{_arch()}:plan2:{n_points}:{plan.signature()}"
    path = cache_path()
    if cache:
        hit = _load(path).get(key)
        if hit:
            plan.set_tuning(**{k: hit[k] for k in names})
            return dict(hit, cached=True)
    call = _plan_caller(plan, n_points)
    measured = {}
    cur = dict.fromkeys(names, 0)

    def run(**kw):
        t = dict(cur, **kw)
        plan.set_tuning(**t)
        ms = _time_ms(call, repeats)
        measured["/".join(str(t[k]) for k in names)] = ms
        return ms

    best = min((run(lds_waves=w, lds_max_rank=r), w, r) for w in waves for r in max_ranks)
    cur.update(lds_waves=best[1], lds_max_rank=best[2])
    ms = best[0]
    st = plan.describe().get("stream_steps", [])
    groups = []
    if any("gemm" not in s and s["rank"] > 10 for s in st):  # several 1024-element tiles per item
        groups.append(("step_tiles", step_tiles))
    if any("gemm" in s for s in st):
        groups.append(("gemm_tiles", gemm_tiles))
    for name, cands in groups:
        b = min((run(**{name: v}), v) for v in cands)
        if b[0] < ms:
            ms = b[0]
            cur[name] = b[1]
    plan.set_tuning(**cur)
    res = dict(cur, ms=ms, measured=measured, t=time.time())
    if cache:
        _store(path, key, res)
    return dict(res, cached=False)


def tune_gemm_min_rank(network, order, groups=(), precision="c64_mfma_fp32", n_points: int = 1, repeats: int = 3,
                       ranks=GEMM_MIN_RANKS, **plan_kw):
    """Builds the plan once per candidate ``gemm_min_rank`` (the smallest bucket output rank fused
    into an MFMA GEMM, a plan build choice) and returns (fastest plan, {rank: ms})."""
    from paper_2012_02430_amd import api

    measured, best = {}, None
    for r in ranks:
        plan = api.Plan(network, order, groups, precision=precision, gemm_min_rank=r, **plan_kw)
        ms = _time_ms(_plan_caller(plan, n_points), repeats)
        measured[r] = ms
        if best is None or ms < best[0]:
            best = (ms, plan)
        else:
            del plan
    return best[1], measured


def tune_energy(model, n_points: int, grad: bool = False, repeats: int = 5, cache: bool = True,
                waves=MULTI_WAVES, caps=MULTI_LDS_CAPS) -> dict:
    """Picks the wavefronts per workgroup and the LDS bytes per workgroup of ``qt_energy_grad``'s
    batched launch (energy or gradient, each with its own pair of tunables) on their joint grid."""
    import numpy as np
    import torch

    kind = "grad" if grad else "energy"
    key = f"{_arch()}:{kind}2:{n_points}:{model.signature()}"
    path = cache_path()

    def apply(w, cap):
        t = model.plans[0].get_tuning()
        if grad:
            model.set_tuning(t["multi_waves"], w, t["multi_lds_cap"], cap)
        else:
            model.set_tuning(w, t["grad_waves"], cap, t["grad_lds_cap"])

    if cache:
        hit = _load(path).get(key)
        if hit:
            apply(hit["waves"], hit["lds_cap"])
            return dict(hit, cached=True)
    rng = np.random.default_rng(0)
    g = torch.tensor(rng.uniform(0, np.pi, (n_points, model.p)), dtype=torch.float64, device="cuda")
    b = torch.tensor(rng.uniform(0, np.pi, (n_points, model.p)), dtype=torch.float64, device="cuda")
    measured = {}
    best = None
    for cap in caps:
        for w in waves:
            apply(w, cap)
            ms = _time_ms(lambda: model.energy_device(g, b, grad=grad), repeats)
            measured[f"{w}/{cap}"] = ms
            if best is None or ms < best[0]:
                best = (ms, w, cap)
    ms, w, cap = best
    apply(w, cap)
    res = {"waves": w, "lds_cap": cap, "ms": ms, "measured": measured, "t": time.time()}
    if cache:
        _store(path, key, res)
    return dict(res, cached=False)
