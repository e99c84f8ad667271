"""Autotuner of the execution tunables (``qt_plan_set_tuning``).

Eq. (1) of the paper fixes the thread count of a pairwise product by a
formula calibrated on one machine.  Here the corresponding choices (wavefronts
per workgroup of the LDS and lightcone launches, the largest step rank run
from LDS rather than streamed) are measured: every candidate is timed with
HIP events on the caller's stream over device-resident inputs, the fastest is
kept, and the winner is cached in a JSON file keyed by device architecture,
the kind of call and the shape signature (network structure, order, slicing,
precision), so a later process applies it without measuring.

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
MULTI_WAVES = (1, 2, 4, 8, 16)


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
    """Median over `repeats` timed calls (HIP events on torch's current stream), after one untimed call."""
    import torch

    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune_plan(plan, n_points: int = 1, repeats: int = 5, cache: bool = True, waves=PLAN_WAVES,
              max_ranks=PLAN_MAX_RANK) -> dict:
    """Picks lds_waves and lds_max_rank for ``qt_contract_batch`` over all slices at n_points points.

    Returns {"lds_waves", "lds_max_rank", "ms", "measured": {...}} and applies the choice to the plan.
    """
    import numpy as np
    import torch

    from paper_2012_02430_amd import _lib as L

    key = f"{_arch()}:plan:{n_points}:{plan.signature()}"
    path = cache_path()
    if cache:
        hit = _load(path).get(key)
        if hit:
            plan.set_tuning(hit["lds_waves"], hit["lds_max_rank"])
            return dict(hit, cached=True)
    lib = L.load()
    p = max(1, plan.p)
    rng = np.random.default_rng(0)
    g = torch.tensor(rng.uniform(0, np.pi, (n_points, p)), dtype=torch.float64, device="cuda")
    b = torch.tensor(rng.uniform(0, np.pi, (n_points, p)), dtype=torch.float64, device="cuda")
    arr = (L.ctypes.c_void_p * 1)(plan.handle.value)
    n_slices = plan.n_slices
    stream = torch.cuda.current_stream().cuda_stream
    outd = torch.empty(n_points * 3, dtype=torch.float64, device="cuda")

    def call():
        L.check(lib.qt_contract_batch(arr, 1, n_points, g.data_ptr(), b.data_ptr(), 0, n_slices,
                                      L.ctypes.cast(outd.data_ptr(), L.ctypes.POINTER(L.qt_amp)), None, stream))

    measured = {}
    best = None
    for w in waves:
        for r in max_ranks:
            plan.set_tuning(w, r)
            ms = _time_ms(call, repeats)
            measured[f"{w}/{r}"] = ms
            if best is None or ms < best[0]:
                best = (ms, w, r)
    ms, w, r = best
    plan.set_tuning(w, r)
    res = {"lds_waves": w, "lds_max_rank": r, "ms": ms, "measured": measured, "t": time.time()}
    if cache:
        _store(path, key, res)
    return dict(res, cached=False)


def tune_energy(model, n_points: int, grad: bool = False, repeats: int = 5, cache: bool = True,
                waves=MULTI_WAVES) -> dict:
    """Picks the wavefronts per workgroup of ``qt_energy_grad``'s batched launch (energy or gradient)."""
    import numpy as np
    import torch

    kind = "grad" if grad else "energy"
    key = f"{_arch()}:{kind}:{n_points}:{model.signature()}"
    path = cache_path()

    def apply(w):
        t = model.plans[0].get_tuning()
        model.set_tuning(w if not grad else t["multi_waves"], w if grad else t["grad_waves"])

    if cache:
        hit = _load(path).get(key)
        if hit:
            apply(hit["waves"])
            return dict(hit, cached=True)
    rng = np.random.default_rng(0)
    g = torch.tensor(rng.uniform(0, np.pi, (n_points, model.p)), dtype=torch.float64, device="cuda")
    b = torch.tensor(rng.uniform(0, np.pi, (n_points, model.p)), dtype=torch.float64, device="cuda")
    measured = {}
    best = None
    for w in waves:
        apply(w)
        ms = _time_ms(lambda: model.energy_device(g, b, grad=grad), repeats)
        measured[str(w)] = ms
        if best is None or ms < best[0]:
            best = (ms, w)
    ms, w = best
    apply(w)
    res = {"waves": w, "ms": ms, "measured": measured, "t": time.time()}
    if cache:
        _store(path, key, res)
    return dict(res, cached=False)
