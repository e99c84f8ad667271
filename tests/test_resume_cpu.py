"""Resuming an interrupted sliced contraction from its journal (CPU only).

The contractor here is the oracle: per-slice values of a step-dependent
slicing plan by plain bucket elimination.  A run that fails after a few
slice ranges and is resumed from the saved journal must give bitwise the
same per-slice values and total as an uninterrupted run, and the total must
be the unsliced amplitude.
"""
import numpy as np
import pytest

import oracle
from paper_2012_02430_amd.api import SliceJournal, run_resumable
from workloads import qaoa_params, regular_graph


class Interrupted(Exception):
    pass


def _case():
    n, p = 14, 2
    edges = regular_graph(n, 3, 0)
    g, b = qaoa_params(p, 2, seed=3)
    nets = [oracle.amplitude_network(n, edges, g[i], b[i]) for i in range(2)]
    order = oracle.min_degree_order(nets[0])
    sl = order[3:7]
    rest = [v for v in order if v not in sl]
    groups = [(3, sl)]
    per = np.array([oracle.sliced_values(T, rest, groups) for T in nets])  # [points][16]
    want = np.array([oracle.contract(T) for T in nets])
    return per, want


def test_resume_after_interruption_is_bitwise_equal(tmp_path):
    per, want = _case()
    calls = []

    def contract(lo, hi):
        calls.append((lo, hi))
        return per[:, lo:hi]

    full = SliceJournal("case", 2, 16)
    tot_full = run_resumable(contract, full, max_len=3)
    assert np.allclose(tot_full, want, rtol=1e-12, atol=0)

    path = tmp_path / "journal.npz"
    state = {"n": 0}

    def failing(lo, hi):
        state["n"] += 1
        if state["n"] == 3:
            raise Interrupted()
        return per[:, lo:hi]

    j = SliceJournal("case", 2, 16)
    with pytest.raises(Interrupted):
        run_resumable(failing, j, max_len=3, path=path)
    j2 = SliceJournal.load(path, "case")
    assert j2.done.sum() == 6 and j2.missing(3)[0] == (6, 9)
    calls.clear()
    tot = run_resumable(contract, j2, max_len=3, path=path)
    assert calls[0] == (6, 9) and all(lo >= 6 for lo, _ in calls)
    assert np.array_equal(j2.values, full.values)
    assert np.array_equal(tot, tot_full)


def test_journal_rejects_a_foreign_file(tmp_path):
    j = SliceJournal("a", 1, 4)
    j.record(0, np.ones((1, 2)))
    j.save(tmp_path / "j.npz")
    with pytest.raises(ValueError):
        SliceJournal.load(tmp_path / "j.npz", "b")
    with pytest.raises(ValueError):
        j.total()
    assert j.missing() == [(2, 4)]
