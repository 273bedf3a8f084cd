"""The server's admission rule, on the host (no GPU): lg_admission_simulate
drives the same decision function the worker threads use, with a simulated
clock and fixed service times."""

import numpy as np
import pytest

from paper_2010_15879_amd import lg

GB = 1 << 30


def replay_check(arrival, need, service, start, finish, status, budget, resident, workers):
    """Independent check of a schedule: FIFO starts, at most `workers` at once,
    and held memory (grow-only per worker, reclaimed only when idle) within
    the budget at every start."""
    ok = [i for i in range(len(arrival)) if status[i] == 0]
    for i in range(1, len(ok)):
        assert start[ok[i]] >= start[ok[i - 1]] - 1e-12          # FIFO
    for i in ok:
        assert start[i] >= arrival[i] - 1e-12
        assert abs(finish[i] - start[i] - service[i]) < 1e-9
        running = [j for j in ok if start[j] <= start[i] < finish[j]]
        assert len(running) <= workers
        assert resident + sum(need[j] for j in running) <= budget  # at least what runs must fit


def test_everything_fits_runs_immediately():
    arrival = [0.0, 0.1, 0.2, 0.3]
    need = [1 * GB] * 4
    service = [1.0] * 4
    st, fi, ss, peak = lg.admission_simulate(arrival, need, service, 100 * GB, 10 * GB, 8)
    assert ss == [0, 0, 0, 0]
    assert st == arrival
    assert peak == 14 * GB


def test_budget_serializes_and_is_never_exceeded():
    rng = np.random.default_rng(3)
    n = 200
    arrival = np.sort(rng.uniform(0, 50, n)).tolist()
    need = rng.integers(1, 40, n).astype(np.uint64) * (GB // 4)
    service = rng.uniform(0.1, 2.0, n).tolist()
    budget, resident = 30 * GB, 18 * GB
    st, fi, ss, peak = lg.admission_simulate(arrival, need.tolist(), service, budget, resident, 8)
    assert peak <= budget
    for i in range(n):
        if resident + int(need[i]) > budget:
            assert ss[i] != 0            # can never fit: rejected
        else:
            assert ss[i] == 0
    replay_check(arrival, need.tolist(), service, st, fi, ss, budget, resident, 8)


def test_worker_count_bounds_concurrency():
    n = 50
    arrival = [0.0] * n
    need = [1] * n
    service = [1.0] * n
    st, fi, ss, peak = lg.admission_simulate(arrival, need, service, 1 << 40, 0, 4)
    assert all(s == 0 for s in ss)
    # 4 workers, 50 unit jobs released together: waves of 4
    assert max(fi) == pytest.approx(np.ceil(n / 4))


def test_work_conserving_under_tight_budget():
    # two jobs that cannot run together: the second starts exactly when the first ends
    st, fi, ss, peak = lg.admission_simulate([0.0, 0.0], [6 * GB, 6 * GB], [2.0, 3.0], 10 * GB, 0, 4)
    assert ss == [0, 0]
    assert st == [0.0, 2.0] and fi == [2.0, 5.0]
    assert peak == 6 * GB
