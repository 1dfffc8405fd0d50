"""Host logic of the overlapped step (no GPU): the worker thread that a side
context keeps for the branch after the column pivots, and the ratio taken
from the device pair of residual sums."""
from __future__ import annotations

import threading

import pytest

torch = pytest.importorskip("torch")

from paper_2104_05877_amd import rpid as R  # noqa: E402


def test_worker_runs_jobs_in_order_on_one_thread():
    w = R._SideWorker()
    try:
        idents = []
        for i in range(5):
            w.start(lambda i=i: (idents.append(threading.get_ident()), i * i)[1])
            assert w.result() == i * i
        # one thread, started once, not the caller's
        assert len(set(idents)) == 1 and idents[0] != threading.get_ident()
    finally:
        w.stop()
    assert not w._thread.is_alive()


def test_worker_runs_beside_the_caller():
    """The job waits for a signal the caller gives only after start() has
    returned: it runs concurrently, or the result would never come."""
    w = R._SideWorker()
    go, seen = threading.Event(), threading.Event()
    try:
        def job():
            seen.set()
            assert go.wait(timeout=10.0)
            return "done"

        w.start(job)
        assert seen.wait(timeout=10.0)
        go.set()
        assert w.result() == "done"
    finally:
        w.stop()


def test_worker_reraises_in_the_caller_and_keeps_serving():
    w = R._SideWorker()
    try:
        def bad():
            raise ValueError("side branch failed")

        w.start(bad)
        with pytest.raises(ValueError, match="side branch failed"):
            w.result()
        w.start(lambda: 7)
        assert w.result() == 7
    finally:
        w.stop()
    assert not w._thread.is_alive()


def test_stop_lets_a_started_job_finish():
    """stop() right after start(), before the result is taken: the job still
    runs to its end, its result stays available, and the thread ends."""
    w = R._SideWorker()
    release, ran = threading.Event(), []

    def job():
        assert release.wait(timeout=10.0)
        ran.append(True)
        return 5

    w.start(job)
    timer = threading.Timer(0.2, release.set)
    timer.start()
    w.stop()
    timer.join()
    assert ran == [True] and w.result() == 5
    assert not w._thread.is_alive()


def test_relative_residual_from_sums():
    assert R._relative(torch.tensor([4.0, 16.0], dtype=torch.float64)) == 0.5
    assert R._relative(torch.tensor([0.0, 9.0], dtype=torch.float64)) == 0.0
    # a zero matrix has no relative residual: reported as 0
    assert R._relative(torch.tensor([0.0, 0.0], dtype=torch.float64)) == 0.0
