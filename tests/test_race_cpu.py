"""The race driver of Algorithm 1 with stand-in legs (no GPU): the first leg
that finishes wins at the next poll and every other leg is stopped."""

import time

from paper_2607_03627_amd.race import Leg, LegResult, run_race


class FakeLeg(Leg):
    def __init__(self, name, finish_after, ok=True):
        self.name = name
        self.finish_after = finish_after
        self.ok = ok
        self.stopped = False

    def start(self):
        self.t0 = time.perf_counter()

    def poll(self):
        dt = time.perf_counter() - self.t0
        if self.finish_after is not None and dt >= self.finish_after:
            return LegResult(self.name, self.ok, dt, "OPTIMAL" if self.ok else "FAILED", 1.0)
        return None

    def stop(self):
        self.stopped = True


def test_first_finisher_wins_and_the_other_is_stopped():
    fast, slow = FakeLeg("fast", 0.05), FakeLeg("slow", None)
    r = run_race([slow, fast], poll_s=0.02, timeout_s=5)
    assert r.winner == "fast"
    assert slow.stopped and not fast.stopped
    assert [x.status for x in r.results] == ["TERMINATED", "OPTIMAL"]


def test_a_leg_that_fails_does_not_win():
    bad, good = FakeLeg("bad", 0.01, ok=False), FakeLeg("good", 0.08)
    r = run_race([bad, good], poll_s=0.02, timeout_s=5)
    assert r.winner == "good"
    assert r.results[0].status == "FAILED"


def test_timeout_without_winner():
    a, b = FakeLeg("a", None), FakeLeg("b", None)
    r = run_race([a, b], poll_s=0.02, timeout_s=0.1)
    assert r.winner is None and a.stopped and b.stopped
