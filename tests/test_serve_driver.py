"""The Poisson serving driver against a host-only stand-in for the server
(no GPU): every query is submitted at its arrival time and collected once,
latencies are measured from arrival, and a server that loses a query makes
the driver fail instead of waiting forever."""

import numpy as np
import pytest

from paper_2512_11606_amd import serve


class FakeServer:
    """Admits up to `slots` queries; each finishes `rounds` rounds after admission."""

    def __init__(self, slots=8, rounds=6, drop=None):
        self.slots, self.rounds, self.drop = slots, rounds, drop
        self.queue, self.running, self.ready = [], {}, []
        self.submitted = []

    def submit(self, tag, source, eps):
        assert eps > 0
        self.submitted.append(tag)
        self.queue.append((tag, source))

    def info(self):
        return {"slots": self.slots, "running": len(self.running), "queued": len(self.queue),
                "ready": len(self.ready)}

    def step(self, rounds):
        while self.queue and len(self.running) < self.slots:
            tag, source = self.queue.pop(0)
            self.running[tag] = (source, 0)
        for tag in list(self.running):
            source, done = self.running[tag]
            done += rounds
            if done >= self.rounds:
                del self.running[tag]
                if tag != self.drop:
                    self.ready.append({"tag": tag, "topk_idx": np.array([source]), "stats": {"converged": 1}})
            else:
                self.running[tag] = (source, done)
        return len(self.ready)

    def results(self, max_n=1024, want_pi=False):
        out, self.ready = self.ready[:max_n], self.ready[max_n:]
        return out


def test_poisson_arrivals_are_seeded_with_the_given_rate():
    a = serve.poisson_arrivals(20000, 500.0, 7)
    assert np.array_equal(a, serve.poisson_arrivals(20000, 500.0, 7))
    assert not np.array_equal(a, serve.poisson_arrivals(20000, 500.0, 8))
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert (gaps >= 0).all()
    # Exponential gaps: mean 1/rate within 3 standard errors (sd = mean / sqrt(n)).
    assert abs(gaps.mean() * 500.0 - 1.0) < 3.0 / np.sqrt(gaps.size)


def test_every_query_is_served_once():
    srv = FakeServer(slots=4, rounds=8)
    srcs = np.arange(40) * 3
    summary, res = serve.run(srv, srcs, [1e-6] * 40, rate_qps=2000.0, rounds_per_step=4)
    assert summary["completed"] == 40 and sorted(res) == list(range(40))
    assert srv.submitted == list(range(40))
    assert all(int(res[t]["topk_idx"][0]) == 3 * t for t in res)
    assert 0 < summary["latency_ms_p50"] <= summary["latency_ms_p99"] <= summary["latency_ms_max"]
    assert summary["slots"] == 4 and summary["steps"] >= 40 // 4 * 2


def test_a_lost_query_is_reported():
    srv = FakeServer(slots=4, rounds=4, drop=5)
    with pytest.raises(RuntimeError, match="without returning 1 queries"):
        serve.run(srv, np.arange(12), [1e-6] * 12, rate_qps=5000.0)
