"""Serving driver: Poisson query arrivals into the continuous-batching server.

The server (ahpp_server_* in include/ahpp.h, C++ in csrc/serve.hip) owns the
device work: admission into free slots, shared rounds, collection.  This
driver only plays the clients: it submits each query at its arrival time,
steps the server while work is pending, and records each query's latency
from arrival to the moment its top-k reaches the host.
"""

from __future__ import annotations

import math
import time
from typing import Optional, Sequence

import numpy as np

from . import ahpp
from .synth import CounterRNG


def poisson_arrivals(n: int, rate_qps: float, seed: int) -> np.ndarray:
    """Arrival offsets (seconds) of n queries with exponential gaps of mean 1/rate."""
    u = CounterRNG(seed, "arrivals").uniform(n)
    gaps = -np.log1p(-u) / float(rate_qps)
    return np.cumsum(gaps)


def run(server: "ahpp.Server", sources: Sequence[int], eps: Sequence[float], rate_qps: float,
        rounds_per_step: int = 4, seed: int = 3003, want_pi: bool = False, max_wall_s: Optional[float] = None):
    """Serves len(sources) queries arriving as a Poisson stream; returns
    (summary dict, results by tag)."""
    n = len(sources)
    arrivals = poisson_arrivals(n, rate_qps, seed)
    finished = {}
    t0 = time.perf_counter()
    nxt = 0
    steps = 0
    while len(finished) < n:
        now = time.perf_counter() - t0
        if max_wall_s is not None and now > max_wall_s:
            break
        while nxt < n and arrivals[nxt] <= now:
            server.submit(nxt, int(sources[nxt]), float(eps[nxt]))
            nxt += 1
        info = server.info()
        if info["running"] == 0 and info["queued"] == 0 and info["ready"] == 0:
            if nxt == n:  # everything submitted, nothing left in the server
                missing = sorted(set(range(n)) - set(finished))
                raise RuntimeError(f"server finished without returning {len(missing)} queries "
                                   f"(first tags {missing[:5]})")
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
            continue
        server.step(rounds_per_step)
        steps += 1
        done_at = time.perf_counter() - t0
        for r in server.results(max_n=4096, want_pi=want_pi):
            finished[r["tag"]] = (done_at, r)
    lat = np.array([(finished[i][0] - arrivals[i]) * 1e3 for i in sorted(finished)])
    end = max(v[0] for v in finished.values()) if finished else 0.0
    summary = {
        "offered_qps": float(rate_qps),
        "queries": n,
        "completed": len(finished),
        "served_qps": len(finished) / end if end > 0 else 0.0,
        "latency_ms_p50": float(np.percentile(lat, 50)) if lat.size else math.nan,
        "latency_ms_p99": float(np.percentile(lat, 99)) if lat.size else math.nan,
        "latency_ms_max": float(lat.max()) if lat.size else math.nan,
        "steps": steps,
        "rounds_per_step": rounds_per_step,
        "slots": server.info()["slots"],
    }
    return summary, {t: r for t, (_, r) in finished.items()}
