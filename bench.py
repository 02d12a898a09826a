"""Benchmark of the AHPP hot path on one MI355X.

Workload (one "step"): 1,024 eps-approximate single-source AHPP queries at
eps = 1e-7, k = 50, answered by one ahpp_query_batch call on the synthetic
power-law graph |U| = 1M, |V| = 500k, 20M edges (Zipf 2.1 degrees, weights
U[0.5, 1]), 10,000 attributes with 20 per U node (Zipf 1.5 popularity, values
in (0, 1]).  Sources: half uniform from the top 1% of U by degree, half
uniform over U.  Inputs are generated on the host and loaded into HBM before
the timed region; the timed region covers the whole batch (rounds of
Algorithm 4 and the top-k) for `--steps` batches.

Also reported: the plain single-query push on the same GPU (100 sources drawn
proportional to degree) with p50 / p99 latency; per-query completion times
inside the batch; a serving sweep of the continuous-batching server on the
5M/2M/100M serving graph (capacity, then Poisson arrivals at four offered
rates up past it; sources proportional to degree, eps uniform on {1e-5,
1e-6, 1e-7, 1e-8}; latency from arrival to top-k on the host); the roofline
of the dominant gather kernel (compulsory bytes / HIP-event time, against
8 TB/s HBM, beside the counter-measured traffic); the load of the
20M/10M/500M graph without and with the lambda cache; and the CPU oracle's
FP64 ASRP on a sample of the batch's own sources.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AHPP queries/s at ε=1e-7, batched vs plain push; p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILES = {"kb_gather<back>": os.path.join(ROOT, "profiles", "kb_gather_back_m1_traffic.json"),
                 "kb_gather<fwd>": os.path.join(ROOT, "profiles", "kb_gather_fwd_m1_traffic.json"),
                 "kb_hot_dense": os.path.join(ROOT, "profiles", "kb_hot_dense_m1_traffic.json")}
# The batched kernels and what fixes their schedules (constants, hot rows,
# work items): a counter summary is used only if taken on these exact files.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2512_11606_amd", "csrc", f)
                  for f in ("batch.hip", "hot_dense.hip", "ahpp_internal.h", "graph_build.hip")]


def _percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def _source_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel_kind_name):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = TRAFFIC_FILES.get(kernel_kind_name)
    if not path or not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel") != kernel_kind_name or d.get("source_sha256_16") != _source_hash(KERNEL_SOURCES):
        return None
    return d.get("bytes_per_launch")


def _cpu_model():
    """The host CPU's model name as lscpu prints it (/proc/cpuinfo if lscpu is missing)."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_SAMPLE = 16        # queries of the headline batch timed on the host
CPU_THREADS_MAX = 16   # the host share of one GPU


def cpu_baseline(g, batch_sources, eps, batch_rows=None):
    """The oracle's FP64 ASRP (lambda from Theorem 3) on the host cores, on a
    sample of the headline batch's own sources (as many of its hub sources as
    of its uniform ones): one query per thread; the value is the sample over
    the wall time, latency the per-query thread times.  batch_rows (query
    index -> the batch's score row): the observed error of those rows
    against the oracle's exact series, max |pi - pi_hat| / eps."""
    import numpy as np

    import oracle
    half = len(batch_sources) // 2
    n = min(CPU_SAMPLE, len(batch_sources))
    sample = np.concatenate([batch_sources[: n // 2], batch_sources[half: half + n - n // 2]]).astype(np.int32)
    og = oracle.OracleGraph.from_graph(g)
    lam = og.lambda_thm3()
    nth = max(1, min(oracle.max_threads(), CPU_THREADS_MAX, sample.size))
    t0 = time.perf_counter()
    _, stats, bad = og.asrp_many(sample, eps, lam, nthreads=nth)
    dtn = time.perf_counter() - t0
    secs = sorted(og.last_secs.tolist())
    observed = None
    if batch_rows:
        observed = {}
        for q, row in batch_rows.items():
            exact, _ = og.power_series(int(batch_sources[q]))
            observed[str(q)] = round(float(np.abs(exact - row).max()) / eps, 4)
    og.close()
    return {"value": round(sample.size / dtn, 3), "unit": "queries/s", "cores": nth, "kind": "oracle",
            "observed_error_over_eps": observed,
            "latency_ms_p50": round(_percentile(secs, 50) * 1e3, 1),
            "latency_ms_p99": round(_percentile(secs, 99) * 1e3, 1),
            "rounds_mean": round(sum(st.iterations for st in stats) / len(stats), 1), "failed": bad,
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"{sample.size} sources of the timed batch ({n // 2} of its top-1% hub sources, "
                      f"{n - n // 2} of its uniform ones), full FP64 ASRP at eps {eps:g} with lambda from "
                      f"Theorem 3, one query per thread on {nth} threads: {dtn:.1f} s wall; latency = each "
                      f"query's own thread time (p99 of {sample.size} is about the maximum)"}


SERVE_EPS = (1e-5, 1e-6, 1e-7, 1e-8)


# The paper's ASRP times on its Amazon graph at eps = 1e-6 (scalability
# figure, 100% of the graph, one CPU thread of a Xeon Silver 4210): the two
# sampling modes give 158,896 ms and 188,102 ms per query.
PAPER_AMAZON_ASRP_MS = (158896.0, 188102.0)


def amazon_leg(ahpp, synth, g, n=16):
    """Plain single-query latency on the Amazon-shaped graph at eps = 1e-6 (the
    oracle's time on one of the same queries is in the CPU baseline leg)."""
    dg = ahpp.load_graph(g, device=0)
    srcs = synth.degree_queries(g, n, 2005)
    ahpp.ahpp_query(dg, int(srcs[0]), 1e-6, k=50)
    lat = []
    for s in srcs.tolist():
        a = time.perf_counter()
        ahpp.ahpp_query(dg, s, 1e-6, k=50, want_pi=False, want_stats=False)
        lat.append((time.perf_counter() - a) * 1e3)
    out = {"workload": "plain single-query push, eps 1e-6, k 50, on a synthetic graph of the paper's Amazon sizes "
                       "(2.3M/8.0M/22.5M, 800 attributes x 10)",
           "queries": n, "latency_ms_p50": round(_percentile(lat, 50), 2),
           "latency_ms_p99": round(_percentile(lat, 99), 2), "lambda": round(dg.lam, 2),
           "paper_asrp_ms_amazon": list(PAPER_AMAZON_ASRP_MS)}
    dg.free()
    return out


SCALING_FRACS = (0.5, 0.6, 0.7, 0.8, 0.9, 1.0)


def scaling_leg(ahpp, synth, g_full, n=4, eps=1e-6):
    """Exp-3 on the Amazon-shaped graph: U nodes, or edges, sampled at 50% to
    100% with their attributes; plain ASRP and APP at eps = 1e-6, k 50, mean
    per query over n degree-weighted sources of each sampled graph (load and
    lambda excluded)."""
    out = {"workload": f"Amazon-shaped graph sampled by U nodes or by edges at 50-100% (with the kept nodes' "
                       f"attributes); plain ASRP and APP at eps {eps:g}, k 50, {n} degree-weighted sources per graph",
           "points": []}
    for mode in ("nodes", "edges"):
        for f in SCALING_FRACS:
            if mode == "edges" and f == 1.0:
                continue  # the whole graph, already measured under "nodes"
            g = g_full if f == 1.0 else synth.sample_graph(g_full, f, mode, seed=3000)
            dg = ahpp.load_graph(g, device=0)
            srcs = synth.degree_queries(g, n, 2008).tolist()
            pt = {"mode": mode, "frac": f, "n_u": g.n_u, "n_v": g.n_v, "m_e": g.m_e, "m_a": g.m_a,
                  "lambda": round(dg.lam, 1)}
            for sch, name in ((0, "ASRP"), (1, "APP")):
                ahpp.ahpp_query_schedule(dg, srcs[0], eps, sch, k=50, want_pi=False)
                lat, rounds = [], []
                for s in srcs:
                    a = time.perf_counter()
                    r = ahpp.ahpp_query_schedule(dg, s, eps, sch, k=50, want_pi=False)
                    lat.append((time.perf_counter() - a) * 1e3)
                    rounds.append(r.stats[0]["iters"])
                pt[name] = {"ms_mean": round(sum(lat) / n, 2), "rounds_mean": round(sum(rounds) / n, 1)}
            dg.free()
            del g
            out["points"].append(pt)
    return out


def mc_leg(ahpp, synth, g, dg, eps=1e-3, p_f=1e-6):
    """Monte Carlo walks at the sample size that gives an eps-approximate row
    with probability 1 - p_f (Section 3.1), beside the push at the same eps."""
    import math
    walks = int(math.ceil(2.0 * (1.0 + eps / 3.0) * math.log(g.n_u / p_f) / eps ** 2))
    src = int(synth.degree_queries(g, 1, 2006)[0])
    ahpp.ahpp_query_mc(dg, src, 1 << 20, seed=1)  # builds the draw tables
    t0 = time.perf_counter()
    res = ahpp.ahpp_query_mc(dg, src, walks, seed=2, k=50)
    mc_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    ahpp.ahpp_query(dg, src, eps, k=50)
    push_ms = (time.perf_counter() - t0) * 1e3
    st = res["stats"]
    return {"workload": f"one source, eps {eps:g} with failure probability {p_f:g}: {walks} walks",
            "walks": walks, "ms": round(mc_ms, 1), "walks_per_s": round(walks / (mc_ms / 1e3), 1),
            "steps_per_s": round(st["steps"] / (mc_ms / 1e3), 1), "push_ms_same_eps": round(push_ms, 2)}


SCHEDULE_NAMES = ("ASRP", "APP", "APP(S)", "APP(E)")


def schedule_leg(ahpp, synth, g, dg, n=4, eps_list=(1e-6, 1e-7)):
    """Exp-2's comparison on the loaded graph: the same sources under ASRP,
    APP (r_max = eps / (|E| + |E_A|)), APP(S) and APP(E), plain path, k 50."""
    srcs = synth.degree_queries(g, n, 2007).tolist()
    out = {"workload": f"{n} degree-weighted sources per eps, plain single-query path, k 50", "eps": {}}
    for eps in eps_list:
        row = {}
        for sch, name in enumerate(SCHEDULE_NAMES):
            ahpp.ahpp_query_schedule(dg, srcs[0], eps, sch, k=50, want_pi=False)
            lat, rounds, sw, pushes = [], [], [], []
            for s in srcs:
                a = time.perf_counter()
                r = ahpp.ahpp_query_schedule(dg, s, eps, sch, k=50, want_pi=False)
                lat.append((time.perf_counter() - a) * 1e3)
                st = r.stats[0]
                rounds.append(st["iters"]); sw.append(st["sync_switch_iter"]); pushes.append(st["n_push"])
            row[name] = {"ms_mean": round(sum(lat) / n, 2), "rounds_mean": round(sum(rounds) / n, 1),
                         "switch_round": sw, "pushes_mean": round(sum(pushes) / n)}
        out["eps"][f"{eps:g}"] = row
    return out


def tiny_leg(ahpp, synth, n=200):
    """Plain single-query latency on the 2k/1k/20k graph (the small parity
    workload), where launch overhead rather than HBM decides the time."""
    g = synth.make_graph("tiny")
    dg = ahpp.load_graph(g, device=0)
    srcs = synth.uniform_queries(g, n, 2000)
    ahpp.ahpp_query(dg, int(srcs[0]), 1e-6, k=20)
    lat = []
    for s in srcs.tolist():
        a = time.perf_counter()
        ahpp.ahpp_query(dg, s, 1e-6, k=20, want_pi=False, want_stats=False)
        lat.append((time.perf_counter() - a) * 1e3)
    dg.free()
    return {"workload": "plain single-query push, 2k/1k/20k unit-weight graph with 100 attributes x 5, eps 1e-6, k 20",
            "queries": n, "latency_ms_p50": round(_percentile(lat, 50), 3),
            "latency_ms_p99": round(_percentile(lat, 99), 3), "queries_per_s": round(n / (sum(lat) / 1e3), 1)}


def prep_cache_leg(ahpp, synth, name="large20m"):
    """Graph load on the 20M/10M/500M graph without and with the lambda
    cache: the first load builds the CSRs and runs Theorem 3's sweeps, then
    files lambda under the key of the inputs; the second load of the same
    inputs reads it back instead of sweeping."""
    import shutil
    import tempfile
    t = time.perf_counter()
    g = synth.make_graph(name)
    gen_s = time.perf_counter() - t
    print(f"[bench] generated {name} in {gen_s:.1f} s", file=sys.stderr, flush=True)
    d = tempfile.mkdtemp(prefix="ahpp-cache-")
    out = {"workload": f"load of {name} ({g.n_u}/{g.n_v}/{g.m_e} edges, {g.m_a} attribute entries) from host COO, "
                       f"fresh then from the lambda cache", "generate_s": round(gen_s, 1)}
    try:
        for leg in ("fresh", "cached"):
            t = time.perf_counter()
            dg = ahpp.load_graph(g, device=0, cache_dir=d)
            wall = time.perf_counter() - t
            info = ahpp.ahpp_graph_info(dg)
            out[leg] = {"wall_s": round(wall, 2), "build_ms": round(info["load_ms"], 1),
                        "lambda_ms": round(info["lambda_ms"], 1), "lambda_cached": info["lambda_cached"],
                        "device_bytes": info["device_bytes"]}
            print(f"[bench] {name} load ({leg}): {wall:.2f} s", file=sys.stderr, flush=True)
            dg.free()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    return out


SWEEP_FRACS = (0.3, 0.6, 0.9, 1.3)   # offered load as a fraction of the measured capacity
LOW_LOAD_QPS, LOW_LOAD_QUERIES = 2.0, 40   # a low arrival rate, served without and with solo queries


def serve_sweep_leg(ahpp, synth, args):
    """Continuous batching on the 5M/2M/100M serving graph: capacity from a
    closed burst (every query queued at once), then Poisson arrivals at
    fractions of it, the last one past it; per rate p50 / p99 latency from
    arrival to top-k on the host.  Then a low rate, batched and with lone
    queries answered on the single-query engine."""
    from paper_2512_11606_amd import serve
    t_gen = time.perf_counter()
    g = synth.make_graph(args.serve_graph)
    dg = ahpp.load_graph(g, device=0)
    load_s = time.perf_counter() - t_gen
    n = args.serve_queries
    n_burst = 2 * args.serve_slots
    total = n_burst + n * len(SWEEP_FRACS) + 2 * LOW_LOAD_QUERIES
    sources = synth.degree_queries(g, total, 2003)
    pick = (synth.CounterRNG(2003, "serve_eps").uniform(total) * len(SERVE_EPS)).astype(int)
    eps = [SERVE_EPS[min(i, len(SERVE_EPS) - 1)] for i in pick]
    srv = ahpp.Server(dg, k=50, max_slots=args.serve_slots)
    out = {"workload": f"serving on {args.serve_graph} ({g.n_u}/{g.n_v}/{g.m_e} edges, {g.n_attr} attributes x "
                       f"{g.m_a // g.n_u}), sources proportional to degree, eps uniform on "
                       f"{list(SERVE_EPS)}, k 50, {srv.info()['slots']} slots, {args.serve_rounds} rounds per step",
           "graph_gen_and_load_s": round(load_s, 1), "rates": []}
    try:
        print(f"[bench] serving burst of {n_burst}", file=sys.stderr, flush=True)
        summ, res = serve.run(srv, sources[:n_burst], eps[:n_burst], rate_qps=1e9,
                              rounds_per_step=args.serve_rounds, max_wall_s=300.0)
        cap = summ["served_qps"]
        out["capacity_qps"] = round(cap, 2)
        out["burst"] = {kk: (round(v, 2) if isinstance(v, float) else v) for kk, v in summ.items()}
        for i, frac in enumerate(SWEEP_FRACS):
            lo = n_burst + i * n
            rate = frac * cap
            print(f"[bench] serving {n} queries at {rate:.1f} q/s", file=sys.stderr, flush=True)
            summ, res = serve.run(srv, sources[lo:lo + n], eps[lo:lo + n], rate_qps=rate,
                                  rounds_per_step=args.serve_rounds, seed=3003 + i, max_wall_s=300.0)
            summ["converged"] = sum(1 for r in res.values() if r["stats"]["converged"] == 1)
            summ["load_fraction"] = frac
            out["rates"].append({kk: (round(v, 2) if isinstance(v, float) else v) for kk, v in summ.items()})
        # Low load: the same arrivals batched in the tiles, then with lone
        # queries on the single-query engine (ahpp_server_set_solo).
        out["low_load"] = []
        for j, solo in enumerate((0, 4)):
            lo = n_burst + len(SWEEP_FRACS) * n + j * LOW_LOAD_QUERIES
            srv.set_solo(solo)
            print(f"[bench] serving {LOW_LOAD_QUERIES} queries at {LOW_LOAD_QPS} q/s, solo_max {solo}",
                  file=sys.stderr, flush=True)
            summ, res = serve.run(srv, sources[lo:lo + LOW_LOAD_QUERIES], eps[lo:lo + LOW_LOAD_QUERIES],
                                  rate_qps=LOW_LOAD_QPS, rounds_per_step=args.serve_rounds, seed=3100 + j,
                                  max_wall_s=300.0)
            summ["converged"] = sum(1 for r in res.values() if r["stats"]["converged"] == 1)
            summ["solo_max"] = solo
            out["low_load"].append({kk: (round(v, 2) if isinstance(v, float) else v) for kk, v in summ.items()})
        srv.set_solo(0)
    finally:
        srv.close()
        dg.free()
    out["note"] = (f"offered 2k-50k queries/s is {2000 / max(cap, 1e-9):.0f}x-{50000 / max(cap, 1e-9):.0f}x "
                   f"the measured capacity of one GPU on this graph")
    return out


def amazon_cpu_leg(synth, n=16):
    """The oracle's FP64 ASRP, one thread, on the first source of the
    Amazon-shaped latency leg (eps 1e-6): context for the paper's figure."""
    import oracle
    g = synth.make_graph("amazon")
    src = int(synth.degree_queries(g, n, 2005)[0])
    og = oracle.OracleGraph.from_graph(g)
    lam = og.lambda_thm3()
    t0 = time.perf_counter()
    _, _, st, _ = og.asrp(src, 1e-6, lam)
    out = {"source": src, "ms_one_thread": round((time.perf_counter() - t0) * 1e3, 1), "rounds": st.iterations}
    og.close()
    return out


def roofline_of(prof, names):
    """Roofline of the kernel kind with the most time: compulsory bytes per
    launch over its mean HIP-event time, against the HBM peak; beside it the
    gathered-model rate and, if a counter summary of the current kernel
    source is committed, the measured traffic and its ratio to compulsory."""
    dom_kind = max(prof, key=lambda kk: prof[kk]["ms"])
    dom = prof[dom_kind]
    name = names[dom_kind]
    launches = max(dom["launches"], 1)
    avg_ms = dom["ms"] / launches
    comp = dom["compulsory"] / launches
    gathered = dom["bytes"] / launches
    achieved = comp / (avg_ms * 1e-3) / 1e9
    traffic = _traffic(name)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
           "launches": dom["launches"], "avg_ms": round(avg_ms, 4), "compulsory_bytes_per_launch": comp,
           "gathered_bytes_per_launch": gathered,
           "gathered_GBps": round(gathered / (avg_ms * 1e-3) / 1e9, 1)}
    if traffic:
        out["traffic_GBps"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        out["traffic_frac"] = round(out["traffic_GBps"] / HBM_PEAK_GBS, 4)
        out["wasted_traffic"] = round(traffic / comp, 3)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--plain", type=int, default=100, help="plain single queries timed for latency")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--no-tiny", action="store_true", help="skip the small-graph latency run")
    ap.add_argument("--no-tune", action="store_true", help="keep the untuned batch schedule")
    ap.add_argument("--no-amazon", action="store_true", help="skip the Amazon-shaped latency and scaling runs")
    ap.add_argument("--no-scaling", action="store_true", help="skip the 50-100%% sampled-graph scaling run")
    ap.add_argument("--no-mc", action="store_true", help="skip the Monte Carlo run")
    ap.add_argument("--no-schedules", action="store_true", help="skip the ASRP / APP / APP(S) / APP(E) comparison")
    ap.add_argument("--no-prep", action="store_true", help="skip the 20M-node load with and without the lambda cache")
    ap.add_argument("--serve-graph", default="serve5m")
    ap.add_argument("--serve-queries", type=int, default=500, help="queries per offered rate of the sweep")
    ap.add_argument("--serve-slots", type=int, default=512)
    ap.add_argument("--serve-rounds", type=int, default=4, help="rounds per server step")
    ap.add_argument("--graph", default="m1")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: queries are independent, the figure is one GPU's share, and "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2512_11606_amd import ahpp, synth

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    eps, k = 1e-7, 50
    g = synth.make_graph(args.graph)
    dg = ahpp.load_graph(g, device=0)
    torch.cuda.synchronize()
    ginfo = ahpp.ahpp_graph_info(dg)
    graph_load = {"build_ms": round(ginfo["load_ms"], 1), "lambda_ms": round(ginfo["lambda_ms"], 1),
                  "lambda_iters": ginfo["lambda_iters"], "device_bytes": ginfo["device_bytes"],
                  "note": "host COO to device CSR, numbering, hot lists and Theorem 3 lambda; outside the timed steps"}
    sources = synth.mixed_batch_queries(g, args.batch, 2002)
    tuned = None if args.no_tune else ahpp.ahpp_graph_tune(dg, max_tiles=max(1, args.batch // 256))

    say("warmup")
    for _ in range(args.warmup):
        ahpp.ahpp_query_batch(dg, sources, eps, k=k, want_pi=False, want_stats=False)
    torch.cuda.synchronize()

    say("timed steps")
    ahpp.ahpp_profile_enable(dg, True)
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        res = ahpp.ahpp_query_batch(dg, sources, eps, k=k, want_pi=False, want_stats=False)
        step_ms.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {kind: ahpp.ahpp_profile_read(dg, kind)
            for kind in (ahpp.PROF_BATCH_BACK, ahpp.PROF_BATCH_FWD, ahpp.PROF_BATCH_HOT)}
    ahpp.ahpp_profile_enable(dg, False)
    elapsed = t1 - t0
    value = args.batch * args.steps / elapsed
    topk_ok = int(res.topk_n.min().item()) == k

    # Per-query completion inside one more (untimed) batch: the round at which
    # each query's stop rule held, as a share of the batch's rounds, times the
    # batch time (every result is returned when the call returns).
    say("per-query statistics")
    st_res = ahpp.ahpp_query_batch(dg, sources, eps, k=k, want_pi=True, want_stats=True)
    sample_q = sorted({0, args.batch // 2 - 1, args.batch // 2, args.batch - 1})
    batch_rows = {q: st_res.pi[q].cpu().numpy().astype(np.float64) for q in sample_q}
    st_res.pi = None
    iters = np.array([st["iters"] for st in st_res.stats], dtype=np.float64)
    batch_ms = float(st_res.stats[0]["ms"])
    done_ms = iters / iters.max() * batch_ms
    completion = {"p50": round(float(np.percentile(done_ms, 50)), 1), "p99": round(float(np.percentile(done_ms, 99)), 1),
                  "rounds_min": int(iters.min()), "rounds_max": int(iters.max()),
                  "note": "each query's stop round / the batch's rounds x the batch's device time; the call returns "
                          "all results together"}

    # Plain single-query push: per-query latency (host call to results).
    say("plain queries")
    plain_src = synth.degree_queries(g, args.plain, 2001)
    ahpp.ahpp_query(dg, int(plain_src[0]), eps, k=k)
    lat = []
    for s_ in plain_src.tolist():
        a = time.perf_counter()
        ahpp.ahpp_query(dg, s_, eps, k=k, want_pi=False, want_stats=False)
        lat.append((time.perf_counter() - a) * 1e3)
    plain_qps = len(lat) / (sum(lat) / 1e3)

    plain_tiny = monte_carlo = schedules = None
    if not args.no_tiny:
        say("small graph")
        plain_tiny = tiny_leg(ahpp, synth)
    if not args.no_mc:
        say("monte carlo")
        monte_carlo = mc_leg(ahpp, synth, g, dg)
    if not args.no_schedules:
        say("push schedules")
        schedules = schedule_leg(ahpp, synth, g, dg)
    names = {ahpp.PROF_BATCH_BACK: "kb_gather<back>", ahpp.PROF_BATCH_FWD: "kb_gather<fwd>",
             ahpp.PROF_BATCH_HOT: "kb_hot_dense"}
    roofline = roofline_of(prof, names)
    kernels = {names[kk]: {"launches": prof[kk]["launches"],
                           "avg_ms": round(prof[kk]["ms"] / max(prof[kk]["launches"], 1), 4),
                           "compulsory_GBps": round(prof[kk]["compulsory"] / max(prof[kk]["ms"], 1e-9) / 1e6, 1),
                           "gathered_GBps": round(prof[kk]["bytes"] / max(prof[kk]["ms"], 1e-9) / 1e6, 1)}
               for kk in names}
    dg.free()
    amazon = scaling = None
    if not args.no_amazon:
        say("amazon-shaped graph")
        g_am = synth.make_graph("amazon")
        amazon = amazon_leg(ahpp, synth, g_am)
        scaling = None if args.no_scaling else scaling_leg(ahpp, synth, g_am)
        del g_am
    serving = None
    if not args.no_serve:
        say("serving sweep")
        serving = serve_sweep_leg(ahpp, synth, args)
    preprocessing = None
    if not args.no_prep:
        say("20M-node load, fresh and cached")
        preprocessing = prep_cache_leg(ahpp, synth)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched AHPP queries, {args.batch} per batch, eps=1e-7, k=50, on the 1M/500k/20M "
                               "Zipf(2.1) bipartite graph with 10k attributes x 20 (Zipf 1.5)",
                   "graph": args.graph, "n_u": g.n_u, "n_v": g.n_v, "m_e": g.m_e, "n_attr": g.n_attr, "m_a": g.m_a,
                   "eps": eps, "k": k, "batch": args.batch, "alpha": 0.15, "beta": 0.35,
                   "lambda": round(ginfo["lam"], 3)},
        "precision": "residues, reserves and carries float32; pushes handed between half-steps as bfloat16 rounded "
                     "toward zero, the exact remainder kept in the float32 state (Theorem 2's bound holds as stated)",
        "hip_graphs": "off: the batch runs plain launches (replaying a captured round measured no faster)",
        "batch_call_ms_p50": round(_percentile(step_ms, 50), 2),
        "batch_call_ms_p99": round(_percentile(step_ms, 99), 2),
        "batch_query_completion_ms": completion,
        "plain_qps": round(plain_qps, 2),
        "plain_queries": len(lat),
        "plain_latency_ms_p50": round(_percentile(lat, 50), 2),
        "plain_latency_ms_p99": round(_percentile(lat, 99), 2),
        "batched_over_plain": round(value / plain_qps, 2),
        "topk_complete": topk_ok,
        "graph_load": graph_load,
        "preprocessing_20m": preprocessing,
        "tuned_schedule": tuned,
        "serving": serving,
        "plain_tiny": plain_tiny,
        "amazon_shaped": amazon,
        "monte_carlo": monte_carlo,
        "push_schedules": schedules,
        "amazon_scaling": scaling,
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu:
        say("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(g, sources, eps, batch_rows)
        out["observed_error_over_eps"] = out["cpu_baseline"]["observed_error_over_eps"]
        if not args.no_amazon:
            out["cpu_baseline"]["amazon_shaped"] = amazon_cpu_leg(synth)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
