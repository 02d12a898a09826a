// C ABI of the AHPP library (declared in include/ahpp.h): argument checks,
// device selection, the host side of the round loop, and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "../../include/ahpp.h"
#include "ahpp_internal.h"

struct ahpp_graph {
    ahpp::Graph g;
};

struct ahpp_server {
    ahpp::Server *impl;
};

namespace ahpp {

namespace {
thread_local std::string g_last_error;

ahpp_status_t fail(int status, const std::string &msg) {
    g_last_error = msg;
    return (ahpp_status_t)status;
}

// Runs the body of an entry point and turns every exception into a status,
// so that none unwinds through the C ABI.
template <class F>
ahpp_status_t guarded(const char *fn, F &&body) {
    try {
        return body();
    } catch (const Failure &f) {
        return fail(f.status, f.msg);
    } catch (const std::bad_alloc &) {
        return fail(AHPP_ERR_OUT_OF_MEMORY, std::string(fn) + ": host allocation failed");
    } catch (const std::exception &e) {
        return fail(AHPP_ERR_DEVICE, std::string(fn) + ": internal error: " + e.what());
    } catch (...) {
        return fail(AHPP_ERR_DEVICE, std::string(fn) + ": internal error");
    }
}

// A start/stop event pair for timing a call on its stream; destroyed with
// the object, also when the call fails half way.
struct EventPair {
    hipEvent_t start = nullptr, stop = nullptr;
    EventPair() {
        check_hip(hipEventCreate(&start), "event");
        check_hip(hipEventCreate(&stop), "event");
    }
    ~EventPair() {
        if (start) (void)hipEventDestroy(start);
        if (stop) (void)hipEventDestroy(stop);
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    float elapsed_ms() const {
        float ms = 0.0f;
        check_hip(hipEventElapsedTime(&ms, start, stop), "event");
        return ms;
    }
};

// Makes `dev` current for the lifetime of the object, restoring the
// caller's device afterwards.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) check_hip(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void ensure_topk_scratch(Graph &g, int64_t n_q) {
    size_t need = topk_scratch_bytes(n_q);
    if (g.tk_scratch_bytes >= need) return;
    if (g.tk_scratch) {
        dfree(g.tk_scratch);
        g.device_bytes -= (int64_t)g.tk_scratch_bytes;
    }
    g.tk_scratch = nullptr;
    g.tk_scratch_bytes = 0;
    g.tk_scratch = dev_alloc(g, need, "top-k scratch");
    g.tk_scratch_bytes = need;
}

// Tiles of kTileQ queries that fit in a quarter of the free device memory, at most 16.
int batch_tiles_fit(const Graph &g) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 4;
    const double per_tile = (double)batch_tile_bytes(g, true);
    int t = (int)std::floor((double)free_b * 0.25 / std::max(per_tile, 1.0));
    return std::max(1, std::min(t, 16));
}

// Tiles run side by side in one batch pass: AHPP_BATCH_TILES if set, else
// the tuned count (ahpp_graph_tune), else as many as fit.
int batch_tiles_in_flight(const Graph &g) {
    if (const char *e = std::getenv("AHPP_BATCH_TILES")) {
        int v = std::atoi(e);
        if (v > 0) return v;
    }
    if (g.tuned_tiles > 0) return g.tuned_tiles;
    return batch_tiles_fit(g);
}

int default_lambda_iters(int64_t n_u, double alpha) {
    double t = std::ceil(std::log(0.01 / (double)std::max<int64_t>(n_u, 1)) / std::log(1.0 - alpha));
    return std::max(1, (int)t);
}

// What the key of a description covers; the round count is the one the load
// uses for Theorem 3 (0 when lambda is given).
KeyInput key_input(const ahpp_graph_desc_t &d) {
    KeyInput k;
    k.n_u = d.n_u;
    k.n_v = d.n_v;
    k.n_attr = d.n_attr;
    k.n_edges = d.n_edges;
    k.n_assoc = d.n_assoc;
    k.has_ew = d.edge_w != nullptr && d.n_edges > 0;
    k.has_aw = d.assoc_w != nullptr && d.n_assoc > 0;
    k.alpha = d.alpha;
    k.beta = d.beta;
    k.lambda_iters = d.lambda > 0 ? 0 : (d.lambda_iters > 0 ? d.lambda_iters : default_lambda_iters(d.n_u, d.alpha));
    return k;
}

// The checks of a description that need no device (sizes, pointers, alpha,
// beta, lambda); ids and weights are checked on the device at load.
std::string desc_error(const ahpp_graph_desc_t *d) {
    if (d->n_u <= 0 || d->n_v < 0 || d->n_attr < 0 || d->n_edges < 0 || d->n_assoc < 0)
        return "sizes must be >= 0 and n_u >= 1";
    if (d->n_u > INT32_MAX || d->n_v > INT32_MAX || d->n_attr > INT32_MAX || 2 * d->n_u > INT32_MAX ||
        d->n_v + d->n_attr > INT32_MAX)
        return "node counts exceed the int32 id range";
    if ((d->n_edges > 0 && (!d->edge_u || !d->edge_v)) || (d->n_assoc > 0 && (!d->assoc_u || !d->assoc_a)))
        return "id arrays must not be NULL when their count is > 0";
    if (!(d->alpha > 0.0 && d->alpha < 1.0)) return "alpha must be in (0,1)";
    if (!(d->beta >= 0.0 && d->beta <= 1.0)) return "beta must be in [0,1]";
    if (std::isnan(d->lambda) || std::isinf(d->lambda)) return "lambda must be finite";
    return "";
}

// Runs rounds until the control block reports done; the host checks after
// chunks of rounds that grow from 4 to 32.
// Rounds still needed, estimated from the max residue: the synchronous phase
// shrinks it by about (1 - alpha) per round (Theorem 1's proof).
int rounds_left(const Graph &g, float max_r, float eps_f) {
    if (!(max_r > eps_f)) return 1;
    const double t = std::log((double)max_r / (double)eps_f) / std::log(1.0 / (1.0 - g.alpha));
    return (int)std::min(32.0, std::max(1.0, std::ceil(t)));
}

// Enqueues rounds in chunks sized by rounds_left until the control block
// reports done; rounds enqueued past the stop are empty launches.
void run_single(Graph &g, const QueryBufs &b, bool own, hipStream_t s) {
    int chunk = 4, launched = 0;
    Control c;
    for (;;) {
        single_query_rounds(g, b, chunk, s, own);
        launched += chunk;
        check_hip(hipMemcpyAsync(&c, b.ctl, sizeof(Control), hipMemcpyDeviceToHost, s), "poll");
        check_hip(hipStreamSynchronize(s), "poll");
        if (c.done) break;
        chunk = rounds_left(g, c.last_max, c.eps_f);
    }
    if (own && g.prof.on) {
        profiler_void_tail(g.prof, 0, launched - c.iter);
        profiler_void_tail(g.prof, 1, launched - c.iter);
    }
}

}  // namespace

void check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) throw Failure{AHPP_ERR_OUT_OF_MEMORY, std::string(what) + ": out of device memory"};
    throw Failure{AHPP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

void profiler_flush(Profiler &p) {
    for (ProfLaunch &l : p.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(l.stop) == hipSuccess && hipEventElapsedTime(&ms, l.start, l.stop) == hipSuccess) {
            p.launches[l.kind] += 1;
            p.ms[l.kind] += ms;
            p.bytes[l.kind] += l.bytes;
            p.compulsory[l.kind] += l.compulsory;
        }
        (void)hipEventDestroy(l.start);
        (void)hipEventDestroy(l.stop);
    }
    p.pending.clear();
}

// Drops the last n recorded launches of `kind`: rounds enqueued after the
// stop rule held run as empty launches and are not kernel work.
void profiler_void_tail(Profiler &p, int kind, int64_t n) {
    for (int64_t i = (int64_t)p.pending.size() - 1; i >= 0 && n > 0; --i) {
        if (p.pending[i].kind != kind) continue;
        (void)hipEventDestroy(p.pending[i].start);
        (void)hipEventDestroy(p.pending[i].stop);
        p.pending.erase(p.pending.begin() + i);
        --n;
    }
}

// With AHPP_GRAPHS=1 the rounds are replayed from captured HIP graphs.  Off
// by default: on MI355X replaying a one-round graph costs more than its
// five launches (2.14 ms against 1.90 ms per query on a 2k-node graph; the
// same on the 1M graph, where rounds are long).  Profiling needs the plain
// launches (it records events around them).
bool graphs_enabled(const Graph &g) {
    if (g.prof.on) return false;
    const char *e = std::getenv("AHPP_GRAPHS");
    return e && std::atoi(e) == 1;
}

// Records the launches issued by record() on the library's capture stream
// and returns the instantiated graph.  The recorded work must not allocate
// or memset (kernels only).
hipGraphExec_t capture_graph(Graph &g, const char *what, const std::function<void(hipStream_t)> &record) {
    if (!g.cap_stream) check_hip(hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking), what);
    check_hip(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal), what);
    try {
        record(g.cap_stream);
    } catch (...) {
        hipGraph_t partial = nullptr;
        (void)hipStreamEndCapture(g.cap_stream, &partial);
        if (partial) (void)hipGraphDestroy(partial);
        throw;
    }
    hipGraph_t graph = nullptr;
    check_hip(hipStreamEndCapture(g.cap_stream, &graph), what);
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    check_hip(e, what);
    return exec;
}

void *dev_alloc(Graph &g, size_t bytes, const char *what) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Failure{AHPP_ERR_OUT_OF_MEMORY, std::string(what) + ": hipMalloc of " + std::to_string(bytes) +
                                                   " bytes failed (" + hipGetErrorString(e) + ")"};
    }
    g.device_bytes += (int64_t)bytes;
    return p;
}

int32_t run_query(Graph &g, const QueryBufs &b, bool own, int32_t source, double eps, int32_t schedule,
                  int32_t max_iters, float *pi_out, float *resid_out, int32_t k, int32_t *topk_idx, float *topk_val,
                  int32_t *topk_n, ahpp_stats_t *stats, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<EventPair> ev;
    if (own) {
        ev.reset(new EventPair());
        check_hip(hipEventRecord(ev->start, s), "event");
    }
    const float eps_f = (float)(eps / g.lambda);
    const int32_t src = g.u_new_host[(size_t)source];
    single_query_init(g, b, src, eps_f, max_iters, s, schedule, (float)(eps / (double)(g.m_e + g.m_a)));
    run_single(g, b, own, s);
    // Scores in input order (the top-k breaks ties by input id).
    float *scores = pi_out ? pi_out : (k > 0 ? b.out : nullptr);
    if (scores) to_input_order(g, b.pi, scores, s);
    if (k > 0)
        topk_launch(scores, g.n_u, 0, 1, nullptr, source, k, topk_idx, topk_val, topk_n, b.tk ? b.tk : g.tk_scratch,
                    s);
    if (resid_out) to_input_order(g, b.r, resid_out, s);
    if (ev) check_hip(hipEventRecord(ev->stop, s), "event");
    Control ctl;
    check_hip(hipMemcpyAsync(&ctl, b.ctl, sizeof(Control), hipMemcpyDeviceToHost, s), "control D2H");
    check_hip(hipStreamSynchronize(s), "query");
    const float ms = ev ? ev->elapsed_ms()
                        : (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                              .count();
    if (stats) {
        double sum_r = 0.0;
        single_query_stats(g, b, &sum_r, s);
        stats->iters = ctl.iter;
        stats->sync_switch_iter = ctl.switch_iter;
        stats->converged = ctl.status == 1;
        stats->reserved = 0;
        stats->n_push = (int64_t)ctl.n_p;
        stats->max_residual = ctl.last_max;
        stats->sum_residual = sum_r;
        stats->ms = ms;
        stats->pad = 0;
    }
    return ctl.status;
}

}  // namespace ahpp

using namespace ahpp;

extern "C" {

const char *ahpp_last_error(void) { return g_last_error.c_str(); }

ahpp_status_t ahpp_server_create(ahpp_graph_t *h, int64_t max_device_bytes, int32_t max_slots, int32_t k,
                                 int32_t max_iters, int32_t keep_pi, ahpp_server_t **out) {
    g_last_error.clear();
    if (!h || !out) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_create: NULL argument");
    *out = nullptr;
    if (k < 1 || k > kMaxTopK) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_create: k must be in [1, 2048]");
    return guarded("ahpp_server_create", [&] {
        DeviceScope scope(h->g.device);
        std::unique_ptr<Server> impl(new Server(h->g, max_device_bytes, max_slots, k, max_iters, keep_pi != 0));
        *out = new ahpp_server{impl.get()};
        impl.release();
        return AHPP_OK;
    });
}

void ahpp_server_free(ahpp_server_t *srv) {
    if (!srv) return;
    try {
        if (srv->impl) {
            DeviceScope scope(srv->impl->graph().device);
            (void)hipDeviceSynchronize();
            delete srv->impl;
        }
    } catch (...) {
    }
    delete srv;
}

ahpp_status_t ahpp_server_submit(ahpp_server_t *srv, int64_t tag, int32_t source, double eps) {
    g_last_error.clear();
    if (!srv || !srv->impl) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_submit: NULL server");
    if (source < 0 || source >= srv->impl->graph().n_u)
        return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_submit: source out of range");
    if (!(eps > 0.0) || std::isinf(eps)) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_submit: eps must be > 0");
    return guarded("ahpp_server_submit", [&] {
        srv->impl->submit(tag, source, eps);
        return AHPP_OK;
    });
}

ahpp_status_t ahpp_server_step(ahpp_server_t *srv, int32_t rounds, int32_t *n_ready, void *hip_stream) {
    g_last_error.clear();
    if (!srv || !srv->impl) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_step: NULL server");
    if (rounds < 0) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_step: rounds < 0");
    return guarded("ahpp_server_step", [&] {
        DeviceScope scope(srv->impl->graph().device);
        const int n = srv->impl->step(rounds, (hipStream_t)hip_stream);
        if (n_ready) *n_ready = n;
        return AHPP_OK;
    });
}

ahpp_status_t ahpp_server_results(ahpp_server_t *srv, int32_t max_n, int64_t *tags, int32_t *topk_idx,
                                  float *topk_val, int32_t *topk_n, ahpp_stats_t *stats, float *pi_out,
                                  int32_t *n_out, void *hip_stream) {
    g_last_error.clear();
    if (!srv || !srv->impl || !n_out) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_results: NULL argument");
    if (max_n < 0) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_results: max_n < 0");
    return guarded("ahpp_server_results", [&] {
        DeviceScope scope(srv->impl->graph().device);
        *n_out = srv->impl->results(max_n, tags, topk_idx, topk_val, topk_n, stats, pi_out, (hipStream_t)hip_stream);
        return AHPP_OK;
    });
}

ahpp_status_t ahpp_server_set_solo(ahpp_server_t *srv, int32_t solo_max) {
    g_last_error.clear();
    if (!srv || !srv->impl) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_set_solo: NULL server");
    if (solo_max < 0 || solo_max > kTileQ)
        return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_set_solo: solo_max must be in [0, 256]");
    srv->impl->set_solo(solo_max);
    return AHPP_OK;
}

ahpp_status_t ahpp_server_info(const ahpp_server_t *srv, int32_t *slots, int32_t *running, int32_t *queued,
                               int32_t *ready) {
    g_last_error.clear();
    if (!srv || !srv->impl) return fail(AHPP_ERR_INVALID_ARG, "ahpp_server_info: NULL server");
    srv->impl->info(slots, running, queued, ready);
    return AHPP_OK;
}

ahpp_status_t ahpp_graph_tune(ahpp_graph_t *h, int32_t max_tiles, ahpp_tune_info_t *out, void *hip_stream) {
    g_last_error.clear();
    if (!h) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_tune: NULL graph");
    Graph &g = h->g;
    return guarded("ahpp_graph_tune", [&] {
        DeviceScope scope(g.device);
        int cap = batch_tiles_fit(g);
        if (max_tiles > 0) cap = std::min(cap, (int)max_tiles);
        const TuneResult r = batch_tune(g, cap, (hipStream_t)hip_stream);
        if (out) *out = ahpp_tune_info_t{r.tiles, r.wg_mult, r.candidates, 0, r.ms_per_tile_round,
                                         r.default_ms_per_tile_round};
        return AHPP_OK;
    });
}

ahpp_status_t ahpp_profile_enable(ahpp_graph_t *h, int32_t on) {
    g_last_error.clear();
    if (!h) return fail(AHPP_ERR_INVALID_ARG, "ahpp_profile_enable: NULL graph");
    Profiler &p = h->g.prof;
    const ahpp_status_t rc = guarded("ahpp_profile_enable", [&] {
        DeviceScope scope(h->g.device);
        profiler_flush(p);
        return AHPP_OK;
    });
    if (rc != AHPP_OK) return rc;
    if (on) {
        for (int k = 0; k < kProfKinds; ++k) {
            p.launches[k] = 0;
            p.ms[k] = 0.0;
            p.bytes[k] = 0.0;
            p.compulsory[k] = 0.0;
        }
    }
    p.on = on != 0;
    return AHPP_OK;
}

ahpp_status_t ahpp_profile_read(ahpp_graph_t *h, int32_t kind, int64_t *launches, double *total_ms,
                                double *algo_bytes, double *compulsory_bytes) {
    g_last_error.clear();
    if (!h) return fail(AHPP_ERR_INVALID_ARG, "ahpp_profile_read: NULL graph");
    if (kind < 0 || kind >= kProfKinds) return fail(AHPP_ERR_INVALID_ARG, "ahpp_profile_read: bad kind");
    Profiler &p = h->g.prof;
    const ahpp_status_t rc = guarded("ahpp_profile_read", [&] {
        DeviceScope scope(h->g.device);
        profiler_flush(p);
        return AHPP_OK;
    });
    if (rc != AHPP_OK) return rc;
    if (launches) *launches = p.launches[kind];
    if (total_ms) *total_ms = p.ms[kind];
    if (algo_bytes) *algo_bytes = p.bytes[kind];
    if (compulsory_bytes) *compulsory_bytes = p.compulsory[kind];
    return AHPP_OK;
}

ahpp_status_t ahpp_graph_load(const ahpp_graph_desc_t *d, ahpp_graph_t **out) {
    g_last_error.clear();
    if (!d || !out) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_load: desc and out must not be NULL");
    *out = nullptr;
    const std::string bad = desc_error(d);
    if (!bad.empty()) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_load: " + bad);
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev <= 0)
        return fail(AHPP_ERR_DEVICE, "ahpp_graph_load: no HIP device");
    if (d->device < 0 || d->device >= n_dev) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_load: bad device ordinal");
    std::unique_ptr<ahpp_graph> hp(new (std::nothrow) ahpp_graph());
    if (!hp) return fail(AHPP_ERR_OUT_OF_MEMORY, "ahpp_graph_load: host allocation failed");
    Graph &g = hp->g;
    g.device = d->device;
    g.n_u = d->n_u;
    g.n_v = d->n_v;
    g.n_a = d->n_attr;
    g.m_e = d->n_edges;
    g.m_a = d->n_assoc;
    g.alpha = d->alpha;
    g.beta = d->beta;
    hipStream_t s = nullptr;
    const ahpp_status_t rc = guarded("ahpp_graph_load", [&] {
        DeviceScope scope(g.device);
        check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
        int n_cu = 0;
        check_hip(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, g.device), "device attributes");
        g.n_cu = n_cu > 0 ? n_cu : 1;
        g.grid_cap = g.n_cu * kBlocksPerCu;
        noalloc_setup(g.device);
        const KeyInput kin = key_input(*d);
        build_graph(g, d->edge_u, d->edge_v, d->edge_w, d->assoc_u, d->assoc_a, d->assoc_w, kin, s);
        alloc_query_state(g);
        ensure_topk_scratch(g, 1);
        if (d->lambda > 0) {
            g.lambda = d->lambda;
            g.lambda_iters = 0;
        } else {
            auto t0 = std::chrono::steady_clock::now();
            g.lambda_iters = kin.lambda_iters;
            const std::string dir = d->cache_dir ? d->cache_dir : "";
            if (!dir.empty() && lambda_cache_read(dir, kin, g.key, &g.lambda)) {
                g.lambda_cached = 1;
            } else {
                g.lambda = compute_lambda(g, g.lambda_iters, s) * (1.0 + 1e-4);
                if (!dir.empty()) g.lambda_cached = lambda_cache_write(dir, kin, g.key, g.lambda) ? 2 : -1;
            }
            g.lambda_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        check_hip(hipStreamSynchronize(s), "load");
        check_hip(hipStreamDestroy(s), "stream");
        s = nullptr;
        return AHPP_OK;
    });
    if (rc != AHPP_OK) {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        try {
            DeviceScope scope(g.device);
            free_graph(g);
        } catch (...) {
        }
        return rc;
    }
    *out = hp.release();
    return AHPP_OK;
}

ahpp_status_t ahpp_graph_info(const ahpp_graph_t *h, ahpp_graph_info_t *info) {
    g_last_error.clear();
    if (!h || !info) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_info: NULL argument");
    const Graph &g = h->g;
    info->n_u = g.n_u;
    info->n_v = g.n_v_input;
    info->n_attr = g.n_a;
    info->n_edges = g.m_e;
    info->n_assoc = g.m_a;
    info->alpha = g.alpha;
    info->beta = g.beta;
    info->lambda = g.lambda;
    info->lambda_iters = g.lambda_iters;
    info->device = g.device;
    info->dangling_u = g.dangling_u;
    info->device_bytes = g.device_bytes;
    info->load_ms = g.load_ms;
    info->lambda_ms = g.lambda_ms;
    info->key[0] = g.key[0];
    info->key[1] = g.key[1];
    info->lambda_cached = g.lambda_cached;
    info->hot_rows = g.hot.n;
    return AHPP_OK;
}

ahpp_status_t ahpp_graph_key(const ahpp_graph_desc_t *d, uint64_t *key) {
    g_last_error.clear();
    if (!d || !key) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_key: desc and key must not be NULL");
    const std::string bad = desc_error(d);
    if (!bad.empty()) return fail(AHPP_ERR_INVALID_ARG, "ahpp_graph_key: " + bad);
    return guarded("ahpp_graph_key", [&] {
        const KeyInput kin = key_input(*d);
        coo_key_host(kin, d->edge_u, d->edge_v, kin.has_ew ? d->edge_w : nullptr, d->assoc_u, d->assoc_a,
                     kin.has_aw ? d->assoc_w : nullptr, key);
        return AHPP_OK;
    });
}

void ahpp_graph_free(ahpp_graph_t *h) {
    if (!h) return;
    try {
        DeviceScope scope(h->g.device);
        (void)hipDeviceSynchronize();
        profiler_flush(h->g.prof);
        free_graph(h->g);
    } catch (...) {
    }
    delete h;
}

namespace {
ahpp_status_t query_impl(const char *name, ahpp_graph_t *h, int32_t source, double eps, int32_t schedule,
                         int32_t max_iters, float *pi_out, float *resid_out, int32_t k, int32_t *topk_idx,
                         float *topk_val, int32_t *topk_n, ahpp_stats_t *stats, void *hip_stream) {
    g_last_error.clear();
    const std::string fn(name);
    if (!h) return fail(AHPP_ERR_INVALID_ARG, fn + ": NULL graph");
    Graph &g = h->g;
    if (source < 0 || source >= g.n_u) return fail(AHPP_ERR_INVALID_ARG, fn + ": source out of range");
    if (!(eps > 0.0) || std::isinf(eps)) return fail(AHPP_ERR_INVALID_ARG, fn + ": eps must be > 0 and finite");
    if (k < 0 || k > kMaxTopK) return fail(AHPP_ERR_INVALID_ARG, fn + ": k must be in [0, 2048]");
    if (k > 0 && (!topk_idx || !topk_val || !topk_n))
        return fail(AHPP_ERR_INVALID_ARG, fn + ": top-k outputs required when k > 0");
    if (schedule < 0 || schedule > 3) return fail(AHPP_ERR_INVALID_ARG, fn + ": schedule must be 0..3");
    if (max_iters <= 0) max_iters = 100000;
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t status = 0;
    const ahpp_status_t rc = guarded(name, [&] {
        DeviceScope scope(g.device);
        status = run_query(g, g.q, true, source, eps, schedule, max_iters, pi_out, resid_out, k, topk_idx, topk_val,
                           topk_n, stats, s);
        return AHPP_OK;
    });
    if (rc != AHPP_OK) return rc;
    if (status != 1) return fail(AHPP_ERR_NOT_CONVERGED, fn + ": max_iters reached before the stop rule held");
    return AHPP_OK;
}
}  // namespace

ahpp_status_t ahpp_query(ahpp_graph_t *h, int32_t source, double eps, int32_t max_iters, float *pi_out,
                         float *resid_out, int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n,
                         ahpp_stats_t *stats, void *hip_stream) {
    return query_impl("ahpp_query", h, source, eps, 0, max_iters, pi_out, resid_out, k, topk_idx, topk_val, topk_n,
                      stats, hip_stream);
}

ahpp_status_t ahpp_query_noalloc(ahpp_graph_t *h, int32_t source, double eps, int32_t max_iters, float *pi_out,
                                 float *resid_out, int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n,
                                 ahpp_stats_t *stats, void *hip_stream) {
    g_last_error.clear();
    const std::string fn("ahpp_query_noalloc");
    if (!h) return fail(AHPP_ERR_INVALID_ARG, fn + ": NULL graph");
    Graph &g = h->g;
    if (source < 0 || source >= g.n_u) return fail(AHPP_ERR_INVALID_ARG, fn + ": source out of range");
    if (!(eps > 0.0) || std::isinf(eps)) return fail(AHPP_ERR_INVALID_ARG, fn + ": eps must be > 0 and finite");
    if (k < 0 || k > kMaxTopK) return fail(AHPP_ERR_INVALID_ARG, fn + ": k must be in [0, 2048]");
    if (k > 0 && (!topk_idx || !topk_val || !topk_n))
        return fail(AHPP_ERR_INVALID_ARG, fn + ": top-k outputs required when k > 0");
    const size_t need = query_bufs_bytes(g);
    if (need > kNoallocScratchBytes)
        return fail(AHPP_ERR_INVALID_ARG, fn + ": the graph needs " + std::to_string(need) +
                                              " bytes of query scratch, above the fixed " +
                                              std::to_string(kNoallocScratchBytes) + " (use ahpp_query)");
    if (max_iters <= 0) max_iters = 100000;
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t status = 0;
    const ahpp_status_t rc = guarded("ahpp_query_noalloc", [&] {
        DeviceScope scope(g.device);
        void *base = noalloc_scratch(g.device);
        if (!base) throw Failure{AHPP_ERR_DEVICE, fn + ": scratch of the device was not set up"};
        const QueryBufs b = carve_query_bufs(g, base);
        status = run_query(g, b, false, source, eps, 0, max_iters, pi_out, resid_out, k, topk_idx, topk_val, topk_n,
                           stats, s);
        return AHPP_OK;
    });
    if (rc != AHPP_OK) return rc;
    if (status != 1) return fail(AHPP_ERR_NOT_CONVERGED, fn + ": max_iters reached before the stop rule held");
    return AHPP_OK;
}

ahpp_status_t ahpp_query_schedule(ahpp_graph_t *h, int32_t source, double eps, int32_t schedule, int32_t max_iters,
                                  float *pi_out, float *resid_out, int32_t k, int32_t *topk_idx, float *topk_val,
                                  int32_t *topk_n, ahpp_stats_t *stats, void *hip_stream) {
    return query_impl("ahpp_query_schedule", h, source, eps, schedule, max_iters, pi_out, resid_out, k, topk_idx,
                      topk_val, topk_n, stats, hip_stream);
}

ahpp_status_t ahpp_query_mc(ahpp_graph_t *h, int32_t source, int64_t n_walks, uint64_t seed, float *pi_out,
                            int32_t k, int32_t *topk_idx, float *topk_val, int32_t *topk_n, ahpp_mc_stats_t *stats,
                            void *hip_stream) {
    g_last_error.clear();
    if (!h) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_mc: NULL graph");
    Graph &g = h->g;
    if (source < 0 || source >= g.n_u) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_mc: source out of range");
    // Stop counts are 32-bit and no node collects more stops than there are
    // walks, so n_walks <= 2^32 - 1 keeps every count exact.
    if (n_walks < 1 || n_walks > (int64_t)UINT32_MAX)
        return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_mc: n_walks must be in [1, 2^32 - 1]");
    if (k < 0 || k > kMaxTopK) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_mc: k must be in [0, 2048]");
    if (k > 0 && (!topk_idx || !topk_val || !topk_n))
        return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_mc: top-k outputs required when k > 0");
    hipStream_t s = (hipStream_t)hip_stream;
    return guarded("ahpp_query_mc", [&] {
        DeviceScope scope(g.device);
        ensure_mc_tables(g, s);
        EventPair ev;
        check_hip(hipEventRecord(ev.start, s), "event");
        // Counts in the residue buffer, scores in the reserve buffer.
        unsigned *count = reinterpret_cast<unsigned *>(g.q.r);
        const McResult r = mc_walks(g, g.u_new_host[(size_t)source], n_walks, seed, 4096, count, s);
        float *scores = pi_out ? pi_out : g.q.pi;
        mc_scores(count, g.u_new, g.n_u, n_walks, scores, s);
        if (k > 0) topk_launch(scores, g.n_u, 0, 1, nullptr, source, k, topk_idx, topk_val, topk_n, g.tk_scratch, s);
        check_hip(hipEventRecord(ev.stop, s), "event");
        check_hip(hipStreamSynchronize(s), "walks");
        const float ms = ev.elapsed_ms();
        if (stats) *stats = ahpp_mc_stats_t{n_walks, r.lost, r.truncated, r.steps, ms, 0.0f};
        return AHPP_OK;
    });
}

ahpp_status_t ahpp_query_batch(ahpp_graph_t *h, int32_t n_q, const int32_t *sources, const double *eps,
                               int32_t max_iters, float *pi_out, int32_t k, int32_t *topk_idx, float *topk_val,
                               int32_t *topk_n, ahpp_stats_t *stats, void *hip_stream) {
    g_last_error.clear();
    if (!h) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: NULL graph");
    Graph &g = h->g;
    if (n_q < 0) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: n_q < 0");
    if (n_q == 0) return AHPP_OK;
    if (!sources || !eps) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: sources and eps required");
    for (int32_t q = 0; q < n_q; ++q) {
        if (sources[q] < 0 || sources[q] >= g.n_u) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: source out of range");
        if (!(eps[q] > 0.0) || std::isinf(eps[q])) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: eps must be > 0");
    }
    if (k < 0 || k > kMaxTopK) return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: k must be in [0, 2048]");
    if (k > 0 && (!topk_idx || !topk_val || !topk_n))
        return fail(AHPP_ERR_INVALID_ARG, "ahpp_query_batch: top-k outputs required when k > 0");
    if (max_iters <= 0) max_iters = 100000;
    hipStream_t s = (hipStream_t)hip_stream;
    bool all_converged = true;
    const ahpp_status_t rc = guarded("ahpp_query_batch", [&] {
        DeviceScope scope(g.device);
        const int tiles_total = (int)((n_q + kTileQ - 1) / kTileQ);
        const int tif = std::min(tiles_total, batch_tiles_in_flight(g));
        // The query-major score buffer is needed only when pi_out is absent.
        ensure_batch_state(g, g.batch, tif, pi_out == nullptr);
        if (k > 0) ensure_topk_scratch(g, (int64_t)tif * kTileQ);
        std::vector<float> eps_f((size_t)n_q);
        for (int32_t q = 0; q < n_q; ++q) eps_f[q] = (float)(eps[q] / g.lambda);
        // Sources on the device for the top-k's exclusion; freed in stream
        // order when the call ends, also on failure.
        struct StreamBuf {
            int32_t *p = nullptr;
            hipStream_t s;
            ~StreamBuf() {
                if (p) (void)hipFreeAsync(p, s);
            }
        } d_src{nullptr, s};
        check_hip(hipMallocAsync((void **)&d_src.p, (size_t)n_q * 4, s), "batch sources");
        check_hip(hipMemcpyAsync(d_src.p, sources, (size_t)n_q * 4, hipMemcpyHostToDevice, s), "batch sources");
        EventPair ev;
        check_hip(hipEventRecord(ev.start, s), "event");
        std::vector<TileCtl> ctl((size_t)tif);
        std::vector<double> sums((size_t)tif * kTileQ);
        std::vector<ahpp_stats_t> st_all(stats ? (size_t)n_q : 0);
        for (int64_t q0 = 0; q0 < n_q; q0 += (int64_t)tif * kTileQ) {
            const int64_t nq = std::min<int64_t>((int64_t)tif * kTileQ, n_q - q0);
            const int nt = (int)((nq + kTileQ - 1) / kTileQ);
            batch_init(g, g.batch, nt, sources + q0, eps_f.data() + q0, nq, max_iters, s);
            g.batch.live_q = nq;
            int chunk = 4, launched = 0, executed = 0;
            for (;;) {
                batch_rounds(g, g.batch, nt, chunk, s);
                launched += chunk;
                check_hip(hipMemcpyAsync(ctl.data(), g.batch.ctl, (size_t)nt * sizeof(TileCtl), hipMemcpyDeviceToHost,
                                         s), "poll");
                check_hip(hipStreamSynchronize(s), "poll");
                bool done = true;
                int64_t live = 0;
                int next = 1;
                for (int t = 0; t < nt; ++t) {
                    done = done && ctl[t].all_done;
                    for (int q = 0; q < kTileQ; ++q) {
                        const QueryCtl &c = ctl[t].q[q];
                        if (c.source < 0) continue;
                        executed = std::max(executed, (int)c.iter);
                        if (!c.done) {
                            ++live;
                            next = std::max(next, rounds_left(g, c.last_max, c.eps_f));
                        }
                    }
                }
                g.batch.live_q = live;
                if (done) break;
                chunk = next;
            }
            if (g.prof.on) {
                for (int kind = 2; kind <= 4; ++kind) profiler_void_tail(g.prof, kind, launched - executed);
            }
            float *scores = pi_out ? pi_out + q0 * g.n_u : g.batch.out;
            batch_scores(g, g.batch, nt, nq, scores, s);
            if (k > 0)
                topk_launch(scores, g.n_u, g.n_u, nq, d_src.p + q0, -1, k, topk_idx + q0 * k, topk_val + q0 * k,
                            topk_n + q0, g.tk_scratch, s);
            for (int64_t q = 0; q < nq; ++q) {
                const QueryCtl &c = ctl[q / kTileQ].q[q % kTileQ];
                if (c.status != 1) all_converged = false;
            }
            if (stats) {
                batch_resid_sums(g, g.batch, 0, nt, sums.data(), s);
                for (int64_t q = 0; q < nq; ++q) {
                    const QueryCtl &c = ctl[q / kTileQ].q[q % kTileQ];
                    ahpp_stats_t &o = st_all[(size_t)(q0 + q)];
                    o.iters = c.iter;
                    o.sync_switch_iter = c.switch_iter;
                    o.converged = c.status == 1;
                    o.reserved = 0;
                    o.n_push = (int64_t)c.n_p;
                    o.max_residual = c.last_max;
                    o.sum_residual = sums[(size_t)q];
                    o.pad = 0;
                }
            }
        }
        check_hip(hipEventRecord(ev.stop, s), "event");
        int32_t *src_dev = d_src.p;
        d_src.p = nullptr;
        check_hip(hipFreeAsync(src_dev, s), "batch sources");
        check_hip(hipStreamSynchronize(s), "batch");
        const float ms = ev.elapsed_ms();
        if (stats)
            for (int32_t q = 0; q < n_q; ++q) {
                st_all[q].ms = ms;
                stats[q] = st_all[q];
            }
        return AHPP_OK;
    });
    if (rc != AHPP_OK) return rc;
    if (!all_converged) return fail(AHPP_ERR_NOT_CONVERGED, "ahpp_query_batch: some query reached max_iters");
    return AHPP_OK;
}

ahpp_status_t ahpp_topk(const ahpp_graph_t *hc, const float *pi, int32_t k, int32_t exclude, int32_t *idx_out,
                        float *val_out, int32_t *n_out, void *hip_stream) {
    g_last_error.clear();
    if (!hc || !pi || !idx_out || !val_out || !n_out) return fail(AHPP_ERR_INVALID_ARG, "ahpp_topk: NULL argument");
    ahpp_graph_t *h = const_cast<ahpp_graph_t *>(hc);
    Graph &g = h->g;
    if (k < 1 || k > kMaxTopK) return fail(AHPP_ERR_INVALID_ARG, "ahpp_topk: k must be in [1, 2048]");
    if (exclude < -1 || exclude >= g.n_u) return fail(AHPP_ERR_INVALID_ARG, "ahpp_topk: exclude out of range");
    return guarded("ahpp_topk", [&] {
        DeviceScope scope(g.device);
        topk_launch(pi, g.n_u, 0, 1, nullptr, exclude, k, idx_out, val_out, n_out, g.tk_scratch,
                    (hipStream_t)hip_stream);
        return AHPP_OK;
    });
}

}  // extern "C"
