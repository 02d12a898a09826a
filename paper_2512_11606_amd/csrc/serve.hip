// Serving engine: continuous batching of AHPP queries on one device.
//
// The engine owns a batch state of `tiles` tiles of kTileQ lanes.  Each lane
// is a slot for one query with its own residues, reserves, threshold, phase
// and stop rule (the per-query control of the batched rounds).  A step
//   1. admits queued queries into free lanes (their columns are cleared and
//      the source gets unit residue, Algorithm 4's initial state),
//   2. runs a fixed number of rounds over the tiles up to the last one with
//      a running lane (stopped lanes keep threshold +inf and do not change;
//      tiles with no running lane return at once),
//   3. collects the lanes whose stop rule held: their reserves are copied out
//      query-major, reduced to the top-k on the device, copied to the host,
//      and the lane is free for the next admission.
// Queries admitted at different steps therefore share every round's passes
// over the graph, and each result is exactly what the query computes alone
// up to floating-point summation order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "ahpp_internal.h"

namespace ahpp {

namespace {
double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

Server::Server(Graph &g, int64_t max_device_bytes, int32_t max_slots, int32_t k, int32_t max_iters, bool keep_pi)
    : g_(g), k_(k), max_iters_(max_iters > 0 ? max_iters : 100000), keep_pi_(keep_pi) {
    const int64_t before = g.device_bytes;
    const int64_t scratch = (int64_t)kTileQ * g.n_u * 4 + (int64_t)kTileQ * k * 8 + 4096 +
                            (int64_t)topk_scratch_bytes(kTileQ);
    int64_t budget = max_device_bytes;
    if (budget <= 0) {
        size_t free_b = 0, total_b = 0;
        check_hip(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        budget = (int64_t)(free_b / 4);
    }
    const int64_t per_tile = batch_tile_bytes(g, false);
    const int64_t tiles = (budget - scratch) / per_tile;
    if (tiles < 1)
        throw Failure{AHPP_ERR_OUT_OF_MEMORY, "ahpp_server_create: budget holds no query tile (" +
                                                  std::to_string(per_tile + scratch) + " bytes needed)"};
    int64_t cap = 1 << 14;
    if (max_slots > 0) cap = std::min<int64_t>(cap, ((int64_t)max_slots + kTileQ - 1) / kTileQ);
    const int nt = (int)std::min<int64_t>(tiles, cap);
    try {
        ensure_batch_state(g, b_, nt, false);
        d_scores_ = (float *)dev_alloc(g, (size_t)kTileQ * g.n_u * 4, "server scores");
        d_sel_ = (int32_t *)dev_alloc(g, 2 * kTileQ * 4, "server lanes");
        d_idx_ = (int32_t *)dev_alloc(g, (size_t)kTileQ * k * 4, "server top-k");
        d_val_ = (float *)dev_alloc(g, (size_t)kTileQ * k * 4, "server top-k");
        d_n_ = (int32_t *)dev_alloc(g, kTileQ * 4, "server top-k");
        d_tk_ = dev_alloc(g, topk_scratch_bytes(kTileQ), "server top-k scratch");
        hipStream_t s = nullptr;
        batch_empty(g, b_, nt, s);
        check_hip(hipStreamSynchronize(s), "server init");
    } catch (...) {
        free_batch_state(b_);
        for (void *p : {(void *)d_scores_, (void *)d_sel_, (void *)d_idx_, (void *)d_val_, (void *)d_n_, d_tk_})
            dfree(p);
        g.device_bytes = before;
        throw;
    }
    lanes_.assign((size_t)nt * kTileQ, Lane{});
    own_bytes_ = g.device_bytes - before;
}

Server::~Server() {
    for (Result &r : ready_) dfree(r.d_pi);
    free_batch_state(b_);
    for (void *p : {(void *)d_scores_, (void *)d_sel_, (void *)d_idx_, (void *)d_val_, (void *)d_n_, d_tk_}) dfree(p);
    g_.device_bytes -= own_bytes_;
}

void Server::submit(int64_t tag, int32_t source, double eps) { queue_.push_back(Pending{tag, source, eps}); }

void Server::serve_solo(double t_step, hipStream_t s) {
    while (!queue_.empty()) {
        const Pending p = queue_.front();
        queue_.pop_front();
        Result r;
        r.tag = p.tag;
        r.d_pi = nullptr;
        try {
            if (keep_pi_) check_hip(hipMalloc((void **)&r.d_pi, (size_t)g_.n_u * 4), "kept vector");
            ahpp_stats_t st;
            run_query(g_, g_.q, true, p.source, p.eps, 0, max_iters_, r.d_pi, nullptr, k_, d_idx_, d_val_, d_n_, &st,
                      s);
            int32_t n = 0;
            check_hip(hipMemcpyAsync(&n, d_n_, 4, hipMemcpyDeviceToHost, s), "collect");
            check_hip(hipStreamSynchronize(s), "collect");
            r.idx.resize((size_t)n);
            r.val.resize((size_t)n);
            if (n > 0) {
                check_hip(hipMemcpyAsync(r.idx.data(), d_idx_, (size_t)n * 4, hipMemcpyDeviceToHost, s), "collect");
                check_hip(hipMemcpyAsync(r.val.data(), d_val_, (size_t)n * 4, hipMemcpyDeviceToHost, s), "collect");
                check_hip(hipStreamSynchronize(s), "collect");
            }
            st.ms = (float)(now_ms() - t_step);
            r.st = st;
        } catch (...) {
            // The query goes back to the head of the queue; its vector is freed.
            dfree(r.d_pi);
            queue_.push_front(p);
            throw;
        }
        ready_.push_back(std::move(r));
    }
}

int Server::step(int rounds, hipStream_t s) {
    const double t_step = now_ms();
    // 0. Low load (at most solo_max queries queued and at most solo_max in
    // the tiles): a tile round moves every lane's bytes however few queries
    // run in it, so the queued ones are answered one after another on the
    // single-query path (the kernels of ahpp_query: the same guarantee, a
    // fraction of a tile round's time per round); queries already in the
    // tiles run on.  Otherwise the queue is admitted into the tiles, so under
    // load the server batches as before.
    if (solo_max_ > 0 && !queue_.empty() && (int64_t)queue_.size() <= solo_max_) {
        const int64_t in_tiles = std::count_if(lanes_.begin(), lanes_.end(), [](const Lane &l) { return l.busy; });
        if (in_tiles <= solo_max_) serve_solo(t_step, s);
    }
    // 1. Admission into free lanes.
    std::vector<AdmitReq> reqs;
    for (size_t i = 0; i < lanes_.size() && !queue_.empty(); ++i) {
        if (lanes_[i].busy) continue;
        const Pending p = queue_.front();
        queue_.pop_front();
        lanes_[i] = Lane{true, p.tag, p.source, t_step};
        reqs.push_back(AdmitReq{(int32_t)(i / kTileQ), (int32_t)(i % kTileQ), p.source, (float)(p.eps / g_.lambda)});
    }
    batch_admit(g_, b_, reqs, max_iters_, s);
    // Admission fills the lowest free lanes, so running queries gather in the
    // low tiles: rounds cover tiles [0, active) only, and each active tile
    // gets a larger share of the workgroups.
    int64_t running = 0;
    int active = 0;
    for (size_t i = 0; i < lanes_.size(); ++i)
        if (lanes_[i].busy) {
            ++running;
            active = (int)(i / kTileQ) + 1;
        }
    // 2. Rounds for every running query.
    if (running > 0) {
        b_.live_q = running;
        batch_rounds(g_, b_, active, rounds, s);
    }
    // 3. Collection of stopped queries.
    std::vector<TileCtl> ctl((size_t)b_.tiles);
    check_hip(hipMemcpyAsync(ctl.data(), b_.ctl, ctl.size() * sizeof(TileCtl), hipMemcpyDeviceToHost, s), "poll");
    check_hip(hipStreamSynchronize(s), "poll");
    std::vector<double> sums(kTileQ);
    for (int t = 0; t < b_.tiles; ++t) {
        int32_t sel[2 * kTileQ];
        int n_sel = 0;
        for (int q = 0; q < kTileQ; ++q) {
            const Lane &l = lanes_[(size_t)t * kTileQ + q];
            if (l.busy && ctl[t].q[q].done) {
                sel[n_sel] = q;
                ++n_sel;
            }
        }
        if (!n_sel) continue;
        for (int j = 0; j < n_sel; ++j) sel[kTileQ + j] = lanes_[(size_t)t * kTileQ + sel[j]].source;
        check_hip(hipMemcpyAsync(d_sel_, sel, sizeof(sel), hipMemcpyHostToDevice, s), "collect");
        batch_lanes_out(g_, b_, t, d_sel_, n_sel, d_scores_, s);
        topk_launch(d_scores_, g_.n_u, g_.n_u, n_sel, d_sel_ + kTileQ, -1, k_, d_idx_, d_val_, d_n_, d_tk_, s);
        batch_resid_sums(g_, b_, t, 1, sums.data(), s);
        std::vector<int32_t> idx((size_t)n_sel * k_), nn((size_t)n_sel);
        std::vector<float> val((size_t)n_sel * k_);
        check_hip(hipMemcpyAsync(idx.data(), d_idx_, idx.size() * 4, hipMemcpyDeviceToHost, s), "collect");
        check_hip(hipMemcpyAsync(val.data(), d_val_, val.size() * 4, hipMemcpyDeviceToHost, s), "collect");
        check_hip(hipMemcpyAsync(nn.data(), d_n_, nn.size() * 4, hipMemcpyDeviceToHost, s), "collect");
        check_hip(hipStreamSynchronize(s), "collect");
        const double t_end = now_ms();
        for (int j = 0; j < n_sel; ++j) {
            const int q = sel[j];
            Lane &l = lanes_[(size_t)t * kTileQ + q];
            const QueryCtl &c = ctl[t].q[q];
            Result r;
            r.tag = l.tag;
            r.idx.assign(idx.begin() + (size_t)j * k_, idx.begin() + (size_t)j * k_ + nn[j]);
            r.val.assign(val.begin() + (size_t)j * k_, val.begin() + (size_t)j * k_ + nn[j]);
            r.st = ahpp_stats_t{c.iter, c.switch_iter, c.status == 1, 0, (int64_t)c.n_p, (double)c.last_max,
                                sums[q], (float)(t_end - l.t_admit), 0.0f};
            r.d_pi = nullptr;
            if (keep_pi_) {
                check_hip(hipMalloc((void **)&r.d_pi, (size_t)g_.n_u * 4), "kept vector");
                check_hip(hipMemcpyAsync(r.d_pi, d_scores_ + (size_t)j * g_.n_u, (size_t)g_.n_u * 4,
                                         hipMemcpyDeviceToDevice, s), "kept vector");
            }
            ready_.push_back(std::move(r));
            l = Lane{};
        }
    }
    if (keep_pi_) check_hip(hipStreamSynchronize(s), "kept vectors");
    return (int)ready_.size();
}

int Server::results(int max_n, int64_t *tags, int32_t *topk_idx, float *topk_val, int32_t *topk_n,
                    ahpp_stats_t *stats, float *pi_out, hipStream_t s) {
    int n = 0;
    while (n < max_n && !ready_.empty()) {
        Result &r = ready_.front();
        if (tags) tags[n] = r.tag;
        if (topk_n) topk_n[n] = (int32_t)r.idx.size();
        for (size_t i = 0; i < r.idx.size(); ++i) {
            if (topk_idx) topk_idx[(size_t)n * k_ + i] = r.idx[i];
            if (topk_val) topk_val[(size_t)n * k_ + i] = r.val[i];
        }
        if (stats) stats[n] = r.st;
        if (pi_out && r.d_pi)
            check_hip(hipMemcpyAsync(pi_out + (size_t)n * g_.n_u, r.d_pi, (size_t)g_.n_u * 4,
                                     hipMemcpyDeviceToDevice, s), "result vector");
        if (r.d_pi) {
            check_hip(hipStreamSynchronize(s), "result vector");
            dfree(r.d_pi);
        }
        ready_.pop_front();
        ++n;
    }
    return n;
}

void Server::info(int32_t *slots, int32_t *running, int32_t *queued, int32_t *ready) const {
    int32_t busy = 0;
    for (const Lane &l : lanes_) busy += l.busy;
    if (slots) *slots = (int32_t)lanes_.size();
    if (running) *running = busy;
    if (queued) *queued = (int32_t)queue_.size();
    if (ready) *ready = (int32_t)ready_.size();
}

}  // namespace ahpp
