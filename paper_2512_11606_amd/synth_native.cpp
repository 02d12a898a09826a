// Multi-threaded host generator for the seeded synthetic graphs of synth.py.
//
// Input generation only: no AHPP arithmetic.  Every function reproduces one
// step of synth.py exactly (same counter-based streams, same rejection order,
// same float rounding), so both generators give identical arrays; synth.py
// stays the readable definition and tests compare the two on small graphs.
// The caller passes what is cheap to compute in numpy (stream keys, Zipf
// CDFs, the attribute permutation).
#include <omp.h>
#include <parallel/algorithm>

#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// SplitMix64's output function (Steele, Lea and Flood, 2014).
inline uint64_t mix64(uint64_t x) {
    uint64_t z = x + kGolden;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Value `ctr` of the stream with key `key`: a double in [0, 1) with 53 bits.
inline double uniform_at(uint64_t key, uint64_t ctr) {
    return (double)(mix64(key + ctr * kGolden) >> 11) * (1.0 / 9007199254740992.0);
}

// numpy.searchsorted(cdf, u, side="right"), clipped to len - 1.
inline int64_t sample_cdf(const double *cdf, int64_t len, double u) {
    const int64_t i = std::upper_bound(cdf, cdf + len, u) - cdf;
    return i < len - 1 ? i : len - 1;
}

struct Cand {
    uint64_t key;
    uint32_t idx;
};

inline bool cand_less(const Cand &a, const Cand &b) { return a.key < b.key || (a.key == b.key && a.idx < b.idx); }

// Node x appears theta[x] times: the urn of one side.
std::vector<int32_t> make_urn(const std::vector<int64_t> &theta) {
    const int64_t n = (int64_t)theta.size();
    std::vector<int64_t> start(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + theta[i];
    std::vector<int32_t> urn((size_t)start[n]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = start[i]; j < start[i + 1]; ++j) urn[j] = (int32_t)i;
    return urn;
}

}  // namespace

extern "C" {

// out[i] = float32(a + b * uniform(key, i)), raised to FLT_MIN when `floor_tiny`.
void sn_uniform_f32(uint64_t key, int64_t n, double a, double b, int32_t floor_tiny, float *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float v = (float)(a + b * uniform_at(key, (uint64_t)i));
        if (floor_tiny && v < FLT_MIN) v = FLT_MIN;
        out[i] = v;
    }
}

// The edge list of synth._draw_edges, sorted by (u, v).  eu / ev hold at
// least m_e + n_u entries.  Returns the number of edges, or -1 when the
// rejection rounds do not reach m_e distinct pairs.
int64_t sn_draw_edges(int64_t n_u, int64_t n_v, int64_t m_e, const double *cdf_u, const double *cdf_v,
                      uint64_t key_theta, uint64_t key_edges, uint64_t key_lonely, int32_t *eu, int32_t *ev) {
    // Degree weights: theta_u from counters [0, n_u), theta_v from [n_u, n_u + n_v).
    std::vector<int64_t> theta_u((size_t)n_u), theta_v((size_t)n_v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_u; ++i) theta_u[i] = sample_cdf(cdf_u, n_v, uniform_at(key_theta, (uint64_t)i)) + 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_v; ++i)
        theta_v[i] = sample_cdf(cdf_v, n_u, uniform_at(key_theta, (uint64_t)(n_u + i))) + 1;
    const std::vector<int32_t> urn_u = make_urn(theta_u), urn_v = make_urn(theta_v);
    const double size_u = (double)urn_u.size(), size_v = (double)urn_v.size();

    std::vector<uint64_t> keys;  // sorted distinct pairs u * n_v + v
    uint64_t ctr = 0;
    int64_t need = m_e;
    int rounds = 0;
    while (need > 0) {
        const int64_t k = (int64_t)((double)need * 1.05) + 16;
        std::vector<Cand> c((size_t)k);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < k; ++i) {
            const int64_t iu = (int64_t)(uniform_at(key_edges, ctr + (uint64_t)i) * size_u);
            const int64_t iv = (int64_t)(uniform_at(key_edges, ctr + (uint64_t)(k + i)) * size_v);
            c[i] = Cand{(uint64_t)urn_u[iu] * (uint64_t)n_v + (uint64_t)urn_v[iv], (uint32_t)i};
        }
        ctr += 2 * (uint64_t)k;
        __gnu_parallel::sort(c.begin(), c.end(), cand_less);
        // First occurrence of each candidate pair that is not already an edge.
        std::vector<uint8_t> keep((size_t)k, 0);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < k; ++i) {
            if (i > 0 && c[i].key == c[i - 1].key) continue;
            keep[i] = !std::binary_search(keys.begin(), keys.end(), c[i].key);
        }
        int64_t fresh = 0;
#pragma omp parallel for reduction(+ : fresh)
        for (int64_t i = 0; i < k; ++i) fresh += keep[i];
        if (fresh > need) {
            // Keep the `need` earliest draws.
            std::vector<uint32_t> first;
            first.reserve((size_t)fresh);
            for (int64_t i = 0; i < k; ++i)
                if (keep[i]) first.push_back(c[i].idx);
            std::nth_element(first.begin(), first.begin() + (need - 1), first.end());
            const uint32_t cut = first[need - 1];
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < k; ++i)
                if (keep[i] && c[i].idx > cut) keep[i] = 0;
        }
        std::vector<uint64_t> add;
        add.reserve((size_t)std::min(fresh, need));
        for (int64_t i = 0; i < k; ++i)
            if (keep[i]) add.push_back(c[i].key);
        std::vector<Cand>().swap(c);
        std::vector<uint8_t>().swap(keep);
        // The parallel merge dereferences the first element of each input, so
        // an empty side (the first round's keys, a round with no fresh pair)
        // is handled here.
        if (keys.empty()) {
            keys.swap(add);
        } else if (!add.empty()) {
            std::vector<uint64_t> merged(keys.size() + add.size());
            __gnu_parallel::merge(keys.begin(), keys.end(), add.begin(), add.end(), merged.begin());
            keys.swap(merged);
        }
        need = m_e - (int64_t)keys.size();
        if (++rounds > 500) return -1;
    }
    // Every U node gets at least one edge.
    std::vector<uint8_t> has((size_t)n_u, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)keys.size(); ++i) has[keys[i] / (uint64_t)n_v] = 1;
    std::vector<uint64_t> extra;
    for (int64_t u = 0; u < n_u; ++u)
        if (!has[u]) {
            const double r = uniform_at(key_lonely, (uint64_t)extra.size());
            extra.push_back((uint64_t)u * (uint64_t)n_v + (uint64_t)urn_v[(int64_t)(r * size_v)]);
        }
    if (!extra.empty()) {
        std::vector<uint64_t> merged(keys.size() + extra.size());
        __gnu_parallel::merge(keys.begin(), keys.end(), extra.begin(), extra.end(), merged.begin());
        keys.swap(merged);
    }
    const int64_t m = (int64_t)keys.size();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        eu[i] = (int32_t)(keys[i] / (uint64_t)n_v);
        ev[i] = (int32_t)(keys[i] % (uint64_t)n_v);
    }
    return m;
}

// The attribute lists of synth._draw_attrs: node u gets the first c distinct
// ranks of its Zipf stream, mapped through perm and sorted by attribute id;
// au / aa hold n_u * c entries in (u, a) order.  Returns the number of
// rejection rounds, or -1 when they do not converge.
int32_t sn_draw_attrs(int64_t n_u, int64_t n_attr, int32_t c, const double *cdf, const int64_t *perm, uint64_t key,
                      int32_t *au, int32_t *aa) {
    std::vector<int64_t> todo((size_t)n_u);
    for (int64_t i = 0; i < n_u; ++i) todo[i] = i;
    int64_t width = 4 * (int64_t)c;
    uint64_t base = 0;
    int rounds = 0;
    while (!todo.empty()) {
        const int64_t m = (int64_t)todo.size();
        std::vector<uint8_t> ok((size_t)m, 0);
#pragma omp parallel
        {
            std::vector<uint8_t> seen((size_t)n_attr, 0);
            std::vector<int64_t> got((size_t)c);
#pragma omp for schedule(dynamic, 4096)
            for (int64_t j = 0; j < m; ++j) {
                int n = 0;
                for (int64_t d = 0; d < width && n < c; ++d) {
                    const int64_t r =
                        sample_cdf(cdf, n_attr, uniform_at(key, base + (uint64_t)j * (uint64_t)width + (uint64_t)d));
                    if (!seen[r]) {
                        seen[r] = 1;
                        got[n++] = r;
                    }
                }
                for (int i = 0; i < n; ++i) seen[got[i]] = 0;
                if (n == c) {
                    ok[j] = 1;
                    const int64_t u = todo[j];
                    int32_t *row = aa + u * c;
                    for (int i = 0; i < c; ++i) row[i] = (int32_t)perm[got[i]];
                    std::sort(row, row + c);
                    for (int i = 0; i < c; ++i) au[u * c + i] = (int32_t)u;
                }
            }
        }
        base += (uint64_t)m * (uint64_t)width;
        std::vector<int64_t> next;
        for (int64_t j = 0; j < m; ++j)
            if (!ok[j]) next.push_back(todo[j]);
        todo.swap(next);
        width *= 2;
        if (++rounds > 30) return -1;
    }
    return rounds;
}

int32_t sn_max_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
