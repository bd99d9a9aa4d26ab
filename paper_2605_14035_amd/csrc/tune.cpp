// Autotuner for the numeric scatter: times the candidates (blocked with
// several LDS block capacities, staged, and, when the caller allows it,
// atomic) on the pattern's own mesh and keeps the fastest.  The atomic
// variant is a candidate only on request because its summation order is not
// fixed.  Results are kept in a process-wide cache keyed by device, element
// type, rule, matrix set, size bucket (bit length of the element count) and
// whether atomics were allowed, so a mesh of a known kind and size is
// scheduled without timing.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lfem_internal.hpp"
#include "side.hpp"

namespace lfem {

namespace {

// a pair of timing events, released on every exit path
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair()
    {
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            release();
            throw Error{LFEM_EHIP, "hipEventCreate failed"};
        }
    }
    ~EventPair() { release(); }
    void release()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        a = b = nullptr;
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
};

float time_variant(Mesh &m, Pattern &p, const NumericOut &o, int variant, hipStream_t s)
{
    EventPair ev;
    launch_numeric(m, p, o, variant, s);  // warm-up (builds lazy structures)
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
        LFEM_HIP(hipEventRecord(ev.a, s));
        launch_numeric(m, p, o, variant, s);
        LFEM_HIP(hipEventRecord(ev.b, s));
        LFEM_HIP(hipEventSynchronize(ev.b));
        float ms = 0.f;
        LFEM_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        best = std::min(best, ms);
    }
    return best;
}

// the result cache
// device, element type, rule, matrices, size bucket, atomic allowed, 16-bit slot map
using TuneKey = std::tuple<int, int, int, unsigned, int, int, int>;
struct TuneResult {
    int variant;
    int cap;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneResult> g_tune_cache;

int size_bucket(int64_t T)
{
    int b = 0;
    while (T > 0) {
        ++b;
        T >>= 1;
    }
    return b;
}

TuneKey tune_key(const Mesh &m, const Pattern &p, unsigned what, bool atomic)
{
    int dev = 0;
    LFEM_HIP(hipGetDevice(&dev));
    return TuneKey{dev, m.etype, m.Q, what, size_bucket(m.T), atomic ? 1 : 0, p.off16 ? 1 : 0};
}

// the staged scatter's size limit (its contribution codes are int32)
bool staged_fits(const Mesh &m) { return static_cast<int64_t>(m.k) * m.k * m.T < (int64_t(1) << 31); }

// apply a cached choice; false when it does not fit this pattern (a block
// capacity below its longest row, a schedule the mesh cannot take)
bool apply_cached(Mesh &m, Pattern &p, const TuneResult &r, hipStream_t s)
{
    if (r.variant == LFEM_SCATTER_BLOCKED) {
        if (r.cap < p.max_row) return false;
        if (!(p.sched.nb > 0 && p.sched.cap == r.cap)) {
            try {
                build_schedule(m, p, r.cap, kBlockMaxRows, s);
            } catch (const Error &e) {
                if (e.code != LFEM_EUNSUPPORTED) throw;
                return false;
            }
        }
    } else if (r.variant == LFEM_SCATTER_STAGED && !staged_fits(m)) {
        return false;
    }
    p.tuned_variant = r.variant;
    return true;
}

}  // namespace

void tune_cache_clear()
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.clear();
}

int default_block_cap(int max_row)
{
    return std::max(max_row, std::min(kBlockCapDefault, kTwoGroupLdsDoubles - side_dump_entries(max_row)));
}

int autotune_pattern(Mesh &m, Pattern &p, unsigned what, unsigned flags, hipStream_t s)
{
    if (m.T == 0 || p.nnz == 0) return p.tuned_variant;
    const bool allow_atomic = flags & LFEM_TUNE_ALLOW_ATOMIC;
    const TuneKey key = tune_key(m, p, what, allow_atomic);
    if (!(flags & LFEM_TUNE_NO_CACHE)) {
        TuneResult hit{};
        bool found = false;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                hit = it->second;
                found = true;
            }
        }
        if (found && apply_cached(m, p, hit, s)) return p.tuned_variant;
    }
    const int nmat = ((what & LFEM_M) ? 1 : 0) + ((what & LFEM_A) ? 1 : 0);
    double *buf = nullptr;
    LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&buf), static_cast<size_t>(nmat) * p.nnz * 8));
    NumericOut o;
    o.what = what;
    int slot = 0;
    if (what & LFEM_M) o.vals_m = buf + static_cast<size_t>(slot++) * p.nnz;
    if (what & LFEM_A) o.vals_a = buf + static_cast<size_t>(slot++) * p.nnz;
    float best = 1e30f;
    int best_variant = LFEM_SCATTER_STAGED, best_cap = 0;
    // LFEM_TUNE_VERBOSE=1 prints every candidate's time to stderr
    const char *env = std::getenv("LFEM_TUNE_VERBOSE");
    const bool verbose = env && env[0] == '1';
    try {
        const int caps[] = {2048, 3072, 4096, 4864, 4992, 6144, 8192};
        for (int cap : caps) {
            if (cap < p.max_row) continue;
            if (static_cast<size_t>(nmat) * cap * 8 + 4 * 1025 > 160 * 1024) continue;
            try {
                build_schedule(m, p, cap, kBlockMaxRows, s);
            } catch (const Error &e) {
                if (e.code != LFEM_EUNSUPPORTED) throw;
                continue;
            }
            const float t = time_variant(m, p, o, LFEM_SCATTER_BLOCKED, s);
            if (verbose)
                std::fprintf(stderr, "[lfem tune] blocked cap %d: %.1f us (blocks %d, halo %.3f)\n",
                             cap, t * 1e3, p.sched.nb, p.sched.halo);
            if (t < best) {
                best = t;
                best_variant = LFEM_SCATTER_BLOCKED;
                best_cap = cap;
            }
        }
        if (staged_fits(m)) {
            const float t = time_variant(m, p, o, LFEM_SCATTER_STAGED, s);
            if (verbose) std::fprintf(stderr, "[lfem tune] staged: %.1f us\n", t * 1e3);
            if (t < best) {
                best = t;
                best_variant = LFEM_SCATTER_STAGED;
            }
        }
        if (allow_atomic) {
            const float t = time_variant(m, p, o, LFEM_SCATTER_ATOMIC, s);
            if (verbose) std::fprintf(stderr, "[lfem tune] atomic: %.1f us\n", t * 1e3);
            if (t < best) {
                best = t;
                best_variant = LFEM_SCATTER_ATOMIC;
            }
        }
        LFEM_REQUIRE(best < 1e30f, LFEM_EUNSUPPORTED, "no scatter variant fits this mesh");
        if (best_variant == LFEM_SCATTER_BLOCKED) build_schedule(m, p, best_cap, kBlockMaxRows, s);
    } catch (...) {
        dev_free(buf);
        throw;
    }
    LFEM_HIP(hipStreamSynchronize(s));
    dev_free(buf);
    p.tuned_variant = best_variant;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = TuneResult{best_variant, best_cap};
    }
    return best_variant;
}

}  // namespace lfem
