// Debug mode: before every launch that reads the connectivity, one thread per
// element checks that its node ids lie in [0, N) and, when the call assembles
// into a pattern, that the slot of every local pair (a, b) lies inside row
// conn[a] and holds column conn[b] (a connectivity edited after the pattern
// was built fails here).  The first failing element (smallest id) is reported
// as LFEM_EINVAL and nothing is launched.  The check synchronises the stream;
// it is meant for development, not for captured graphs.
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "lfem_internal.hpp"

namespace lfem {

namespace {

inline unsigned grid_for(int64_t n, int nt) { return static_cast<unsigned>((n + nt - 1) / nt); }

// (element << 8 | reason) of the first failure, ULLONG_MAX when none
__device__ unsigned long long g_dbg_first;

__global__ __launch_bounds__(256) void k_debug_check(int k, int64_t T, int64_t N, const int32_t *__restrict__ conn,
                                                     const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col_idx,
                                                     const uint8_t *__restrict__ off8,
                                                     const uint16_t *__restrict__ off16, int kkp, int slots)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    unsigned reason = 0;
    for (int a = 0; a < k && !reason; ++a) {
        const int32_t n = conn[a * T + e];
        if (n < 0 || n >= N) reason = 1;
    }
    if (!reason && slots) {
        for (int a = 0; a < k && !reason; ++a) {
            const int32_t ra = conn[a * T + e];
            const int32_t r0 = row_ptr[ra], r1 = row_ptr[ra + 1];
            for (int b = 0; b < k; ++b) {
                const int32_t off = off16 ? static_cast<int32_t>(off16[e * k * k + a * k + b])
                                          : static_cast<int32_t>(off8[e * kkp + a * k + b]);
                if (r0 + off >= r1) {
                    reason = 2;
                    break;
                }
                if (col_idx[r0 + off] != conn[b * T + e]) {
                    reason = 3;
                    break;
                }
            }
        }
    }
    if (reason) atomicMin(&g_dbg_first, (static_cast<unsigned long long>(e) << 8) | reason);
}

int initial_debug()
{
    const char *env = std::getenv("LFEM_DEBUG");
    return env && env[0] == '1' ? 1 : 0;
}

std::atomic<int> g_debug{initial_debug()};
std::mutex g_debug_mu;  // one check at a time (the result word is shared)

}  // namespace

int set_debug(int on) { return g_debug.exchange(on ? 1 : 0); }

void debug_check(const Mesh &m, const Pattern *p, hipStream_t s)
{
    if (!g_debug.load() || m.T == 0) return;
    std::lock_guard<std::mutex> lock(g_debug_mu);
    unsigned long long first = ULLONG_MAX;
    LFEM_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_dbg_first), &first, sizeof(first), 0, hipMemcpyHostToDevice, s));
    const bool slots = p && p->nnz > 0;
    k_debug_check<<<grid_for(m.T, 256), 256, 0, s>>>(m.k, m.T, m.N, m.conn, slots ? p->row_ptr : nullptr,
                                                     slots ? p->col_idx : nullptr, slots ? p->off8 : nullptr,
                                                     slots ? p->off16 : nullptr, slots ? p->kkp : 0, slots ? 1 : 0);
    LFEM_HIP(hipGetLastError());
    LFEM_HIP(hipMemcpyFromSymbolAsync(&first, HIP_SYMBOL(g_dbg_first), sizeof(first), 0, hipMemcpyDeviceToHost, s));
    LFEM_HIP(hipStreamSynchronize(s));
    if (first == ULLONG_MAX) return;
    static const char *what[] = {"", "node id outside [0, N)",
                                 "local pair slot outside its row (connectivity changed since the pattern was built?)",
                                 "local pair slot holds another column (connectivity changed since the pattern was "
                                 "built?)"};
    const unsigned reason = static_cast<unsigned>(first & 0xff);
    char msg[256];
    std::snprintf(msg, sizeof msg, "debug check: element %lld: %s", static_cast<long long>(first >> 8),
                  reason <= 3 ? what[reason] : "unknown");
    throw Error{LFEM_EINVAL, msg};
}

}  // namespace lfem
