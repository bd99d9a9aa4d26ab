// Symbolic phase: everything that depends only on the element array.
//
//  * node -> element incidence (counting sort; each node's list ascending)
//  * structural CSR pattern: row i holds every node that shares an element
//    with node i, ascending (the paper keeps COO triples and lets sparse()
//    sort them, Listing 1 lines 10-11 and 22; here the pattern is computed
//    once and reused, as section 4.2 notes FEM packages do)
//  * slot map: for element e and local pair (a, b) the column offset of
//    conn[b][e] inside row conn[a][e], one byte each
//  * staged-scatter contribution lists (slot -> (element, pair), ascending)
//  * row-block schedule of the blocked scatter (host side)
#include <algorithm>
#include <cstring>

#include "lfem_internal.hpp"

namespace lfem {

namespace {

constexpr int SCAN_NT = 256;
constexpr int SCAN_TILE = 1024;

template <typename TI, typename TO>
__global__ __launch_bounds__(SCAN_NT) void k_scan_tile(const TI *__restrict__ in,
                                                       TO *__restrict__ out, int64_t n,
                                                       int64_t *__restrict__ sums)
{
    __shared__ int64_t s[SCAN_NT];
    const int t = threadIdx.x;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + t * 4;
    int64_t v[4], acc = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? static_cast<int64_t>(in[base + i]) : 0;
        acc += v[i];
    }
    s[t] = acc;
    __syncthreads();
    for (int off = 1; off < SCAN_NT; off <<= 1) {
        const int64_t add = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int64_t run = s[t] - acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) out[base + i] = static_cast<TO>(run);
        run += v[i];
    }
    if (t == SCAN_NT - 1) sums[blockIdx.x] = s[t];
}

template <typename TO>
__global__ void k_scan_add(TO *__restrict__ out, int64_t n, const int64_t *__restrict__ offs)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = static_cast<TO>(static_cast<int64_t>(out[i]) + offs[i / SCAN_TILE]);
}

__global__ void k_copy_total(const int64_t *__restrict__ sums, int64_t *__restrict__ total)
{
    *total = sums[0];
}

template <typename TO>
__global__ void k_write_last(TO *__restrict__ out, int64_t n, const int64_t *__restrict__ total)
{
    out[n] = static_cast<TO>(*total);
}

// exclusive scan of n values; out[n] (if write_last) and *d_total get the total
template <typename TI, typename TO>
void scan_rec(const TI *in, TO *out, int64_t n, int64_t *d_total, hipStream_t s)
{
    const int64_t ntiles = std::max<int64_t>(1, (n + SCAN_TILE - 1) / SCAN_TILE);
    int64_t *sums = nullptr;
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&sums), ntiles * sizeof(int64_t), s));
    k_scan_tile<TI, TO><<<ntiles, SCAN_NT, 0, s>>>(in, out, n, sums);
    LFEM_HIP(hipGetLastError());
    if (ntiles > 1) {
        int64_t *offs = nullptr;
        LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&offs), ntiles * sizeof(int64_t), s));
        scan_rec<int64_t, int64_t>(sums, offs, ntiles, d_total, s);
        k_scan_add<TO><<<(n + 255) / 256, 256, 0, s>>>(out, n, offs);
        LFEM_HIP(hipGetLastError());
        LFEM_HIP(hipFreeAsync(offs, s));
    } else {
        k_copy_total<<<1, 1, 0, s>>>(sums, d_total);
        LFEM_HIP(hipGetLastError());
    }
    LFEM_HIP(hipFreeAsync(sums, s));
}

// ---------------------------------------------------------------------------
// node -> element incidence
// ---------------------------------------------------------------------------
__global__ void k_inc_count(const int32_t *__restrict__ conn, int64_t kT, int64_t N,
                            int32_t *__restrict__ cnt, int32_t *__restrict__ flags)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= kT) return;
    const int32_t node = conn[i];
    if (node < 0 || node >= N)
        atomicOr(&flags[0], 1);
    else
        atomicAdd(&cnt[node], 1);
}

__global__ void k_inc_fill(const int32_t *__restrict__ conn, int64_t kT, int64_t T, int64_t N,
                           const int32_t *__restrict__ ptr, int32_t *__restrict__ cursor,
                           int32_t *__restrict__ ne)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= kT) return;
    const int32_t node = conn[i];
    if (node < 0 || node >= N) return;
    // the incidence (e, a) is coded by its position a * T + e in conn
    const int32_t pos = atomicAdd(&cursor[node], 1);
    ne[ptr[node] + pos] = static_cast<int32_t>(i);
}

// sort every short list [ptr[i], ptr[i+1]) ascending (insertion sort)
__global__ void k_sort_lists(int64_t n, const int32_t *__restrict__ ptr, int32_t *__restrict__ v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = ptr[i], e = ptr[i + 1];
    for (int32_t s = b + 1; s < e; ++s) {
        const int32_t x = v[s];
        int32_t t = s - 1;
        while (t >= b && v[t] > x) {
            v[t + 1] = v[t];
            --t;
        }
        v[t + 1] = x;
    }
}

__global__ void k_validate(const int32_t *__restrict__ conn, int64_t T, int k,
                           int32_t *__restrict__ flags)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (conn[a * T + e] == conn[b * T + e]) atomicOr(&flags[1], 1);
}

// ---------------------------------------------------------------------------
// rows: the sorted set of nodes sharing an element with node i
// ---------------------------------------------------------------------------
// one thread per row with an insertion-sorted buffer of RMAX entries in LDS:
// elements of up to kMaxNodes8 nodes (byte slot maps) take 64 rows of 255,
// larger ones 16 rows of kMaxRowWide
constexpr int ROW_NT = 64;
constexpr int ROW_MAX = 255;
constexpr int ROW_NT_WIDE = 16;

// element e of the incidence code c = a * T + e (0 <= a < k, c < 2^31): the
// FP64 quotient is within 2^-21 of c / T, so truncating it is off by at most
// one, which one correction step fixes (no 32-bit integer division per code)
__device__ __forceinline__ int64_t inc_elem(int32_t c, int64_t T, double inv_t)
{
    const int64_t a = static_cast<int64_t>(static_cast<double>(c) * inv_t);
    int64_t e = c - a * T;
    if (e < 0)
        e += T;
    else if (e >= T)
        e -= T;
    return e;
}

template <int FILL, int RMAX = ROW_MAX, int NTR = ROW_NT>
__global__ __launch_bounds__(NTR) void k_rows(int64_t N, int k, int64_t T,
                                                 const int32_t *__restrict__ conn,
                                                 const int32_t *__restrict__ ne_ptr,
                                                 const int32_t *__restrict__ ne,
                                                 int32_t *__restrict__ rowlen,
                                                 const int32_t *__restrict__ row_ptr,
                                                 int32_t *__restrict__ col_idx,
                                                 int32_t *__restrict__ flags)
{
    __shared__ int32_t buf[RMAX * NTR];
    const int t = threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * NTR + t;
    if (i >= N) return;  // no barrier below
    int len = 0;
    bool overflow = false;
    const double inv_t = 1.0 / static_cast<double>(T > 0 ? T : 1);
    const int32_t s0 = ne_ptr[i], s1 = ne_ptr[i + 1];
    if (RMAX > ROW_MAX && static_cast<int64_t>(s1 - s0) * k <= RMAX) {
        // long rows of large elements, every candidate fitting: collect them
        // with repeats, sort (Shell's method, Ciura's gaps: no quadratic cost
        // when the incidences do not arrive in node order) and drop the
        // repeats (for short rows the insertion below is faster)
        int n = 0;
        for (int32_t s = s0; s < s1; ++s) {
            const int64_t e = inc_elem(ne[s], T, inv_t);
            for (int b = 0; b < k; ++b) buf[(n++) * NTR + t] = conn[b * T + e];
        }
        constexpr int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
        for (int gi = 0; gi < 8; ++gi) {
            const int h = gaps[gi];
            for (int r = h; r < n; ++r) {
                const int32_t v = buf[r * NTR + t];
                int q = r;
                while (q >= h && buf[(q - h) * NTR + t] > v) {
                    buf[q * NTR + t] = buf[(q - h) * NTR + t];
                    q -= h;
                }
                buf[q * NTR + t] = v;
            }
        }
        for (int r = 0; r < n; ++r) {
            const int32_t v = buf[r * NTR + t];
            if (len == 0 || buf[(len - 1) * NTR + t] != v) buf[(len++) * NTR + t] = v;
        }
    } else {
        // insertion into the sorted row, which also detects a row longer than RMAX
        for (int32_t s = s0; s < s1 && !overflow; ++s) {
            const int64_t e = inc_elem(ne[s], T, inv_t);
            for (int b = 0; b < k; ++b) {
                const int32_t j = conn[b * T + e];
                int lo = 0, hi = len;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (buf[mid * NTR + t] < j)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < len && buf[lo * NTR + t] == j) continue;
                if (len == RMAX) {
                    overflow = true;
                    break;
                }
                for (int r = len; r > lo; --r) buf[r * NTR + t] = buf[(r - 1) * NTR + t];
                buf[lo * NTR + t] = j;
                ++len;
            }
        }
    }
    if (overflow) atomicOr(&flags[2], 1);
    if (!FILL) {
        rowlen[i] = len;
    } else {
        const int32_t b = row_ptr[i];
        for (int r = 0; r < len; ++r) col_idx[b + r] = buf[r * NTR + t];
    }
}

// ---------------------------------------------------------------------------
// slot map
// ---------------------------------------------------------------------------
__global__ void k_offsets(int k, int64_t T, const int32_t *__restrict__ conn,
                          const int32_t *__restrict__ row_ptr,
                          const int32_t *__restrict__ col_idx, uint8_t *__restrict__ off8,
                          int kkp, int32_t *__restrict__ flags)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    uint32_t words[kMaxSlotWords];  // kkp / 4 <= kMaxSlotWords (checked on the host)
    for (int w = 0; w < kkp / 4; ++w) words[w] = 0;
    for (int a = 0; a < k; ++a) {
        const int32_t row = conn[a * T + e];
        const int32_t beg = row_ptr[row], end = row_ptr[row + 1];
        for (int b = 0; b < k; ++b) {
            const int32_t col = conn[b * T + e];
            int32_t lo = beg, hi = end;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (col_idx[mid] < col)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo >= end || col_idx[lo] != col) atomicOr(&flags[3], 1);
            const int slot = a * k + b;
            words[slot >> 2] |= static_cast<uint32_t>((lo - beg) & 0xff) << (8 * (slot & 3));
        }
    }
    uint32_t *dst = reinterpret_cast<uint32_t *>(off8 + e * kkp);
    for (int w = 0; w < kkp / 4; ++w) dst[w] = words[w];
}

// the same with 16-bit offsets (off16[e * k * k + a * k + b]), for large elements
__global__ void k_offsets16(int k, int64_t T, const int32_t *__restrict__ conn,
                            const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                            uint16_t *__restrict__ off16, int32_t *__restrict__ flags)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    for (int a = 0; a < k; ++a) {
        const int32_t row = conn[a * T + e];
        const int32_t beg = row_ptr[row], end = row_ptr[row + 1];
        for (int b = 0; b < k; ++b) {
            const int32_t col = conn[b * T + e];
            int32_t lo = beg, hi = end;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (col_idx[mid] < col)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo >= end || col_idx[lo] != col) atomicOr(&flags[3], 1);
            off16[(e * k + a) * k + b] = static_cast<uint16_t>(lo - beg);
        }
    }
}

// column offset of local pair (a, b) of element e in row conn[a]: byte map
// (stride kkp) or 16-bit map (stride k * k)
__device__ __forceinline__ int32_t slot_offset(const uint8_t *off8, const uint16_t *off16, int kkp, int k,
                                               int64_t e, int ab)
{
    return off16 ? static_cast<int32_t>(off16[e * k * k + ab]) : static_cast<int32_t>(off8[e * kkp + ab]);
}

// ---------------------------------------------------------------------------
// staged scatter: slot -> contributions
// ---------------------------------------------------------------------------
__global__ void k_contrib_count(int k, int64_t T, const int32_t *__restrict__ conn,
                                const int32_t *__restrict__ row_ptr,
                                const uint8_t *__restrict__ off8, int kkp,
                                int32_t *__restrict__ cnt, const uint16_t *__restrict__ off16 = nullptr)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    for (int a = 0; a < k; ++a) {
        const int32_t rb = row_ptr[conn[a * T + e]];
        for (int b = 0; b < k; ++b) atomicAdd(&cnt[rb + slot_offset(off8, off16, kkp, k, e, a * k + b)], 1);
    }
}

// contribution codes e * k * k + a * k + b (the host checks k * k * T < 2^31)
__global__ void k_contrib_fill(int k, int64_t T, const int32_t *__restrict__ conn,
                               const int32_t *__restrict__ row_ptr,
                               const uint8_t *__restrict__ off8, const uint16_t *__restrict__ off16, int kkp,
                               const int32_t *__restrict__ cptr, int32_t *__restrict__ cursor,
                               int32_t *__restrict__ clist)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    for (int a = 0; a < k; ++a) {
        const int32_t rb = row_ptr[conn[a * T + e]];
        for (int b = 0; b < k; ++b) {
            const int32_t slot = rb + slot_offset(off8, off16, kkp, k, e, a * k + b);
            const int32_t pos = atomicAdd(&cursor[slot], 1);
            clist[cptr[slot] + pos] = static_cast<int32_t>((e * k + a) * k + b);
        }
    }
}

// block-ordered copies of the node ids and slot offsets of every list entry, and
// a bit per local pair that is set when the target CSR entry receives three or
// more contributions (mult = contributions per entry)
__global__ void k_block_gather(int64_t L, int k, int64_t T, const int32_t *__restrict__ elems,
                               const int32_t *__restrict__ conn, const uint8_t *__restrict__ off8,
                               int kkp, const int32_t *__restrict__ row_ptr,
                               const int32_t *__restrict__ mult, int mw,
                               int32_t *__restrict__ bconn, uint8_t *__restrict__ boff,
                               uint32_t *__restrict__ bmask)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= L) return;
    const int64_t e = elems[i];
    for (int a = 0; a < k; ++a) bconn[a * L + i] = conn[a * T + e];
    const uint32_t *src = reinterpret_cast<const uint32_t *>(off8 + e * kkp);
    uint32_t *dst = reinterpret_cast<uint32_t *>(boff + i * kkp);
    for (int w = 0; w < kkp / 4; ++w) dst[w] = src[w];
    uint32_t words[4] = {0, 0, 0, 0};
    for (int a = 0; a < k; ++a) {
        const int32_t rb = row_ptr[conn[a * T + e]];
        for (int b = 0; b < k; ++b) {
            const int slot = a * k + b;
            if (mult[rb + off8[e * kkp + slot]] >= 3) words[slot >> 5] |= 1u << (slot & 31);
        }
    }
    for (int w = 0; w < mw; ++w) bmask[i * mw + w] = words[w];
}

// flag <- 1 if an off-diagonal entry receives three or more contributions
__global__ void k_offdiag_check(int k, int64_t T, const int32_t *__restrict__ conn,
                                const int32_t *__restrict__ row_ptr,
                                const uint8_t *__restrict__ off8, int kkp,
                                const int32_t *__restrict__ mult, int32_t *__restrict__ flag)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    for (int a = 0; a < k; ++a) {
        const int32_t rb = row_ptr[conn[a * T + e]];
        for (int b = 0; b < k; ++b)
            if (a != b && mult[rb + off8[e * kkp + a * k + b]] >= 3) atomicOr(flag, 1);
    }
}

// per row: offset of the diagonal inside the row, and its number of contributions
__global__ void k_diag_info(int64_t N, const int32_t *__restrict__ row_ptr,
                            const int32_t *__restrict__ col_idx,
                            const int32_t *__restrict__ mult, int32_t *__restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t lo = row_ptr[i], hi = row_ptr[i + 1];
    const int32_t beg = lo;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col_idx[mid] < i)
            lo = mid + 1;
        else
            hi = mid;
    }
    const bool found = lo < row_ptr[i + 1] && col_idx[lo] == i;
    out[i] = found ? lo - beg : 0;
    out[N + i] = found ? mult[lo] : 0;
}

inline unsigned grid_for(int64_t n, int nt) { return static_cast<unsigned>((n + nt - 1) / nt); }

template <typename X>
X *dev_alloc(size_t count)
{
    X *p = nullptr;
    LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(X)));
    return p;
}

// flag[s] = 1 if slot s has more than kReduceBatch contributions
__global__ __launch_bounds__(256) void k_long_flag(int64_t nnz, const int32_t *__restrict__ cptr,
                                                   int32_t *__restrict__ flag)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    flag[s] = cptr[s + 1] - cptr[s] > kReduceBatch ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_long_fill(int64_t nnz, const int32_t *__restrict__ flag,
                                                   const int32_t *__restrict__ pos, int32_t *__restrict__ out)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    if (flag[s]) out[pos[s]] = static_cast<int32_t>(s);
}

}  // namespace

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *d_total,
                        hipStream_t s)
{
    scan_rec<int32_t, int32_t>(in, out, n, d_total, s);
    k_write_last<int32_t><<<1, 1, 0, s>>>(out, n, d_total);
    LFEM_HIP(hipGetLastError());
}

void build_incidence(Mesh &m, hipStream_t s)
{
    const int64_t kT = static_cast<int64_t>(m.k) * m.T;
    m.ne_ptr = dev_alloc<int32_t>(m.N + 1);
    m.ne = dev_alloc<int32_t>(kT);
    int32_t *cnt = nullptr;
    int64_t *tot = nullptr;
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&cnt), (m.N + 1) * sizeof(int32_t), s));
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&tot), sizeof(int64_t), s));
    LFEM_HIP(hipMemsetAsync(cnt, 0, (m.N + 1) * sizeof(int32_t), s));
    LFEM_HIP(hipMemsetAsync(m.flags, 0, 4 * sizeof(int32_t), s));
    if (kT > 0) {
        k_inc_count<<<grid_for(kT, 256), 256, 0, s>>>(m.conn, kT, m.N, cnt, m.flags);
        LFEM_HIP(hipGetLastError());
    }
    exclusive_scan_i32(cnt, m.ne_ptr, m.N, tot, s);
    LFEM_HIP(hipMemsetAsync(cnt, 0, (m.N + 1) * sizeof(int32_t), s));
    if (kT > 0) {
        k_inc_fill<<<grid_for(kT, 256), 256, 0, s>>>(m.conn, kT, m.T, m.N, m.ne_ptr, cnt, m.ne);
        LFEM_HIP(hipGetLastError());
        k_validate<<<grid_for(m.T, 256), 256, 0, s>>>(m.conn, m.T, m.k, m.flags);
        LFEM_HIP(hipGetLastError());
    }
    if (m.N > 0) {
        k_sort_lists<<<grid_for(m.N, 256), 256, 0, s>>>(m.N, m.ne_ptr, m.ne);
        LFEM_HIP(hipGetLastError());
    }
    LFEM_HIP(hipFreeAsync(cnt, s));
    LFEM_HIP(hipFreeAsync(tot, s));
}

void build_pattern(Mesh &m, Pattern &p, hipStream_t s)
{
    p.mesh = &m;
    int32_t flags[4] = {0, 0, 0, 0};
    LFEM_HIP(hipMemcpyAsync(flags, m.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
    LFEM_HIP(hipStreamSynchronize(s));
    LFEM_REQUIRE(!flags[0], LFEM_EINVAL, "connectivity holds a node id outside [0, n_nodes)");
    LFEM_REQUIRE(!flags[1], LFEM_EINVAL, "an element lists the same node twice");

    int32_t *rowlen = nullptr;
    int64_t *tot = nullptr;
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&rowlen), (m.N + 1) * sizeof(int32_t), s));
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&tot), sizeof(int64_t), s));
    p.row_ptr = dev_alloc<int32_t>(m.N + 1);
    // elements of up to kMaxNodes8 nodes first try rows of at most 255
    // entries (byte slot maps, every scatter); a longer row (a node of very
    // high valence) switches the pattern to the 16-bit slot map and rows of up
    // to kMaxRowWide entries, which the staged and atomic scatters take
    bool wide = m.k > kMaxNodes8;
    int64_t nnz = 0;
    for (;;) {
        if (m.N > 0) {
            if (wide)
                k_rows<0, kMaxRowWide, ROW_NT_WIDE><<<grid_for(m.N, ROW_NT_WIDE), ROW_NT_WIDE, 0, s>>>(
                    m.N, m.k, m.T, m.conn, m.ne_ptr, m.ne, rowlen, nullptr, nullptr, m.flags);
            else
                k_rows<0><<<grid_for(m.N, ROW_NT), ROW_NT, 0, s>>>(m.N, m.k, m.T, m.conn, m.ne_ptr, m.ne, rowlen,
                                                                   nullptr, nullptr, m.flags);
            LFEM_HIP(hipGetLastError());
        }
        exclusive_scan_i32(rowlen, p.row_ptr, m.N, tot, s);
        LFEM_HIP(hipMemcpyAsync(&nnz, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LFEM_HIP(hipMemcpyAsync(flags, m.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
        LFEM_HIP(hipStreamSynchronize(s));
        if (!flags[2] || wide) break;
        wide = true;
        LFEM_HIP(hipMemsetAsync(m.flags + 2, 0, sizeof(int32_t), s));
    }
    LFEM_HIP(hipFreeAsync(rowlen, s));
    LFEM_HIP(hipFreeAsync(tot, s));
    LFEM_REQUIRE(!flags[2], LFEM_ERANGE, "a CSR row would hold more than 1023 entries");
    LFEM_REQUIRE(nnz < (int64_t(1) << 31), LFEM_ERANGE, "nnz does not fit in int32");
    p.nnz = nnz;
    p.col_idx = dev_alloc<int32_t>(nnz);
    if (m.N > 0) {
        if (wide)
            k_rows<1, kMaxRowWide, ROW_NT_WIDE><<<grid_for(m.N, ROW_NT_WIDE), ROW_NT_WIDE, 0, s>>>(
                m.N, m.k, m.T, m.conn, m.ne_ptr, m.ne, nullptr, p.row_ptr, p.col_idx, m.flags);
        else
            k_rows<1><<<grid_for(m.N, ROW_NT), ROW_NT, 0, s>>>(m.N, m.k, m.T, m.conn, m.ne_ptr, m.ne, nullptr,
                                                               p.row_ptr, p.col_idx, m.flags);
        LFEM_HIP(hipGetLastError());
    }
    p.kkp = (m.k * m.k + 3) / 4 * 4;
    LFEM_REQUIRE(m.k <= kMaxNodes, LFEM_EUNSUPPORTED, "element has more nodes than the slot map holds");
    if (wide) {
        p.off16 = dev_alloc<uint16_t>(static_cast<size_t>(m.k) * m.k * m.T);
        if (m.T > 0) {
            k_offsets16<<<grid_for(m.T, 256), 256, 0, s>>>(m.k, m.T, m.conn, p.row_ptr, p.col_idx, p.off16,
                                                           m.flags);
            LFEM_HIP(hipGetLastError());
        }
    } else {
        LFEM_REQUIRE(p.kkp / 4 <= kMaxSlotWords, LFEM_EUNSUPPORTED, "element has more nodes than the slot map holds");
        p.off8 = dev_alloc<uint8_t>(static_cast<size_t>(p.kkp) * m.T);
        if (m.T > 0) {
            k_offsets<<<grid_for(m.T, 256), 256, 0, s>>>(m.k, m.T, m.conn, p.row_ptr, p.col_idx, p.off8,
                                                         p.kkp, m.flags);
            LFEM_HIP(hipGetLastError());
        }
    }
    // host copies for the block schedule
    p.h_row_ptr.resize(m.N + 1);
    p.h_ne_ptr.resize(m.N + 1);
    p.h_ne.resize(static_cast<size_t>(m.k) * m.T);
    p.h_conn.resize(static_cast<size_t>(m.k) * m.T);
    LFEM_HIP(hipMemcpyAsync(p.h_row_ptr.data(), p.row_ptr, (m.N + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    LFEM_HIP(hipMemcpyAsync(p.h_ne_ptr.data(), m.ne_ptr, (m.N + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    if (m.T > 0) {
        LFEM_HIP(hipMemcpyAsync(p.h_ne.data(), m.ne, p.h_ne.size() * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
        LFEM_HIP(hipMemcpyAsync(p.h_conn.data(), m.conn, p.h_conn.size() * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
    }
    LFEM_HIP(hipMemcpyAsync(flags, m.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
    LFEM_HIP(hipStreamSynchronize(s));
    LFEM_REQUIRE(!flags[3], LFEM_EHIP, "slot map: a local pair was not found in its row");
    int max_row = 0;
    for (int64_t i = 0; i < m.N; ++i)
        max_row = std::max(max_row, p.h_row_ptr[i + 1] - p.h_row_ptr[i]);
    p.max_row = max_row;
}

void build_staged(Mesh &m, Pattern &p, hipStream_t s)
{
    if (p.cptr) return;
    LFEM_REQUIRE(static_cast<int64_t>(m.k) * m.k * m.T < (int64_t(1) << 31), LFEM_EUNSUPPORTED,
                 "staged scatter supports fewer than 2^31 / k^2 elements");
    const int64_t kkT = static_cast<int64_t>(m.k) * m.k * m.T;
    int32_t *cnt = nullptr;
    int64_t *tot = nullptr;
    p.cptr = dev_alloc<int32_t>(p.nnz + 1);
    p.clist = dev_alloc<int32_t>(kkT);
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&cnt), (p.nnz + 1) * sizeof(int32_t), s));
    LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&tot), sizeof(int64_t), s));
    LFEM_HIP(hipMemsetAsync(cnt, 0, (p.nnz + 1) * sizeof(int32_t), s));
    if (m.T > 0) {
        k_contrib_count<<<grid_for(m.T, 256), 256, 0, s>>>(m.k, m.T, m.conn, p.row_ptr, p.off8,
                                                           p.kkp, cnt, p.off16);
        LFEM_HIP(hipGetLastError());
    }
    exclusive_scan_i32(cnt, p.cptr, p.nnz, tot, s);
    LFEM_HIP(hipMemsetAsync(cnt, 0, (p.nnz + 1) * sizeof(int32_t), s));
    if (m.T > 0) {
        k_contrib_fill<<<grid_for(m.T, 256), 256, 0, s>>>(m.k, m.T, m.conn, p.row_ptr, p.off8, p.off16,
                                                          p.kkp, p.cptr, cnt, p.clist);
        LFEM_HIP(hipGetLastError());
    }
    if (p.nnz > 0) {
        k_sort_lists<<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, p.cptr, p.clist);
        LFEM_HIP(hipGetLastError());
    }
    // the slots with long lists, in ascending order: flag, scan, fill
    p.nlong = 0;
    if (p.nnz > 0) {
        int32_t *pos = nullptr;
        LFEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&pos), (p.nnz + 1) * sizeof(int32_t), s));
        k_long_flag<<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, p.cptr, cnt);
        LFEM_HIP(hipGetLastError());
        exclusive_scan_i32(cnt, pos, p.nnz, tot, s);
        int64_t nlong = 0;
        LFEM_HIP(hipMemcpyAsync(&nlong, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LFEM_HIP(hipStreamSynchronize(s));
        LFEM_REQUIRE(nlong >= 0 && nlong <= p.nnz, LFEM_EHIP, "long-list count out of range");
        p.nlong = nlong;
        p.long_slots = dev_alloc<int32_t>(nlong);
        if (nlong > 0) {
            k_long_fill<<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, cnt, pos, p.long_slots);
            LFEM_HIP(hipGetLastError());
        }
        LFEM_HIP(hipFreeAsync(pos, s));
    }
    LFEM_HIP(hipFreeAsync(cnt, s));
    LFEM_HIP(hipFreeAsync(tot, s));
}

void free_schedule(BlockSchedule &b)
{
    dev_free(b.row_begin);
    dev_free(b.elem_ptr);
    dev_free(b.colors);
    dev_free(b.bconn);
    dev_free(b.boff);
    dev_free(b.bmask);
    dev_free(b.bnode);
    dev_free(b.brec);
    dev_free(b.bord);
    dev_free(b.bord_ptr);
    b = BlockSchedule{};
}

// Host: contiguous row blocks with at most `cap` CSR values and `max_rows`
// rows; each block lists every element touching one of its rows (halo
// elements appear in several blocks).
//
// Entries that receive at most two contributions are summed in any order (the
// value starts at +0, 0 + a = a, a + b = b + a).  Entries with three or more
// need a fixed order:
//  - side mode (only diagonal entries have >= 3 contributions: curves, surfaces,
//    planar meshes): lists are in element order; every such diagonal
//    contribution gets its own LDS side slot, slots of one entry are contiguous
//    in element order, and the entry is summed from its slots after one barrier;
//  - colour mode (otherwise): lists are greedily coloured so that two elements
//    of one colour share no node and ordered by colour, then element id; the
//    ordered contributions are added one colour at a time.
void build_schedule(Mesh &m, Pattern &p, int cap, int max_rows, hipStream_t s)
{
    LFEM_REQUIRE(max_rows >= 1 && max_rows <= kBlockMaxRows, LFEM_EINVAL, "rows per block out of range");
    LFEM_REQUIRE(m.p <= 2, LFEM_EUNSUPPORTED, "block schedules cover orders 1 and 2");
    LFEM_REQUIRE(p.off8 != nullptr, LFEM_EUNSUPPORTED,
                 "block schedules need rows of at most 255 entries (byte slot maps)");
    free_schedule(p.sched);
    ++p.sched_gen;
    BlockSchedule &b = p.sched;
    b.cap = cap;
    LFEM_REQUIRE(p.max_row <= cap, LFEM_EINVAL, "block capacity below the longest row");
    const int64_t T = m.T;
    const int k = m.k;
    // contributions per CSR entry, off-diagonal check, diagonal position and count per row
    int32_t *mult = dev_alloc<int32_t>(p.nnz + 1);
    int32_t *flag = mult + p.nnz;
    int32_t *dinfo = dev_alloc<int32_t>(2 * m.N + 1);
    LFEM_HIP(hipMemsetAsync(mult, 0, (p.nnz + 1) * sizeof(int32_t), s));
    if (T > 0) {
        k_contrib_count<<<grid_for(T, 256), 256, 0, s>>>(k, T, m.conn, p.row_ptr, p.off8, p.kkp,
                                                         mult);
        LFEM_HIP(hipGetLastError());
        k_offdiag_check<<<grid_for(T, 256), 256, 0, s>>>(k, T, m.conn, p.row_ptr, p.off8, p.kkp,
                                                         mult, flag);
        LFEM_HIP(hipGetLastError());
    }
    if (m.N > 0) {
        k_diag_info<<<grid_for(m.N, 256), 256, 0, s>>>(m.N, p.row_ptr, p.col_idx, mult, dinfo);
        LFEM_HIP(hipGetLastError());
    }
    std::vector<int32_t> hd(2 * m.N);
    int32_t hflag = 0;
    LFEM_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (m.N > 0)
        LFEM_HIP(hipMemcpyAsync(hd.data(), dinfo, 2 * m.N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LFEM_HIP(hipStreamSynchronize(s));
    dev_free(dinfo);
    const int32_t *dpos = hd.data();         // diagonal's offset inside its row
    const int32_t *dmul = hd.data() + m.N;   // contributions to the diagonal entry
    // (tetrahedral meshes always take colour mode: their side-slot kernels would
    // need the Q-point data of 11 points in registers)
    b.side_mode = hflag == 0 && m.d <= 2;
    b.diag_only = b.side_mode;

    std::vector<int32_t> rb, ep, el, ordp, rec;
    std::vector<uint8_t> col;
    std::vector<uint32_t> node;       // side mode: [len][k] row start | side slot << 16
    std::vector<uint32_t> ord;        // per ordered entry: (lds index | count << 16, first slot)
    rb.push_back(0);
    ep.push_back(0);
    ordp.push_back(0);
    std::vector<int32_t> stamp(static_cast<size_t>(T), -1);
    std::vector<uint64_t> used(b.side_mode ? 0 : static_cast<size_t>(m.N), 0);
    std::vector<int32_t> list, first, rank;
    std::vector<std::pair<uint8_t, int32_t>> keyed;
    const int32_t *rp = p.h_row_ptr.data();
    const size_t max_elems = b.side_mode ? static_cast<size_t>(kSideThreads) * (m.p == 1 ? 4 : 1)
                                         : static_cast<size_t>(T) + 1;
    int64_t total = 0;
    int32_t r0 = 0;
    int nb = 0;
    b.max_colors = 1;
    while (r0 < m.N) {
        // grow the block while its values (plus, in side mode, its side slots)
        // fit and, in side mode, its element list stays within max_elems
        int32_t r1 = r0;
        int64_t slots = 0;
        list.clear();
        while (r1 < m.N && r1 - r0 < max_rows) {
            const int64_t add = (b.side_mode && dmul[r1] >= 3) ? dmul[r1] : 0;
            if (rp[r1 + 1] - rp[r0] + slots + add > cap) break;
            const size_t before = list.size();
            for (int32_t q = p.h_ne_ptr[r1]; q < p.h_ne_ptr[r1 + 1]; ++q) {
                const int32_t e = static_cast<int32_t>(p.h_ne[q] % T);
                if (stamp[e] != nb) {
                    stamp[e] = nb;
                    list.push_back(e);
                }
            }
            if (list.size() > max_elems && r1 > r0) {
                for (size_t i = before; i < list.size(); ++i) stamp[list[i]] = -1;
                list.resize(before);
                break;
            }
            slots += add;
            ++r1;
        }
        LFEM_REQUIRE(r1 > r0, LFEM_EINVAL, "block capacity below one row and its side slots");
        std::sort(list.begin(), list.end());
        const int32_t o0 = static_cast<int32_t>(ord.size() / 2);
        if (b.side_mode) {
            // side slots of the ordered diagonals of this block, in element order
            first.assign(r1 - r0, -1);
            rank.assign(r1 - r0, 0);
            int32_t nslot = 0;
            for (int32_t r = r0; r < r1; ++r)
                if (dmul[r] >= 3) {
                    first[r - r0] = nslot;
                    LFEM_REQUIRE(dmul[r] < 256, LFEM_EUNSUPPORTED, "diagonal with >255 contributions");
                    ord.push_back(static_cast<uint32_t>(rp[r] - rp[r0] + dpos[r]) |
                                  (static_cast<uint32_t>(dmul[r]) << 16));
                    ord.push_back(static_cast<uint32_t>(nslot));
                    nslot += dmul[r];
                }
            LFEM_REQUIRE(nslot < 65535 && rp[r1] - rp[r0] < 65535, LFEM_EUNSUPPORTED,
                         "block too large for 16-bit side slots");
            b.max_side = std::max(b.max_side, static_cast<int>(nslot));
            for (int32_t e : list) {
                el.push_back(e);
                col.push_back(0);
                for (int a = 0; a < k; ++a) {
                    uint32_t start = 0xffff, slot = 0xffff;
                    const int32_t nd = p.h_conn[a * T + e];
                    if (nd >= r0 && nd < r1) {
                        start = static_cast<uint32_t>(rp[nd] - rp[r0]);
                        if (first[nd - r0] >= 0)
                            slot = static_cast<uint32_t>(first[nd - r0] + rank[nd - r0]++);
                    }
                    node.push_back(start | (slot << 16));
                }
            }
            ordp.push_back(static_cast<int32_t>(ord.size() / 2));
        } else {
            keyed.clear();
            for (int32_t e : list) {
                uint64_t mask = 0;
                for (int a = 0; a < k; ++a) mask |= used[p.h_conn[a * T + e]];
                LFEM_REQUIRE(~mask != 0, LFEM_EUNSUPPORTED, "block colouring needs more than 64 colours");
                const int c = __builtin_ctzll(~mask);
                for (int a = 0; a < k; ++a) used[p.h_conn[a * T + e]] |= (uint64_t(1) << c);
                keyed.emplace_back(static_cast<uint8_t>(c), e);
                b.max_colors = std::max(b.max_colors, c + 1);
            }
            for (int32_t e : list)
                for (int a = 0; a < k; ++a) used[p.h_conn[a * T + e]] = 0;
            std::stable_sort(keyed.begin(), keyed.end(),
                             [](const std::pair<uint8_t, int32_t> &x,
                                const std::pair<uint8_t, int32_t> &y) { return x.first < y.first; });
            for (auto &kv : keyed) {
                el.push_back(kv.second);
                col.push_back(kv.first);
            }
            ordp.push_back(o0);
        }
        const int32_t o1 = ordp.back();
        b.max_ord = std::max(b.max_ord, static_cast<int>(o1 - o0));
        const int32_t e1 = static_cast<int32_t>(el.size());
        const int32_t e0 = e1 - static_cast<int32_t>(list.size());
        rec.insert(rec.end(), {e0, e1, r0, r1, rp[r0], rp[r1] - rp[r0], o0, o1});
        total += static_cast<int64_t>(list.size());
        b.max_rows = std::max(b.max_rows, static_cast<int>(r1 - r0));
        b.max_elems = std::max(b.max_elems, static_cast<int>(list.size()));
        rb.push_back(r1);
        ep.push_back(e1);
        r0 = r1;
        ++nb;
    }
    b.nb = nb;
    b.len = static_cast<int64_t>(el.size());
    b.halo = T > 0 ? static_cast<double>(total) / static_cast<double>(T) : 0.0;
    b.row_begin = dev_alloc<int32_t>(rb.size());
    b.elem_ptr = dev_alloc<int32_t>(ep.size());
    b.colors = dev_alloc<uint8_t>(col.size());
    b.bconn = dev_alloc<int32_t>(static_cast<size_t>(k) * el.size());
    b.boff = dev_alloc<uint8_t>(static_cast<size_t>(p.kkp) * el.size());
    b.mw = (k * k + 31) / 32;
    b.bmask = dev_alloc<uint32_t>(static_cast<size_t>(b.mw) * el.size());
    b.bnode = dev_alloc<uint32_t>(node.size());
    b.bord = dev_alloc<uint32_t>(ord.size());
    b.bord_ptr = dev_alloc<int32_t>(ordp.size());
    b.brec = dev_alloc<int32_t>(rec.size());
    int32_t *elems = dev_alloc<int32_t>(el.size());
    LFEM_HIP(hipMemcpyAsync(b.row_begin, rb.data(), rb.size() * 4, hipMemcpyHostToDevice, s));
    LFEM_HIP(hipMemcpyAsync(b.elem_ptr, ep.data(), ep.size() * 4, hipMemcpyHostToDevice, s));
    LFEM_HIP(hipMemcpyAsync(b.bord_ptr, ordp.data(), ordp.size() * 4, hipMemcpyHostToDevice, s));
    LFEM_HIP(hipMemcpyAsync(b.brec, rec.data(), rec.size() * 4, hipMemcpyHostToDevice, s));
    if (!node.empty())
        LFEM_HIP(hipMemcpyAsync(b.bnode, node.data(), node.size() * 4, hipMemcpyHostToDevice, s));
    if (!ord.empty())
        LFEM_HIP(hipMemcpyAsync(b.bord, ord.data(), ord.size() * 4, hipMemcpyHostToDevice, s));
    if (!el.empty()) {
        LFEM_HIP(hipMemcpyAsync(elems, el.data(), el.size() * 4, hipMemcpyHostToDevice, s));
        LFEM_HIP(hipMemcpyAsync(b.colors, col.data(), col.size(), hipMemcpyHostToDevice, s));
        k_block_gather<<<grid_for(b.len, 256), 256, 0, s>>>(b.len, k, T, elems, m.conn, p.off8,
                                                            p.kkp, p.row_ptr, mult, b.mw, b.bconn,
                                                            b.boff, b.bmask);
        LFEM_HIP(hipGetLastError());
    }
    LFEM_HIP(hipStreamSynchronize(s));
    dev_free(elems);
    dev_free(mult);
}

}  // namespace lfem
