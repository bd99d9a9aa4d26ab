// Numeric phase: fused geometry + local matrices + scatter into CSR values.
//
// Per element and quadrature point (section 3.2 and Listing 1 (c)-(e)):
//   J = DF = sum_a x_a (grad_hat phi_a)^T              (n x d)
//   G = J^T J,  mu = sqrt(det G)  (curve / surface: |t| or |t1 x t2|),
//               mu = |det J|       (bulk)
//   K = G^{-1}: the tangential gradient of phi_a is J K g_a, so
//   grad phi_a . grad phi_b = g_a^T K g_b  (equal to the paper's C^T [g;0]
//   with C = L^{-1}, L = [J, normal]; no normal vector is needed)
//   M_loc[a][b] += w mu c_h phi_a phi_b,  A_loc[a][b] += w mu a_h g_a^T K g_b
// Only the k(k+1)/2 pairs a <= b are formed (both matrices are symmetric).
//
// Scatter variants:
//   atomic  - FP64 atomics into zeroed values (order not fixed)
//   staged  - local matrices written structure-of-arrays, then one thread per
//             CSR slot sums its contribution list in ascending element order
//   blocked - one workgroup owns a contiguous block of rows whose values live
//             in LDS; it recomputes every element touching the block and
//             adds them colour by colour (elements of one colour share no
//             node), then writes the block once.  Fixed order.
#include <cmath>

#include "element.hpp"
#include "lfem_internal.hpp"

namespace lfem {

namespace {

// Local matrices of one element from its node coordinates x.  NM mass-class
// outputs (slot s uses nodal coefficient cm[s] or 1 when null), HA: one
// stiffness output (coefficient ca or 1).  Returns the number of degenerate
// quadrature points.
template <class E, int NM, bool HA>
__device__ __forceinline__ int element_local(
    const int32_t (&nid)[E::k], const double (&x)[E::n][E::k], const double *__restrict__ tab,
    int Q, const double *__restrict__ cm0, const double *__restrict__ cm1,
    const double *__restrict__ ca, double (&LM)[NM > 0 ? NM : 1][E::np], double (&LA)[E::np])
{
    double J0[E::n][E::d], H[E::n][E::nh > 0 ? E::nh : 1];
    jacobian_setup<E>(x, J0, H);
    double cmv[NM > 0 ? NM : 1][E::k];
    double cav[E::k];
    const double *cms[2] = {cm0, cm1};
#pragma unroll
    for (int s = 0; s < NM; ++s)
        if (cms[s]) {
#pragma unroll
            for (int a = 0; a < E::k; ++a) cmv[s][a] = cms[s][nid[a]];
        }
    if (HA && ca) {
#pragma unroll
        for (int a = 0; a < E::k; ++a) cav[a] = ca[nid[a]];
    }
#pragma unroll
    for (int s = 0; s < NM; ++s)
#pragma unroll
        for (int p = 0; p < E::np; ++p) LM[s][p] = 0.0;
#pragma unroll
    for (int p = 0; p < E::np; ++p) LA[p] = 0.0;
    int bad = 0;
    for (int q = 0; q < Q; ++q) {
        const double *__restrict__ t = tab + q * E::stride;
        double J[E::n][E::d];
        jacobian_at<E>(J0, H, t + E::off_xi, J);
        double K[E::d][E::d], mu;
        geometry<E>(J, K, mu);
        bad += !(mu > 0.0 && mu < INFINITY);
        const double wmu = t[0] * mu;
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            double f = wmu;
            if (cms[s]) {
                double ch = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) ch = fma(cmv[s][a], t[E::off_phi + a], ch);
                f *= ch;
            }
#pragma unroll
            for (int p = 0; p < E::np; ++p) LM[s][p] = fma(f, t[E::off_pp + p], LM[s][p]);
        }
        if constexpr (HA) {
            double fa = wmu;
            if (ca) {
                double ah = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) ah = fma(cav[a], t[E::off_phi + a], ah);
                fa *= ah;
            }
            // scale K once; then A_loc[a][b] += g_a^T (fa K) g_b
#pragma unroll
            for (int m = 0; m < E::d; ++m)
#pragma unroll
                for (int l = 0; l < E::d; ++l) K[m][l] *= fa;
            double h[E::k][E::d];
#pragma unroll
            for (int a = 0; a < E::k; ++a)
#pragma unroll
                for (int m = 0; m < E::d; ++m) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < E::d; ++l) acc = fma(K[m][l], t[E::off_g + a * E::d + l], acc);
                    h[a][m] = acc;
                }
            int p = 0;
#pragma unroll
            for (int a = 0; a < E::k; ++a)
#pragma unroll
                for (int b = a; b < E::k; ++b) {
                    double acc = LA[p];
#pragma unroll
                    for (int m = 0; m < E::d; ++m) acc = fma(h[a][m], t[E::off_g + b * E::d + m], acc);
                    LA[p] = acc;
                    ++p;
                }
        }
    }
    return bad;
}

template <int K>
__host__ __device__ constexpr int pair_index(int a, int b)
{
    // upper-triangle row-major index of (min, max)
    return a <= b ? a * K - a * (a - 1) / 2 + (b - a) : b * K - b * (b - 1) / 2 + (a - b);
}

template <class E, int NM, bool HA>
__device__ __forceinline__ double local_value(int mat, int a, int b,
                                              const double (&LM)[NM > 0 ? NM : 1][E::np],
                                              const double (&LA)[E::np])
{
    const int p = pair_index<E::k>(a, b);
    return mat < NM ? LM[mat][p] : LA[p];
}

// ---------------------------------------------------------------------------
// atomic variant
// ---------------------------------------------------------------------------
template <class E, int NM, bool HA>
__global__ __launch_bounds__(256) void k_atomic(
    const double *__restrict__ coords, const int32_t *__restrict__ conn,
    const double *__restrict__ tab, int64_t N, int64_t T, int Q, const double *__restrict__ cm0,
    const double *__restrict__ cm1, const double *__restrict__ ca,
    const int32_t *__restrict__ row_ptr, const uint8_t *__restrict__ off8, int kkp,
    double *__restrict__ v0, double *__restrict__ v1, double *__restrict__ v2,
    unsigned long long *__restrict__ degenerate)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    int32_t nid[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    double x[E::n][E::k];
    gather_coords<E>(nid, coords, N, x);
    double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
    const int bad = element_local<E, NM, HA>(nid, x, tab, Q, cm0, cm1, ca, LM, LA);
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
    constexpr int NMAT = NM + (HA ? 1 : 0);
    double *outs[3] = {v0, v1, v2};
    const uint8_t *o = off8 + e * kkp;
#pragma unroll
    for (int a = 0; a < E::k; ++a) {
        const int32_t rb = row_ptr[nid[a]];
#pragma unroll
        for (int b = 0; b < E::k; ++b) {
            const int32_t slot = rb + o[a * E::k + b];
#pragma unroll
            for (int mat = 0; mat < NMAT; ++mat)
                unsafeAtomicAdd(outs[mat] + slot, local_value<E, NM, HA>(mat, a, b, LM, LA));
        }
    }
}

// ---------------------------------------------------------------------------
// staged variant
// ---------------------------------------------------------------------------
template <class E, int NM, bool HA>
__global__ __launch_bounds__(256) void k_stage(
    const double *__restrict__ coords, const int32_t *__restrict__ conn,
    const double *__restrict__ tab, int64_t N, int64_t T, int Q, const double *__restrict__ cm0,
    const double *__restrict__ cm1, const double *__restrict__ ca, double *__restrict__ stage,
    unsigned long long *__restrict__ degenerate)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    int32_t nid[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    double x[E::n][E::k];
    gather_coords<E>(nid, coords, N, x);
    double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
    const int bad = element_local<E, NM, HA>(nid, x, tab, Q, cm0, cm1, ca, LM, LA);
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
#pragma unroll
    for (int s = 0; s < NM; ++s)
#pragma unroll
        for (int p = 0; p < E::np; ++p) stage[(s * E::np + p) * T + e] = LM[s][p];
    if constexpr (HA) {
#pragma unroll
        for (int p = 0; p < E::np; ++p) stage[(NM * E::np + p) * T + e] = LA[p];
    }
}

template <int K, int NMAT>
__global__ __launch_bounds__(256) void k_reduce(int64_t nnz, int64_t T,
                                                const int32_t *__restrict__ cptr,
                                                const int32_t *__restrict__ clist,
                                                const double *__restrict__ stage,
                                                double *__restrict__ v0, double *__restrict__ v1,
                                                double *__restrict__ v2)
{
    constexpr int NP = K * (K + 1) / 2;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    double acc[NMAT];
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat) acc[mat] = 0.0;
    const int32_t b = cptr[s], end = cptr[s + 1];
    for (int32_t c = b; c < end; ++c) {
        const int32_t code = clist[c];
        const int64_t e = code >> 7;
        const int ab = code & 127;
        const int a = ab / K, bb = ab - a * K;
        const int p = pair_index<K>(a, bb);
#pragma unroll
        for (int mat = 0; mat < NMAT; ++mat) acc[mat] += stage[(mat * NP + p) * T + e];
    }
    double *outs[3] = {v0, v1, v2};
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat) outs[mat][s] = acc[mat];
}

// ---------------------------------------------------------------------------
// blocked variant
// ---------------------------------------------------------------------------
// Workgroup i runs on XCD i % 8; give each XCD a contiguous range of blocks so
// that neighbouring blocks (which share halo elements and nodes) share an L2.
__device__ __forceinline__ int xcd_block(int bid, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = bid & 7, local = bid >> 3;
    return xcd * per + min(xcd, rem) + local;
}

// add the contributions whose "ordered" bit equals ORDERED into the LDS block
template <class E, int NM, bool HA, bool ORDERED, int KW, int MW>
__device__ __forceinline__ void scatter_lds(const int32_t (&rb)[E::k], const uint32_t (&ow)[KW],
                                            const uint32_t (&om)[MW],
                                            const double (&LM)[NM > 0 ? NM : 1][E::np],
                                            const double (&LA)[E::np], double *lds, int cap)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
#pragma unroll
    for (int a = 0; a < E::k; ++a) {
        if (rb[a] < 0) continue;
#pragma unroll
        for (int b = 0; b < E::k; ++b) {
            const int slot = a * E::k + b;
            const bool ordered = (om[slot >> 5] >> (slot & 31)) & 1u;
            if (ordered != ORDERED) continue;
            const int32_t li = rb[a] + static_cast<int32_t>((ow[slot >> 2] >> (8 * (slot & 3))) & 0xffu);
#pragma unroll
            for (int mat = 0; mat < NMAT; ++mat)
                __hip_atomic_fetch_add(&lds[mat * cap + li], local_value<E, NM, HA>(mat, a, b, LM, LA),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

template <class E, int NM, bool HA, int NT, bool SIDE>
__global__ __launch_bounds__(NT) void k_blocked(
    const double *__restrict__ coords, const double *__restrict__ tab, int64_t N, int Q,
    const double *__restrict__ cm0, const double *__restrict__ cm1, const double *__restrict__ ca,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ brow,
    const int32_t *__restrict__ beptr, const uint8_t *__restrict__ bcol,
    const int32_t *__restrict__ bconn, const uint8_t *__restrict__ boff,
    const uint32_t *__restrict__ bmask, const uint16_t *__restrict__ bside,
    const uint32_t *__restrict__ bord, const int32_t *__restrict__ bord_ptr, int64_t blen, int nb,
    int cap, int max_side, double *__restrict__ v0, double *__restrict__ v1,
    double *__restrict__ v2, unsigned long long *__restrict__ degenerate)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    constexpr int KKP = (E::k * E::k + 3) / 4 * 4;
    constexpr int MW = (E::k * E::k + 31) / 32;
    constexpr int KS = (E::k + 1) / 2 * 2;
    // LDS: per matrix a region of cap doubles holding the block's values and, in
    // side mode, its side slots right after them; then the block's row offsets
    extern __shared__ double lds[];
    int32_t *rp = reinterpret_cast<int32_t *>(lds + NMAT * cap);
    const int tid = threadIdx.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int32_t e0 = beptr[blk], e1 = beptr[blk + 1];
    const int32_t r0 = brow[blk], r1 = brow[blk + 1];
    // element data of one chunk: colour, node ids, slot offsets, coordinates.
    // The first chunk's loads are issued before the LDS set-up so that the two
    // chains of dependent loads overlap.
    int color = -1;
    int32_t nid[E::k];
    uint32_t ow[KKP / 4];
    uint32_t om[SIDE ? 1 : MW];
    uint32_t osd[SIDE ? KS / 2 : 1];
    double x[E::n][E::k];
    auto load_chunk = [&](int32_t idx) {
        color = -1;
        if (idx < e1) {
            color = SIDE ? 0 : bcol[idx];
#pragma unroll
            for (int a = 0; a < E::k; ++a) nid[a] = bconn[a * blen + idx];
            const uint32_t *op = reinterpret_cast<const uint32_t *>(boff + static_cast<int64_t>(idx) * KKP);
#pragma unroll
            for (int w = 0; w < KKP / 4; ++w) ow[w] = op[w];
            if constexpr (SIDE) {
                const uint32_t *sp = reinterpret_cast<const uint32_t *>(bside + static_cast<int64_t>(idx) * KS);
#pragma unroll
                for (int w = 0; w < KS / 2; ++w) osd[w] = sp[w];
            } else {
#pragma unroll
                for (int w = 0; w < MW; ++w) om[w] = bmask[static_cast<int64_t>(idx) * MW + w];
            }
            gather_coords<E>(nid, coords, N, x);
        }
    };
    load_chunk(e0 + tid);
    const int32_t base = row_ptr[r0];
    const int32_t nloc = row_ptr[r1] - base;
    for (int i = tid; i < nloc; i += NT)
#pragma unroll
        for (int mat = 0; mat < NMAT; ++mat) lds[mat * cap + i] = 0.0;
    for (int i = tid; i <= r1 - r0; i += NT) rp[i] = row_ptr[r0 + i] - base;
    __syncthreads();
    int bad = 0;
    for (int32_t c0 = e0; c0 < e1; c0 += NT) {
        if (c0 != e0) load_chunk(c0 + tid);
        int32_t rb[E::k];
        double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
        if (color >= 0) {
#pragma unroll
            for (int a = 0; a < E::k; ++a)
                rb[a] = (nid[a] >= r0 && nid[a] < r1) ? rp[nid[a] - r0] : -1;
            bad += element_local<E, NM, HA>(nid, x, tab, Q, cm0, cm1, ca, LM, LA);
        }
        if constexpr (SIDE) {
            // Every contribution except the ordered diagonals goes to LDS at once
            // (order-free, at most two per entry); ordered diagonal contributions
            // are stored in their own side slots and summed after the loop.
            if (color >= 0) {
#pragma unroll
                for (int a = 0; a < E::k; ++a) {
                    if (rb[a] < 0) continue;
                    const uint32_t sslot = (osd[a >> 1] >> (16 * (a & 1))) & 0xffffu;
#pragma unroll
                    for (int b = 0; b < E::k; ++b) {
                        const int slot = a * E::k + b;
                        if (a == b && sslot != 0xffffu) {
#pragma unroll
                            for (int mat = 0; mat < NMAT; ++mat)
                                lds[mat * cap + nloc + sslot] = local_value<E, NM, HA>(mat, a, a, LM, LA);
                            continue;
                        }
                        const int32_t li = rb[a] + static_cast<int32_t>((ow[slot >> 2] >> (8 * (slot & 3))) & 0xffu);
#pragma unroll
                        for (int mat = 0; mat < NMAT; ++mat)
                            __hip_atomic_fetch_add(&lds[mat * cap + li], local_value<E, NM, HA>(mat, a, b, LM, LA),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
        } else {
            // Entries with at most two contributions: LDS starts at +0, so 0 + a = a
            // exactly and a + b = b + a -- the result does not depend on the order and
            // all threads add at once (ds_add_f64, no return).
            if (color >= 0) scatter_lds<E, NM, HA, false>(rb, ow, om, LM, LA, lds, cap);
            // Entries with three or more contributions: one colour at a time (elements
            // of one colour share no node), so their summation order is fixed.
            const int cfirst = bcol[c0];
            const int clast = bcol[min(c0 + NT, e1) - 1];
            for (int c = cfirst; c <= clast; ++c) {
                __syncthreads();
                if (color == c) scatter_lds<E, NM, HA, true>(rb, ow, om, LM, LA, lds, cap);
            }
        }
    }
    if constexpr (SIDE) {
        // ordered diagonals: sum each entry's side slots in element order
        __syncthreads();
        const int32_t o0 = bord_ptr[blk], o1 = bord_ptr[blk + 1];
        for (int32_t r = o0 + tid; r < o1; r += NT) {
            const uint32_t w0 = bord[2 * static_cast<int64_t>(r)];
            const uint32_t first = bord[2 * static_cast<int64_t>(r) + 1];
            const uint32_t idx = w0 & 0xffffu, cnt = w0 >> 16;
#pragma unroll
            for (int mat = 0; mat < NMAT; ++mat) {
                double acc = 0.0;
                for (uint32_t j = 0; j < cnt; ++j) acc += lds[mat * cap + nloc + first + j];
                lds[mat * cap + idx] = acc;
            }
        }
    }
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
    __syncthreads();
    double *outs[3] = {v0, v1, v2};
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat)
        for (int i = tid; i < nloc; i += NT) outs[mat][base + i] = lds[mat * cap + i];
}

__global__ void k_fill_zero(double *__restrict__ x, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

inline unsigned grid_for(int64_t n, int nt) { return static_cast<unsigned>((n + nt - 1) / nt); }

struct Outs {
    const double *cm0 = nullptr, *cm1 = nullptr, *ca = nullptr;
    double *v[3] = {nullptr, nullptr, nullptr};
    int nm = 0;
    bool ha = false;
};

Outs arrange(const NumericOut &o)
{
    Outs r;
    if (o.what & LFEM_M) {
        r.v[r.nm] = o.vals_m;
        if (r.nm == 0) r.cm0 = nullptr; else r.cm1 = nullptr;
        ++r.nm;
    }
    if (o.what & LFEM_MC) {
        r.v[r.nm] = o.vals_mc;
        if (r.nm == 0) r.cm0 = o.coef_c; else r.cm1 = o.coef_c;
        ++r.nm;
    }
    if (o.what & LFEM_A) {
        r.ha = true;
        r.v[r.nm] = o.vals_a;
        r.ca = o.coef_a;
    }
    return r;
}

template <class E, int NM, bool HA, int NT, bool SIDE>
void launch_blocked(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s);

template <class E, int NM, bool HA>
void run(Mesh &m, Pattern &p, const Outs &o, int variant, hipStream_t s)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    if (m.T == 0 || p.nnz == 0) {
        for (int mat = 0; mat < NMAT; ++mat)
            if (p.nnz > 0) {
                k_fill_zero<<<grid_for(p.nnz, 256), 256, 0, s>>>(o.v[mat], p.nnz);
            }
        return;
    }
    if (variant == LFEM_SCATTER_ATOMIC) {
        for (int mat = 0; mat < NMAT; ++mat)
            k_fill_zero<<<grid_for(p.nnz, 256), 256, 0, s>>>(o.v[mat], p.nnz);
        k_atomic<E, NM, HA><<<grid_for(m.T, 256), 256, 0, s>>>(
            m.coords, m.conn, m.tab, m.N, m.T, m.Q, o.cm0, o.cm1, o.ca, p.row_ptr, p.off8, p.kkp,
            o.v[0], o.v[1], o.v[2], m.degenerate);
        LFEM_HIP(hipGetLastError());
        return;
    }
    if (variant == LFEM_SCATTER_STAGED) {
        build_staged(m, p, s);
        const size_t need = static_cast<size_t>(NMAT) * E::np * m.T * sizeof(double);
        if (p.stage_bytes < need) {
            dev_free(p.stage);
            p.stage = nullptr;
            p.stage_bytes = 0;
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&p.stage), need));
            p.stage_bytes = need;
        }
        k_stage<E, NM, HA><<<grid_for(m.T, 256), 256, 0, s>>>(
            m.coords, m.conn, m.tab, m.N, m.T, m.Q, o.cm0, o.cm1, o.ca, p.stage, m.degenerate);
        LFEM_HIP(hipGetLastError());
        k_reduce<E::k, NMAT><<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, m.T, p.cptr, p.clist,
                                                                   p.stage, o.v[0], o.v[1], o.v[2]);
        LFEM_HIP(hipGetLastError());
        return;
    }
    // blocked
    LFEM_REQUIRE(p.sched.nb > 0, LFEM_EUNSUPPORTED, "pattern has no block schedule");
    constexpr int NT = 256;
    const bool side = p.sched.side_mode;
    const size_t lds = static_cast<size_t>(NMAT) * p.sched.cap * sizeof(double) +
                       static_cast<size_t>(p.sched.max_rows + 1) * sizeof(int32_t);
    LFEM_REQUIRE(lds <= 160 * 1024, LFEM_EUNSUPPORTED, "block schedule exceeds LDS");
    if (side) return launch_blocked<E, NM, HA, NT, true>(m, p, o, lds, s);
    return launch_blocked<E, NM, HA, NT, false>(m, p, o, lds, s);
}

template <class E, int NM, bool HA, int NT, bool SIDE>
void launch_blocked(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s)
{
    auto kern = k_blocked<E, NM, HA, NT, SIDE>;
    static thread_local size_t attr_lds = 64 * 1024;
    if (lds > attr_lds) {
        LFEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds)));
        attr_lds = lds;
    }
    kern<<<p.sched.nb, NT, lds, s>>>(m.coords, m.tab, m.N, m.Q, o.cm0, o.cm1, o.ca, p.row_ptr,
                                     p.sched.row_begin, p.sched.elem_ptr, p.sched.colors,
                                     p.sched.bconn, p.sched.boff, p.sched.bmask, p.sched.bside,
                                     p.sched.bord, p.sched.bord_ptr, p.sched.len, p.sched.nb,
                                     p.sched.cap, p.sched.max_side, o.v[0], o.v[1], o.v[2],
                                     m.degenerate);
    LFEM_HIP(hipGetLastError());
}

template <class E>
void run_type(Mesh &m, Pattern &p, const Outs &o, int variant, hipStream_t s)
{
    switch (o.nm * 2 + (o.ha ? 1 : 0)) {
    case 1: run<E, 0, true>(m, p, o, variant, s); break;
    case 2: run<E, 1, false>(m, p, o, variant, s); break;
    case 3: run<E, 1, true>(m, p, o, variant, s); break;
    case 4: run<E, 2, false>(m, p, o, variant, s); break;
    case 5: run<E, 2, true>(m, p, o, variant, s); break;
    default: throw Error{LFEM_EINVAL, "no matrix selected"};
    }
}

}  // namespace

void fill_zero(double *x, int64_t n, hipStream_t s)
{
    if (n > 0) k_fill_zero<<<grid_for(n, 256), 256, 0, s>>>(x, n);
    LFEM_HIP(hipGetLastError());
}

void launch_numeric(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    const Outs o = arrange(no);
    switch (m.etype) {
    case S1P1: run_type<ET<1, 1, 1>>(m, p, o, variant, s); break;
    case S1P2: run_type<ET<1, 1, 2>>(m, p, o, variant, s); break;
    case S2P1: run_type<ET<1, 2, 1>>(m, p, o, variant, s); break;
    case S2P2: run_type<ET<1, 2, 2>>(m, p, o, variant, s); break;
    case B2P1: run_type<ET<0, 2, 1>>(m, p, o, variant, s); break;
    case B2P2: run_type<ET<0, 2, 2>>(m, p, o, variant, s); break;
    case B3P1: run_type<ET<0, 3, 1>>(m, p, o, variant, s); break;
    case B3P2: run_type<ET<0, 3, 2>>(m, p, o, variant, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

}  // namespace lfem
