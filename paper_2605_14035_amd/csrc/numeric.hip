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

// Local matrices of element e.  NM mass-class outputs (slot s uses nodal
// coefficient cm[s] or 1 when null), HA: one stiffness output (coefficient ca
// or 1).  Returns the number of degenerate quadrature points.
template <class E, int NM, bool HA>
__device__ __forceinline__ int element_local(
    int64_t e, const double *__restrict__ coords, const int32_t *__restrict__ conn,
    const double *__restrict__ tab, int64_t N, int64_t T, int Q, const double *__restrict__ cm0,
    const double *__restrict__ cm1, const double *__restrict__ ca, int32_t (&nid)[E::k],
    double (&LM)[NM > 0 ? NM : 1][E::np], double (&LA)[E::np])
{
    double x[E::n][E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
#pragma unroll
    for (int a = 0; a < E::k; ++a)
#pragma unroll
        for (int c = 0; c < E::n; ++c) x[c][a] = coords[c * N + nid[a]];
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
#pragma unroll
        for (int c = 0; c < E::n; ++c)
#pragma unroll
            for (int m = 0; m < E::d; ++m) {
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) acc = fma(x[c][a], t[E::off_g + a * E::d + m], acc);
                J[c][m] = acc;
            }
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
                for (int a = 0; a < E::k; ++a) ch = fma(cmv[s][a], t[1 + a], ch);
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
                for (int a = 0; a < E::k; ++a) ah = fma(cav[a], t[1 + a], ah);
                fa *= ah;
            }
            double h[E::k][E::d];
#pragma unroll
            for (int a = 0; a < E::k; ++a)
#pragma unroll
                for (int m = 0; m < E::d; ++m) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < E::d; ++l) acc = fma(K[m][l], t[E::off_g + a * E::d + l], acc);
                    h[a][m] = acc * fa;
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
    double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
    const int bad = element_local<E, NM, HA>(e, coords, conn, tab, N, T, Q, cm0, cm1, ca, nid, LM, LA);
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
    double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
    const int bad = element_local<E, NM, HA>(e, coords, conn, tab, N, T, Q, cm0, cm1, ca, nid, LM, LA);
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

template <class E, int NM, bool HA, int NT>
__global__ __launch_bounds__(NT) void k_blocked(
    const double *__restrict__ coords, const int32_t *__restrict__ conn,
    const double *__restrict__ tab, int64_t N, int64_t T, int Q, const double *__restrict__ cm0,
    const double *__restrict__ cm1, const double *__restrict__ ca,
    const int32_t *__restrict__ row_ptr, const uint8_t *__restrict__ off8, int kkp,
    const int32_t *__restrict__ brow, const int32_t *__restrict__ beptr,
    const int32_t *__restrict__ belem, const uint8_t *__restrict__ bcol, int nb, int cap,
    double *__restrict__ v0, double *__restrict__ v1, double *__restrict__ v2,
    unsigned long long *__restrict__ degenerate)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    extern __shared__ double lds[];
    int32_t *rp = reinterpret_cast<int32_t *>(lds + NMAT * cap);
    const int tid = threadIdx.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int32_t r0 = brow[blk], r1 = brow[blk + 1];
    const int32_t base = row_ptr[r0];
    const int32_t nloc = row_ptr[r1] - base;
    for (int i = tid; i < nloc; i += NT)
#pragma unroll
        for (int mat = 0; mat < NMAT; ++mat) lds[mat * cap + i] = 0.0;
    for (int i = tid; i <= r1 - r0; i += NT) rp[i] = row_ptr[r0 + i] - base;
    const int32_t e0 = beptr[blk], e1 = beptr[blk + 1];
    int bad = 0;
    for (int32_t c0 = e0; c0 < e1; c0 += NT) {
        const int32_t idx = c0 + tid;
        const bool act = idx < e1;
        int color = -1;
        int64_t e = 0;
        int32_t nid[E::k];
        double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
        if (act) {
            e = belem[idx];
            color = bcol[idx];
            bad += element_local<E, NM, HA>(e, coords, conn, tab, N, T, Q, cm0, cm1, ca, nid, LM, LA);
        }
        const int cfirst = bcol[c0];
        const int clast = bcol[min(c0 + NT, e1) - 1];
        for (int c = cfirst; c <= clast; ++c) {
            __syncthreads();
            if (color == c) {
                const uint8_t *o = off8 + e * kkp;
#pragma unroll
                for (int a = 0; a < E::k; ++a) {
                    if (nid[a] < r0 || nid[a] >= r1) continue;
                    const int32_t rb = rp[nid[a] - r0];
#pragma unroll
                    for (int b = 0; b < E::k; ++b) {
                        const int32_t li = rb + o[a * E::k + b];
#pragma unroll
                        for (int mat = 0; mat < NMAT; ++mat)
                            lds[mat * cap + li] += local_value<E, NM, HA>(mat, a, b, LM, LA);
                    }
                }
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
    const size_t lds = static_cast<size_t>(NMAT) * p.sched.cap * sizeof(double) +
                       static_cast<size_t>(p.sched.max_rows + 1) * sizeof(int32_t);
    LFEM_REQUIRE(lds <= 160 * 1024, LFEM_EUNSUPPORTED, "block schedule exceeds LDS");
    auto kern = k_blocked<E, NM, HA, NT>;
    static thread_local size_t attr_lds = 64 * 1024;
    if (lds > attr_lds) {
        LFEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds)));
        attr_lds = lds;
    }
    kern<<<p.sched.nb, NT, lds, s>>>(m.coords, m.conn, m.tab, m.N, m.T, m.Q, o.cm0, o.cm1, o.ca,
                                     p.row_ptr, p.off8, p.kkp, p.sched.row_begin, p.sched.elem_ptr,
                                     p.sched.elems, p.sched.colors, p.sched.nb, p.sched.cap, o.v[0],
                                     o.v[1], o.v[2], m.degenerate);
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
