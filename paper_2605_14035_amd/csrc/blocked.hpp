// Device code of the fused geometry + local-matrix computation and of the
// blocked (LDS row block) scatter, shared by the single-mesh and the batched
// kernels.
#pragma once

#include "element.hpp"
#include "lfem_internal.hpp"

namespace lfem {

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
        cdouble *t = const_table(tab) + q * E::stride;
        double J[E::n][E::d];
        jacobian_q<E>(x, J0, H, t, J);
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

// Local matrices of one element, mass-class outputs formed after the point
// loop: the loop keeps only the stiffness accumulators in registers and
// stores the per-point mass factors f_q = w_q mu_q c_h(xi_q) in this thread's
// LDS column fl[(s * Q + q) * NT]; each mass value is then
// M_ab = sum_q f_q phi_a phi_b (xi_q) from the pair-major table, handed to
// put(p, mat, value) pair by pair with the stiffness value LA[p] (mat = NM).
// Same sums as element_local, with about 2 * NM * np fewer live registers
// through the point loop.
template <class E, int Q, int NM, bool HA, int NT, class Put>
__device__ __forceinline__ int element_local_put(
    const int32_t (&nid)[E::k], const double (&x)[E::n][E::k], const double *__restrict__ tab,
    const double *__restrict__ tabp, const double *__restrict__ cm0, const double *__restrict__ cm1,
    const double *__restrict__ ca, double *fl, Put &&put)
{
    constexpr int PS = Q * (1 + E::nsym);  // pair-major table: Q mass values, then Q * nsym stiffness
    double J0[E::n][E::d], H[E::n][E::nh > 0 ? E::nh : 1];
    jacobian_setup<E>(x, J0, H);
    double LA[E::np];
#pragma unroll
    for (int p = 0; p < E::np; ++p) LA[p] = 0.0;
    const double *cms[2] = {cm0, cm1};
    int bad = 0;
    // one point per iteration, not unrolled: unrolling lets the table loads of
    // every point be hoisted, which costs more registers than it saves
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        cdouble *t = const_table(tab) + q * E::stride;
        double J[E::n][E::d];
        jacobian_q<E>(x, J0, H, t, J);
        double K[E::d][E::d], mu;
        geometry<E>(J, K, mu);
        bad += !(mu > 0.0 && mu < INFINITY);
        const double wmu = t[0] * mu;
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            double fs = wmu;
            if (cms[s]) {
                double ch = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) ch = fma(cms[s][nid[a]], t[E::off_phi + a], ch);
                fs *= ch;
            }
            fl[(s * Q + q) * NT] = fs;
        }
        if constexpr (HA) {
            double fa = wmu;
            if (ca) {
                double ah = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) ah = fma(ca[nid[a]], t[E::off_phi + a], ah);
                fa *= ah;
            }
#pragma unroll
            for (int m = 0; m < E::d; ++m)
#pragma unroll
                for (int l = 0; l < E::d; ++l) K[m][l] *= fa;
            // row a of the pairs: h_a = K g_a, then A_ab += h_a . g_b (only the
            // current h_a is live)
            int p = 0;
#pragma unroll
            for (int a = 0; a < E::k; ++a) {
                double h[E::d];
#pragma unroll
                for (int m = 0; m < E::d; ++m) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < E::d; ++l) acc = fma(K[m][l], t[E::off_g + a * E::d + l], acc);
                    h[m] = acc;
                }
#pragma unroll
                for (int b = a; b < E::k; ++b) {
                    double acc = LA[p];
#pragma unroll
                    for (int m = 0; m < E::d; ++m) acc = fma(h[m], t[E::off_g + b * E::d + m], acc);
                    LA[p] = acc;
                    ++p;
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < E::np; ++p) {
        cdouble *tp = const_table(tabp) + p * PS;
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc = fma(fl[(s * Q + q) * NT], tp[q], acc);
            put(p, s, acc);
        }
        if constexpr (HA) put(p, NM, LA[p]);
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

// Arguments of the blocked scatter for one mesh (device pointers and sizes).
struct BlockArgs {
    const double *coords;
    const double *tab, *tabp;
    int64_t N;
    int Q;
    int etype;
    const double *cm0, *cm1, *ca;
    const int32_t *row_ptr, *brow, *beptr;
    const uint8_t *bcol;
    const int32_t *bconn;
    const uint8_t *boff;
    const uint32_t *bmask;
    const uint32_t *bnode;
    const uint32_t *bord;
    const int32_t *bord_ptr;
    const int32_t *brec;
    int64_t blen;
    int nb, cap, max_side;
    double *v[3];
    unsigned long long *degenerate;
};

inline BlockArgs block_args(const Mesh &m, const Pattern &p, const double *cm0, const double *cm1,
                            const double *ca, double *v0, double *v1, double *v2)
{
    BlockArgs g{};
    g.coords = m.coords;
    g.tab = m.tab;
    g.tabp = m.tabp;
    g.N = m.N;
    g.Q = m.Q;
    g.etype = m.etype;
    g.cm0 = cm0;
    g.cm1 = cm1;
    g.ca = ca;
    g.row_ptr = p.row_ptr;
    g.brow = p.sched.row_begin;
    g.beptr = p.sched.elem_ptr;
    g.bcol = p.sched.colors;
    g.bconn = p.sched.bconn;
    g.boff = p.sched.boff;
    g.bmask = p.sched.bmask;
    g.bnode = p.sched.bnode;
    g.bord = p.sched.bord;
    g.bord_ptr = p.sched.bord_ptr;
    g.brec = p.sched.brec;
    g.blen = p.sched.len;
    g.nb = p.sched.nb;
    g.cap = p.sched.cap;
    g.max_side = p.sched.max_side;
    g.v[0] = v0;
    g.v[1] = v1;
    g.v[2] = v2;
    g.degenerate = m.degenerate;
    return g;
}

// bytes of dynamic LDS the blocked scatter needs for NMAT matrices
inline size_t block_lds_bytes(const Pattern &p, int nmat)
{
    return static_cast<size_t>(nmat) * p.sched.cap * sizeof(double) +
           static_cast<size_t>(p.sched.max_rows + 1) * sizeof(int32_t);
}

// One row block (index blk) of mesh g in colour mode, by a workgroup of NT
// threads with NMAT * g.cap doubles + row offsets of dynamic LDS.
template <class E, int NM, bool HA, int NT>
__device__ __forceinline__ void blocked_block(const BlockArgs &g, const int blk, double *lds)
{
    const double *__restrict__ coords = g.coords;
    const double *__restrict__ tab = g.tab;
    const int64_t N = g.N;
    const int Q = g.Q;
    const double *__restrict__ cm0 = g.cm0;
    const double *__restrict__ cm1 = g.cm1;
    const double *__restrict__ ca = g.ca;
    const int32_t *__restrict__ row_ptr = g.row_ptr;
    const int32_t *__restrict__ brow = g.brow;
    const int32_t *__restrict__ beptr = g.beptr;
    const uint8_t *__restrict__ bcol = g.bcol;
    const int32_t *__restrict__ bconn = g.bconn;
    const uint8_t *__restrict__ boff = g.boff;
    const uint32_t *__restrict__ bmask = g.bmask;
    const int64_t blen = g.blen;
    const int cap = g.cap;
    double *__restrict__ v0 = g.v[0];
    double *__restrict__ v1 = g.v[1];
    double *__restrict__ v2 = g.v[2];
    unsigned long long *__restrict__ degenerate = g.degenerate;
    constexpr int NMAT = NM + (HA ? 1 : 0);
    constexpr int KKP = (E::k * E::k + 3) / 4 * 4;
    constexpr int MW = (E::k * E::k + 31) / 32;
    // LDS: per matrix a region of cap doubles holding the block's values, then
    // the block's row offsets
    int32_t *rp = reinterpret_cast<int32_t *>(lds + NMAT * cap);
    const int tid = threadIdx.x;
    const int32_t e0 = beptr[blk], e1 = beptr[blk + 1];
    const int32_t r0 = brow[blk], r1 = brow[blk + 1];
    // element data of one chunk: colour, node ids, slot offsets, coordinates.
    // The first chunk's loads are issued before the LDS set-up so that the two
    // chains of dependent loads overlap.
    int color = -1;
    int32_t nid[E::k];
    uint32_t ow[KKP / 4];
    uint32_t om[MW];
    double x[E::n][E::k];
    auto load_chunk = [&](int32_t idx) {
        color = -1;
        if (idx < e1) {
            color = bcol[idx];
#pragma unroll
            for (int a = 0; a < E::k; ++a) nid[a] = bconn[a * blen + idx];
            const uint32_t *op = reinterpret_cast<const uint32_t *>(boff + static_cast<int64_t>(idx) * KKP);
#pragma unroll
            for (int w = 0; w < KKP / 4; ++w) ow[w] = op[w];
#pragma unroll
            for (int w = 0; w < MW; ++w) om[w] = bmask[static_cast<int64_t>(idx) * MW + w];
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
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
    __syncthreads();
    double *outs[3] = {v0, v1, v2};
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat)
        for (int i = tid; i < nloc; i += NT) outs[mat][base + i] = lds[mat * cap + i];
}


}  // namespace lfem
