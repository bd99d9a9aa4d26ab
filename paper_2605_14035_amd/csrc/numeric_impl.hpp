// Kernels and launchers of the numeric phase, instantiated per element family
// by numeric_curve.hip, numeric_surface.hip, numeric_planar.hip and
// numeric_tet.hip.
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
//   staged  - local matrices written element by element, then one thread per
//             CSR slot sums its contribution list in ascending element order
//   blocked - one workgroup owns a contiguous block of rows whose values live
//             in LDS; it recomputes every element touching the block and
//             writes the block once.  Entries with at most two contributions
//             are added in any order (exact); the others in a fixed order:
//             from per-contribution side slots summed in element order
//             (curves, surfaces, planar meshes, where only diagonals have
//             more), or colour by colour (tetrahedra; elements of one colour
//             share no node).
#pragma once

#include <algorithm>
#include <cmath>

#include <map>
#include <tuple>
#include <type_traits>

#include "side.hpp"

namespace lfem {

namespace {

// ---------------------------------------------------------------------------
// atomic variant: one thread per element, values added to the global CSR
// values with FP64 atomics (formed pair by pair, or accumulated point by point
// for tetrahedra)
// ---------------------------------------------------------------------------
// column offset of local pair (a, b) of element e: byte slot map (stride kkp)
// or, for patterns with rows longer than 255 entries, the 16-bit one
template <int K>
__device__ __forceinline__ int32_t pair_slot(const uint8_t *__restrict__ off8, const uint16_t *__restrict__ off16,
                                             int kkp, int64_t e, int a, int b)
{
    return off16 ? static_cast<int32_t>(off16[(e * K + a) * K + b]) : static_cast<int32_t>(off8[e * kkp + a * K + b]);
}

template <class E, int Q, int NM, bool HA>
__global__ __launch_bounds__(256) void k_atomic(const BlockArgs g, int64_t T, const int32_t *__restrict__ conn,
                                                const int32_t *__restrict__ row_ptr,
                                                const uint8_t *__restrict__ off8,
                                                const uint16_t *__restrict__ off16, int kkp)
{
    const int64_t e = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    constexpr int NMAT = NM + (HA ? 1 : 0);
    int32_t nid[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    double x[E::n][E::k];
    gather_coords<E>(nid, g.coords, g.N, x);
    if constexpr (E::d == 3) {
        // tetrahedra: accumulate the local matrices point by point (see k_stage)
        double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
        const int bad = element_local<E, NM, HA>(nid, x, g.tab, Q, g.cm0, g.cm1, g.ca, LM, LA);
        if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
#pragma unroll
        for (int a = 0; a < E::k; ++a) {
            const int32_t rb = row_ptr[nid[a]];
#pragma unroll
            for (int b = 0; b < E::k; ++b)
#pragma unroll
                for (int mat = 0; mat < NMAT; ++mat)
                    unsafeAtomicAdd(g.v[mat] + rb + pair_slot<E::k>(off8, off16, kkp, e, a, b),
                                    local_value<E, NM, HA>(mat, a, b, LM, LA));
        }
        return;
    }
    double f[NM > 0 ? NM : 1][Q];
    double kq[HA ? Q : 1][E::nsym];
    const int bad = side_qdata<E, Q, NM, HA, kCoefRuntime>(nid, x, g.tab, g.cm0, g.cm1, g.ca, f, kq);
    if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
    int p = 0;
#pragma unroll
    for (int a = 0; a < E::k; ++a)
#pragma unroll
        for (int b = a; b < E::k; ++b, ++p) {
            double v[NMAT];
            pair_values<E, Q, NM, HA>(p, f, kq, g.tabp, v);
            const int32_t sa = row_ptr[nid[a]] + pair_slot<E::k>(off8, off16, kkp, e, a, b);
#pragma unroll
            for (int mat = 0; mat < NMAT; ++mat) unsafeAtomicAdd(g.v[mat] + sa, v[mat]);
            if (a != b) {
                const int32_t sb = row_ptr[nid[b]] + pair_slot<E::k>(off8, off16, kkp, e, b, a);
#pragma unroll
                for (int mat = 0; mat < NMAT; ++mat) unsafeAtomicAdd(g.v[mat] + sb, v[mat]);
            }
        }
}

// ---------------------------------------------------------------------------
// staged variant: one thread per element writes its local values, element
// by element, stage[(e * np + p) * NMAT + mat].  The reduction reads, for one
// CSR value, the contributions of the few elements around its row; keeping
// each element's values together lets the values of one row share cache
// lines (about 22 % faster on P2 tetrahedra than one plane per pair).
// ---------------------------------------------------------------------------
// pair table staged in LDS for orders 3 and 4 (tens of KB: more than the
// scalar cache holds, so scalar loads would go to L2 for every pair)
template <class E>
constexpr bool stage_tab_lds() { return E::d <= 2 && E::p >= 3; }

// tetrahedra under rules of up to 11 points: the per-point mass factors of
// each thread (NM * Q doubles)
template <class E, int Q, int NM>
constexpr size_t stage_lds_bytes()
{
    return stage_tab_lds<E>() ? size_t(E::np) * Q * (1 + E::nsym) * sizeof(double)
                              : (E::d == 3 && Q <= 11 ? size_t(NM > 0 ? NM : 1) * Q * 256 * sizeof(double) : 0);
}

// vertex v if row-major pair p is the diagonal pair (v, v) of a vertex, else -1
template <class E>
__host__ __device__ constexpr int vertex_of_diag_pair(int p)
{
    for (int v = 0; v <= E::d; ++v)
        if (p == pair_index<E::k>(v, v)) return v;
    return -1;
}

template <class E, int Q, int NM, bool HA>
__device__ __forceinline__ void stage_body(const BlockArgs &g, int64_t T, const int32_t *__restrict__ conn,
                                           double *__restrict__ stage, double *__restrict__ dstage)
{
    // contiguous element ranges per XCD: neighbouring elements share nodes,
    // whose coordinates then come from one L2
    const int64_t e = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    constexpr bool TAB_LDS = stage_tab_lds<E>();
    const double *tabp = g.tabp;
    if constexpr (TAB_LDS) {
        extern __shared__ double tab_lds[];
        constexpr int n = E::np * Q * (1 + E::nsym);
        for (int i = threadIdx.x; i < n; i += blockDim.x) tab_lds[i] = g.tabp[i];
        __syncthreads();
        tabp = tab_lds;
    }
    if (e >= T) return;  // after the only barrier
    constexpr int NMAT = NM + (HA ? 1 : 0);
    int32_t nid[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    double x[E::n][E::k];
    gather_coords<E>(nid, g.coords, g.N, x);
    if constexpr (E::d == 3) {
        // tetrahedra: the per-point data (7 doubles a point: 77 for 11 points,
        // 245 for 35) outweighs the local stiffness matrix, so that one is
        // accumulated point by point; the mass values are formed after the
        // point loop from the Q per-point factors, which keeps their 55
        // accumulators out of the loop's registers
        double *out = stage + e * E::np * NMAT;
        if constexpr (Q <= 11) {
            extern __shared__ double fl_lds[];
            const int bad = element_local_put<E, Q, NM, HA, 256>(
                nid, x, g.tab, g.tabp, g.cm0, g.cm1, g.ca, fl_lds + threadIdx.x, [&](int p, int mat, double v) {
                    out[p * NMAT + mat] = v;
                    const int vd = vertex_of_diag_pair<E>(p);
                    if (vd >= 0) dstage[(vd * T + e) * NMAT + mat] = v;
                });
            if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
        } else {
            // many points: one LDS read per point and pair would dominate, and
            // the kernel takes one wave per SIMD either way
            double LM[NM > 0 ? NM : 1][E::np], LA[E::np];
            const int bad = element_local<E, NM, HA>(nid, x, g.tab, Q, g.cm0, g.cm1, g.ca, LM, LA);
            if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
#pragma unroll
            for (int p = 0; p < E::np; ++p)
#pragma unroll
                for (int mat = 0; mat < NMAT; ++mat) {
                    const double v = mat < NM ? LM[mat][p] : LA[p];
                    out[p * NMAT + mat] = v;
                    const int vd = vertex_of_diag_pair<E>(p);
                    if (vd >= 0) dstage[(vd * T + e) * NMAT + mat] = v;
                }
        }
    } else {
        double f[NM > 0 ? NM : 1][Q];
        double kq[HA ? Q : 1][E::nsym];
        const int bad = side_qdata<E, Q, NM, HA, kCoefRuntime>(nid, x, g.tab, g.cm0, g.cm1, g.ca, f, kq);
        if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
#pragma unroll
        for (int p = 0; p < E::np; ++p) {
            double v[NMAT];
            pair_values<E, Q, NM, HA, TAB_LDS>(p, f, kq, tabp, v);
#pragma unroll
            for (int mat = 0; mat < NMAT; ++mat) {
                stage[(e * E::np + p) * NMAT + mat] = v[mat];
                const int vd = vertex_of_diag_pair<E>(p);
                if (vd >= 0) dstage[(vd * T + e) * NMAT + mat] = v[mat];
            }
        }
    }
}

template <class E, int Q, int NM, bool HA>
__global__ __launch_bounds__(256) void k_stage(const BlockArgs g, int64_t T, const int32_t *__restrict__ conn,
                                               double *__restrict__ stage, double *__restrict__ dstage)
{
    stage_body<E, Q, NM, HA>(g, T, conn, stage, dstage);
}

// the same for P2 tetrahedra under rules of up to 11 points, held to at most
// 256 registers, two waves per SIMD (the unbounded kernel takes 266 and runs
// one wave per SIMD; with the bound a few registers spill): 876 -> 781 us on
// the 64^3 Kuhn cube, M and A_a
template <class E, int Q, int NM, bool HA>
__global__ __launch_bounds__(256, 2) void k_stage2(const BlockArgs g, int64_t T, const int32_t *__restrict__ conn,
                                                   double *__restrict__ stage, double *__restrict__ dstage)
{
    stage_body<E, Q, NM, HA>(g, T, conn, stage, dstage);
}

// Orders 3 and 4 on tetrahedra: 20 and 35 nodes, 210 and 630 local pairs,
// more than one thread's registers hold.  One wave per element, four waves
// (four elements) per workgroup sharing the reference table in LDS.  Lanes
// q < Q evaluate the geometry of point q (Jacobian from the tabulated
// reference gradients, measure, inverse metric) into LDS; then the local
// matrices are two dense contractions per element on the matrix cores
// (FP64 MFMA, 16 x 16 output tiles, 4 inner terms per instruction):
//   A_ab = sum_{(q,m)} H_{(q,m),a} G_{(q,m),b},  H_{(q,m),a} = (K'_q g_a(xi_q))_m,
//          G_{(q,m),b} = (g_b(xi_q))_m,
//   M_ab = sum_q (f_q phi_a(xi_q)) phi_b(xi_q),
// f_q = w_q mu_q c_h(xi_q), K'_q = w_q mu_q a_h(xi_q) K_q, g the reference
// gradients.  Only the tiles on and above the diagonal are formed (the
// matrices are symmetric); the values of the pairs a <= b are staged element
// by element for the staged reduction, or with ATOMIC added to the CSR values.
typedef double lfem_v4d __attribute__((ext_vector_type(4)));

constexpr int kWaveElems = 4;  // elements (waves) per workgroup

template <class E, int Q, int NM, bool HA, bool ATOMIC>
__global__ __launch_bounds__(64 * kWaveElems) void k_wave(const BlockArgs g, int64_t T,
                                                          const int32_t *__restrict__ conn,
                                                          double *__restrict__ stage,
                                                          const int32_t *__restrict__ row_ptr,
                                                          const uint16_t *__restrict__ off16)
{
    constexpr int K = E::k, D = E::d, NA = E::n, NP = E::np, NMAT = NM + (HA ? 1 : 0);
    constexpr int RS = 1 + K + K * D;            // per point: weight, phi (K), grad phi (K x D)
    constexpr int NMS = NM > 0 ? NM : 1;
    constexpr int QS = NMS + 6;                  // per point: mass factors, then w mu a_h K (m <= l)
    constexpr int NTL = (K + 15) / 16;           // 16 x 16 tiles per side
    constexpr int SA = (D * Q + 3) / 4;          // inner steps of the stiffness contraction
    constexpr int SM = (Q + 3) / 4;              // inner steps of the mass contraction
    constexpr int W = kWaveElems;
    static_assert(D == 3 && NA == 3 && Q <= 64, "one lane per point of a tetrahedral rule");
    __shared__ double ref[Q * RS];
    __shared__ double xs[2][W][K * NA];  // node coordinates, double-buffered across elements
    __shared__ double qd[W][Q * QS];
    __shared__ int32_t nid[2][W][K];
    static_assert(K * NA <= 128, "two coordinates per lane");
    const int wave = static_cast<int>(threadIdx.x) >> 6, lane = static_cast<int>(threadIdx.x) & 63;
    for (int i = threadIdx.x; i < Q * RS; i += 64 * W) {
        const int q = i / RS, j = i - q * RS;
        const int src = j == 0 ? 0 : (j <= K ? E::off_phi + (j - 1) : E::off_g + (j - 1 - K));
        ref[i] = g.tab[q * E::stride + src];
    }
    const double *cms[2] = {g.cm0, g.cm1};
    // the same trip count in every wave, so the barriers below are uniform
    const int64_t per = static_cast<int64_t>(gridDim.x) * W;
    const int64_t iters = (T + per - 1) / per;
    const int li = lane & 15, lk = lane >> 4;  // MFMA operand row / inner index of this lane
    // the first element's node ids and coordinates; later elements' are loaded
    // while the previous one computes (ids during its geometry, coordinates
    // during its contractions)
    {
        const int64_t e0 = static_cast<int64_t>(blockIdx.x) * W + wave;
        if (e0 < T && lane < K) nid[0][wave][lane] = conn[lane * T + e0];
        __syncthreads();
        if (e0 < T)
            for (int i = lane; i < K * NA; i += 64) {
                const int a = i / NA, c = i - a * NA;
                xs[0][wave][i] = g.coords[c * g.N + nid[0][wave][a]];
            }
        __syncthreads();
    }
    // workgroups in launch order (an XCD-aware mapping leaves whole XCDs idle
    // in a partial last round)
    const int64_t gb = blockIdx.x;
    for (int64_t it = 0; it < iters; ++it) {
        const int cb = static_cast<int>(it & 1), nb = cb ^ 1;
        const int64_t e = (it * gridDim.x + gb) * W + wave;
        const bool active = e < T;
        const int64_t en = ((it + 1) * gridDim.x + gb) * W + wave;
        const bool nact = it + 1 < iters && en < T;
        int32_t nid_next = 0;
        if (nact && lane < K) nid_next = conn[lane * T + en];
        if (active && lane < Q) {
            const double *r = ref + lane * RS;
            double J[NA][D];
#pragma unroll
            for (int c = 0; c < NA; ++c)
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    double acc = 0.0;
                    for (int a = 0; a < K; ++a) acc = fma(xs[cb][wave][a * NA + c], r[1 + K + a * D + m], acc);
                    J[c][m] = acc;
                }
            double Km[D][D], mu;
            geometry<E>(J, Km, mu);
            if (!(mu > 0.0 && mu < INFINITY)) atomicAdd(g.degenerate, 1ull);
            const double wmu = r[0] * mu;
            double *qq = qd[wave] + lane * QS;
#pragma unroll
            for (int s = 0; s < NM; ++s) {
                double f = wmu;
                if (cms[s]) {
                    double ch = 0.0;
                    for (int a = 0; a < K; ++a) ch = fma(cms[s][nid[cb][wave][a]], r[1 + a], ch);
                    f *= ch;
                }
                qq[s] = f;
            }
            if constexpr (HA) {
                double fa = wmu;
                if (g.ca) {
                    double ah = 0.0;
                    for (int a = 0; a < K; ++a) ah = fma(g.ca[nid[cb][wave][a]], r[1 + a], ah);
                    fa *= ah;
                }
                qq[NMS + 0] = fa * Km[0][0];
                qq[NMS + 1] = fa * Km[0][1];
                qq[NMS + 2] = fa * Km[0][2];
                qq[NMS + 3] = fa * Km[1][1];
                qq[NMS + 4] = fa * Km[1][2];
                qq[NMS + 5] = fa * Km[2][2];
            }
        }
        if (nact && lane < K) nid[nb][wave][lane] = nid_next;
        __syncthreads();  // point data and the next element's node ids in place
        double cx[2] = {0.0, 0.0};
        if (nact)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int i = lane + 64 * u;
                if (i < K * NA) {
                    const int a = i / NA, c = i - a * NA;
                    cx[u] = g.coords[c * g.N + nid[nb][wave][a]];
                }
            }
        if (active) {
            lfem_v4d accA[NTL][NTL], accM[NMS][NTL][NTL];
#pragma unroll
            for (int R = 0; R < NTL; ++R)
#pragma unroll
                for (int C = 0; C < NTL; ++C) {
                    accA[R][C] = lfem_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s = 0; s < NMS; ++s) accM[s][R][C] = lfem_v4d{0.0, 0.0, 0.0, 0.0};
                }
            if constexpr (HA) {
                // inner index kk = 4 st + lk = 3 q + m over (point, component)
#pragma unroll 3
                for (int st = 0; st < SA; ++st) {
                    const int kk = 4 * st + lk;
                    const bool kin = kk < D * Q;
                    const int q = kin ? kk / D : 0, m = kin ? kk - D * (kk / D) : 0;
                    const double *r = ref + q * RS;
                    const double *qq = qd[wave] + q * QS + NMS;
                    // row m of the symmetric K'_q (stored m <= l as 00 01 02 11 12 22)
                    const double k0 = kin ? qq[m == 0 ? 0 : (m == 1 ? 1 : 2)] : 0.0;
                    const double k1 = kin ? qq[m == 0 ? 1 : (m == 1 ? 3 : 4)] : 0.0;
                    const double k2 = kin ? qq[m == 0 ? 2 : (m == 1 ? 4 : 5)] : 0.0;
                    double bop[NTL];
#pragma unroll
                    for (int C = 0; C < NTL; ++C) {
                        const int b = C * 16 + li;
                        bop[C] = kin && b < K ? r[1 + K + b * D + m] : 0.0;
                    }
#pragma unroll
                    for (int R = 0; R < NTL; ++R) {
                        const int a = R * 16 + li;
                        double aop = 0.0;
                        if (kin && a < K) {
                            const double *ga = r + 1 + K + a * D;
                            aop = fma(k0, ga[0], fma(k1, ga[1], k2 * ga[2]));
                        }
#pragma unroll
                        for (int C = R; C < NTL; ++C)
                            accA[R][C] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[C], accA[R][C], 0, 0, 0);
                    }
                }
            }
            if constexpr (NM > 0) {
#pragma unroll 3
                for (int st = 0; st < SM; ++st) {
                    const int q = 4 * st + lk;
                    const bool qin = q < Q;
                    const int qc = qin ? q : 0;  // padding terms read point 0 and multiply by 0
                    const double *r = ref + qc * RS;
                    double bop[NTL];
#pragma unroll
                    for (int C = 0; C < NTL; ++C) {
                        const int b = C * 16 + li;
                        bop[C] = qin && b < K ? r[1 + b] : 0.0;
                    }
#pragma unroll
                    for (int R = 0; R < NTL; ++R) {
                        const int a = R * 16 + li;
                        const double pa = qin && a < K ? r[1 + a] : 0.0;
#pragma unroll
                        for (int s = 0; s < NM; ++s) {
                            const double aop = pa * qd[wave][qc * QS + s];
#pragma unroll
                            for (int C = R; C < NTL; ++C)
                                accM[s][R][C] =
                                    __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[C], accM[s][R][C], 0, 0, 0);
                        }
                    }
                }
            }
            // tile (R, C) element r of this lane: a = 16 R + lk + 4 r, b = 16 C + li
#pragma unroll
            for (int R = 0; R < NTL; ++R)
#pragma unroll
                for (int C = R; C < NTL; ++C)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int a = R * 16 + lk + 4 * rr, b = C * 16 + li;
                        if (a >= K || b >= K || a > b) continue;
                        double v[NMAT];
#pragma unroll
                        for (int s = 0; s < NM; ++s) v[s] = accM[s][R][C][rr];
                        if constexpr (HA) v[NM] = accA[R][C][rr];
                        if constexpr (ATOMIC) {
                            const int32_t sab = row_ptr[nid[cb][wave][a]] + off16[(e * K + a) * K + b];
#pragma unroll
                            for (int mat = 0; mat < NMAT; ++mat) unsafeAtomicAdd(g.v[mat] + sab, v[mat]);
                            if (a != b) {
                                const int32_t sba = row_ptr[nid[cb][wave][b]] + off16[(e * K + b) * K + a];
#pragma unroll
                                for (int mat = 0; mat < NMAT; ++mat) unsafeAtomicAdd(g.v[mat] + sba, v[mat]);
                            }
                        } else {
                            const int p = pair_index<K>(a, b);
#pragma unroll
                            for (int mat = 0; mat < NMAT; ++mat) stage[(e * NP + p) * NMAT + mat] = v[mat];
                        }
                    }
        }
        if (nact)
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (lane + 64 * u < K * NA) xs[nb][wave][lane + 64 * u] = cx[u];
        __syncthreads();  // the next element's coordinates in place; the point data consumed
    }
}

// Orders 3 and 4 on triangles (surfaces and planar meshes: 10 and 15 nodes,
// one 16 x 16 matrix-core tile per element): four elements per wave, one
// lane per (element, point) for the geometry (w mu c_h and w mu a_h K at the
// 16-point rule), then per element the contractions
//   A_ab = sum_{(q,m)} (K'_q g_a(xi_q))_m (g_b(xi_q))_m   (2 Q inner terms),
//   M_ab = sum_q (f_q phi_a(xi_q)) phi_b(xi_q)              (Q inner terms),
// on FP64 MFMA, the four elements' chains interleaved.  The values of the
// pairs a <= b are staged element by element, or with ATOMIC added to the CSR
// values through the slot map.
template <class E, int Q, int NM, bool HA, bool ATOMIC>
__global__ __launch_bounds__(256) void k_wave_tri(const BlockArgs g, int64_t T, const int32_t *__restrict__ conn,
                                                  double *__restrict__ stage, const int32_t *__restrict__ row_ptr,
                                                  const uint8_t *__restrict__ off8,
                                                  const uint16_t *__restrict__ off16, int kkp)
{
    constexpr int K = E::k, D = E::d, NA = E::n, NP = E::np, NMAT = NM + (HA ? 1 : 0);
    constexpr int RS = 1 + K + K * D;  // per point: weight, phi (K), grad phi (K x D)
    constexpr int NMS = NM > 0 ? NM : 1;
    constexpr int QS = NMS + 3;        // per point: mass factors, then w mu a_h K (00 01 11)
    constexpr int SA = (D * Q + 3) / 4, SM = (Q + 3) / 4;
    constexpr int EW = 4;              // elements per wave
    constexpr int W = 4;               // waves per workgroup
    static_assert(D == 2 && K <= 16 && Q <= 16, "one tile and one lane group per element");
    __shared__ double ref[Q * RS];
    __shared__ double xs[W][EW][K * NA];
    __shared__ double qd[W][EW][Q * QS];
    __shared__ int32_t nid[W][EW][K];
    const int wave = static_cast<int>(threadIdx.x) >> 6, lane = static_cast<int>(threadIdx.x) & 63;
    for (int i = threadIdx.x; i < Q * RS; i += 64 * W) {
        const int q = i / RS, j = i - q * RS;
        const int src = j == 0 ? 0 : (j <= K ? E::off_phi + (j - 1) : E::off_g + (j - 1 - K));
        ref[i] = g.tab[q * E::stride + src];
    }
    const double *cms[2] = {g.cm0, g.cm1};
    const int64_t per = static_cast<int64_t>(gridDim.x) * W * EW;
    const int64_t iters = (T + per - 1) / per;  // the same in every wave: uniform barriers
    const int li = lane & 15, lk = lane >> 4;
    const int64_t gb = blockIdx.x;  // launch order: a partial last round keeps every XCD busy
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t e0 = ((it * gridDim.x + gb) * W + wave) * EW;  // this wave's first element
        __syncthreads();  // reference table in place; the previous elements' data consumed
        for (int i = lane; i < EW * K; i += 64) {
            const int j = i / K, a = i - j * K;
            if (e0 + j < T) nid[wave][j][a] = conn[a * T + e0 + j];
        }
        __syncthreads();
        for (int i = lane; i < EW * K * NA; i += 64) {
            const int j = i / (K * NA), r = i - j * (K * NA), a = r / NA, c = r - a * NA;
            if (e0 + j < T) xs[wave][j][r] = g.coords[c * g.N + nid[wave][j][a]];
        }
        __syncthreads();
        {
            const int j = lane >> 4, q = lane & 15;
            if (q < Q && e0 + j < T) {
                const double *r = ref + q * RS;
                double J[NA][D];
#pragma unroll
                for (int c = 0; c < NA; ++c)
#pragma unroll
                    for (int m = 0; m < D; ++m) {
                        double acc = 0.0;
#pragma unroll
                        for (int a = 0; a < K; ++a) acc = fma(xs[wave][j][a * NA + c], r[1 + K + a * D + m], acc);
                        J[c][m] = acc;
                    }
                double Km[D][D], mu;
                geometry<E>(J, Km, mu);
                if (!(mu > 0.0 && mu < INFINITY)) atomicAdd(g.degenerate, 1ull);
                const double wmu = r[0] * mu;
                double *qq = qd[wave][j] + q * QS;
#pragma unroll
                for (int s = 0; s < NM; ++s) {
                    double f = wmu;
                    if (cms[s]) {
                        double ch = 0.0;
#pragma unroll
                        for (int a = 0; a < K; ++a) ch = fma(cms[s][nid[wave][j][a]], r[1 + a], ch);
                        f *= ch;
                    }
                    qq[s] = f;
                }
                if constexpr (HA) {
                    double fa = wmu;
                    if (g.ca) {
                        double ah = 0.0;
#pragma unroll
                        for (int a = 0; a < K; ++a) ah = fma(g.ca[nid[wave][j][a]], r[1 + a], ah);
                        fa *= ah;
                    }
                    qq[NMS + 0] = fa * Km[0][0];
                    qq[NMS + 1] = fa * Km[0][1];
                    qq[NMS + 2] = fa * Km[1][1];
                }
            }
        }
        __syncthreads();
        lfem_v4d accA[EW], accM[NMS][EW];
#pragma unroll
        for (int j = 0; j < EW; ++j) {
            accA[j] = lfem_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < NMS; ++s) accM[s][j] = lfem_v4d{0.0, 0.0, 0.0, 0.0};
        }
        if constexpr (HA) {
            // inner index kk = 4 st + lk = 2 q + m over (point, component)
#pragma unroll
            for (int st = 0; st < SA; ++st) {
                const int kk = 4 * st + lk;
                const bool kin = kk < D * Q;
                const int q = kin ? kk / D : 0, m = kin ? kk - D * (kk / D) : 0;
                const double *r = ref + q * RS;
                const double bop = kin && li < K ? r[1 + K + li * D + m] : 0.0;
                const bool ain = kin && li < K;
                const double ga0 = ain ? r[1 + K + li * D] : 0.0, ga1 = ain ? r[1 + K + li * D + 1] : 0.0;
#pragma unroll
                for (int j = 0; j < EW; ++j) {
                    const double *qq = qd[wave][j] + q * QS + NMS;
                    // row m of the symmetric K'_q
                    const double k0 = qq[m == 0 ? 0 : 1], k1 = qq[m == 0 ? 1 : 2];
                    const double aop = fma(k0, ga0, k1 * ga1);
                    accA[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, accA[j], 0, 0, 0);
                }
            }
        }
        if constexpr (NM > 0) {
#pragma unroll
            for (int st = 0; st < SM; ++st) {
                const int q = 4 * st + lk;
                const int qc = q < Q ? q : 0;  // padding terms multiply by 0
                const double *r = ref + qc * RS;
                const double ph = q < Q && li < K ? r[1 + li] : 0.0;
#pragma unroll
                for (int j = 0; j < EW; ++j)
#pragma unroll
                    for (int s = 0; s < NM; ++s)
                        accM[s][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ph * qd[wave][j][qc * QS + s], ph,
                                                                         accM[s][j], 0, 0, 0);
            }
        }
        // element j, value r of this lane: a = lk + 4 r, b = li
#pragma unroll
        for (int j = 0; j < EW; ++j) {
            const int64_t e = e0 + j;
            if (e >= T) continue;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int a = lk + 4 * rr, b = li;
                if (a >= K || b >= K || a > b) continue;
                double v[NMAT];
#pragma unroll
                for (int s = 0; s < NM; ++s) v[s] = accM[s][j][rr];
                if constexpr (HA) v[NM] = accA[j][rr];
                if constexpr (ATOMIC) {
                    const int32_t sab = row_ptr[nid[wave][j][a]] + pair_slot<K>(off8, off16, kkp, e, a, b);
#pragma unroll
                    for (int mat = 0; mat < NMAT; ++mat) unsafeAtomicAdd(g.v[mat] + sab, v[mat]);
                    if (a != b) {
                        const int32_t sba = row_ptr[nid[wave][j][b]] + pair_slot<K>(off8, off16, kkp, e, b, a);
#pragma unroll
                        for (int mat = 0; mat < NMAT; ++mat) unsafeAtomicAdd(g.v[mat] + sba, v[mat]);
                    }
                } else {
                    const int p = pair_index<K>(a, b);
#pragma unroll
                    for (int mat = 0; mat < NMAT; ++mat) stage[(e * NP + p) * NMAT + mat] = v[mat];
                }
            }
        }
    }
}

// sum of the contributions of CSR value s, in ascending element order, up to
// kReduceBatch loads in flight
template <int K, int NMAT, int NV = 0>
__device__ __forceinline__ void reduce_slot(int64_t s, int32_t c_begin, int32_t c_end,
                                            const int32_t *__restrict__ clist,
                                            const double *__restrict__ stage, double *const (&outs)[3],
                                            const double *__restrict__ dstage = nullptr, int64_t T = 0)
{
    constexpr int NP = K * (K + 1) / 2;
    constexpr int U = kReduceBatch;
    double acc[NMAT];
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat) acc[mat] = 0.0;
    for (int32_t c0 = c_begin; c0 < c_end; c0 += U) {
        const int cnt = min(U, c_end - c0);
        int32_t code[U];
        double v[U][NMAT];
#pragma unroll
        for (int i = 0; i < U; ++i) code[i] = i < cnt ? clist[c0 + i] : 0;
#pragma unroll
        for (int i = 0; i < U; ++i)
            if (i < cnt) {
                const int64_t e = code[i] / (K * K);
                const int ab = code[i] - static_cast<int>(e) * (K * K);
                const int a = ab / K, bb = ab - a * K;
                const int p = pair_index<K>(a, bb);
                if (NV > 0 && a == bb && a < NV) {
#pragma unroll
                    for (int mat = 0; mat < NMAT; ++mat) v[i][mat] = dstage[(a * T + e) * NMAT + mat];
                } else {
#pragma unroll
                    for (int mat = 0; mat < NMAT; ++mat) v[i][mat] = stage[(e * NP + p) * NMAT + mat];
                }
            }
#pragma unroll
        for (int i = 0; i < U; ++i)
            if (i < cnt) {
#pragma unroll
                for (int mat = 0; mat < NMAT; ++mat) acc[mat] += v[i][mat];
            }
    }
    // written once, not read again here: non-temporal (the staged values that
    // neighbouring rows still gather stay in the caches)
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat) __builtin_nontemporal_store(acc[mat], &outs[mat][s]);
}

// one thread per CSR value with at most kReduceBatch contributions (a single
// round of loads); the longer lists are left to k_reduce_long.  The reads are
// at the minimum the method allows (each element's staged record and the
// contribution lists fetched about once, 2.6 GB for the 64^3 cube against
// 2.25 GB), scattered over the staging array; two values per thread with
// their loads interleaved changed nothing.
template <int K, int NMAT>
__global__ __launch_bounds__(256) void k_reduce(int64_t nnz, const int32_t *__restrict__ cptr,
                                                const int32_t *__restrict__ clist,
                                                const double *__restrict__ stage,
                                                double *__restrict__ v0, double *__restrict__ v1,
                                                double *__restrict__ v2)
{
    // contiguous value ranges per XCD: the values of neighbouring rows read the
    // same elements' staged matrices, which then come from one L2 rather than
    // being fetched into several (HBM reads of the c3 reduction 6.7 -> 2.6 GB)
    const int64_t s = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    const int32_t c0 = cptr[s], c1 = cptr[s + 1];
    if (c1 - c0 > kReduceBatch) return;
    double *const outs[3] = {v0, v1, v2};
    reduce_slot<K, NMAT>(s, c0, c1, clist, stage, outs);
}

// one thread per listed CSR value with a long list (same order of summation)
template <int K, int NMAT, int NV>
__global__ __launch_bounds__(256) void k_reduce_long(int64_t nlong, const int32_t *__restrict__ slots,
                                                     const int32_t *__restrict__ cptr,
                                                     const int32_t *__restrict__ clist,
                                                     const double *__restrict__ stage,
                                                     const double *__restrict__ dstage, int64_t T,
                                                     double *__restrict__ v0, double *__restrict__ v1,
                                                     double *__restrict__ v2)
{
    const int64_t i = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (i >= nlong) return;
    const int64_t s = slots[i];
    double *const outs[3] = {v0, v1, v2};
    reduce_slot<K, NMAT, NV>(s, cptr[s], cptr[s + 1], clist, stage, outs, dstage, T);
}

template <class E, int NM, bool HA, int NT>
__global__ __launch_bounds__(NT) void k_blocked(const BlockArgs g)
{
    extern __shared__ double lds[];
    blocked_block<E, NM, HA, NT>(g, xcd_block(blockIdx.x, g.nb), lds);
}

// Persistent side-slot kernel: workgroup w handles the blocks whose launch
// order index is w, w + G, w + 2G, ... (G = gridDim.x, a multiple of 8 when
// smaller than the block count, so every block of one workgroup lies in the
// range of its XCD).  The next block's loads overlap the current block:
//  - EARLY (a compile-time coefficient set and blocks of one chunk, which
//    leaves registers for it): its record and element words are loaded
//    before the current compute, its coordinates right after it;
//  - otherwise its record and element words right after the current compute,
//    its coordinates after the current write-out has been issued.
// Loads complete in order, so waiting for one also waits for every load
// issued before it; the explicit waits below keep the next block's loads out
// of the current block's waits.
template <class E, int Q, int NM, bool HA, int CF, int NT, bool MULTI>
__global__ __launch_bounds__(NT) void k_side(const BlockArgs g, int rs)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    constexpr bool EARLY = CF != kCoefRuntime && !MULTI;
    extern __shared__ double lds[];
    for (int i = threadIdx.x; i < NMAT * rs; i += NT) lds[i] = 0.0;
    __syncthreads();
    int vb = blockIdx.x;
    SideBlock<E> s;
    side_load_rec<E>(g, xcd_block(vb, g.nb), s);
    side_load_first<E>(g, s);
    side_load_coords<E>(g, s);
    for (;;) {
        const int vn = vb + static_cast<int>(gridDim.x);
        const bool more = vn < g.nb;
        SideBlock<E> nxt;
        if constexpr (EARLY) {
            // this block's loads (and the previous write-out) complete here
            __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
            if (more) {
                side_load_rec<E>(g, xcd_block(vn, g.nb), nxt);
                side_load_first<E>(g, nxt);
            }
        }
        const int bad = side_compute<E, Q, NM, HA, CF, NT, MULTI>(g, s, lds, g.cap, rs);
        if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
        if constexpr (EARLY) {
            if (more) side_load_coords<E>(g, nxt);
        } else {
            // this block's ordered-entry records resident before the next loads
            asm volatile("" ::"v"(s.ord0), "v"(s.ord1));
            if (more) {
                side_load_rec<E>(g, xcd_block(vn, g.nb), nxt);
                side_load_first<E>(g, nxt);
            }
        }
        __syncthreads();
        side_reduce<E, NMAT, NT>(g, s, lds, rs);
        __syncthreads();
        side_write<NMAT, NT>(g, s.base, s.nloc, lds, rs);
        if (!more) break;
        if constexpr (!EARLY) side_load_coords<E>(g, nxt);
        __syncthreads();
        s = nxt;
        vb = vn;
    }
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

// the rules of each element dimension as compile-time constants: the two
// defaults (points: segment 2, 3; triangle 3, 6; tetrahedron 4, 11) and the
// high-order ones (segment 5, 6; triangle 16; tetrahedron 35)
template <class E>
constexpr bool high_order_rule(int Q)
{
    return Q > (E::d == 1 ? 3 : (E::d == 2 ? 6 : 11));
}

template <class E, class F>
void with_rule(int Q, F &&fn)
{
    constexpr int QA = E::d == 1 ? 2 : (E::d == 2 ? 3 : 4);
    constexpr int QB = E::d == 1 ? 3 : (E::d == 2 ? 6 : 11);
    if constexpr (E::p <= 2) {  // orders 3 and 4 take only the high-order rules
        if (Q == QA) return fn(std::integral_constant<int, QA>{});
        if (Q == QB) return fn(std::integral_constant<int, QB>{});
    }
    if constexpr (E::d == 1) {
        if (Q == 5) return fn(std::integral_constant<int, 5>{});
        if (Q == 6) return fn(std::integral_constant<int, 6>{});
    }
    if constexpr (E::d == 2) {
        if (Q == 16) return fn(std::integral_constant<int, 16>{});
    }
    if constexpr (E::d == 3) {
        if (Q == 35) return fn(std::integral_constant<int, 35>{});
    }
    throw Error{LFEM_EUNSUPPORTED, "quadrature rule"};
}

void allow_lds(const void *kern, size_t lds);
template <class E, int NM, bool HA, int NT>
void launch_blocked(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s);
template <class E, int NM, bool HA, int NT>
void launch_side(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s);

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
    if constexpr (E::d == 2 && E::p >= 3) {
        // four elements per wave on the matrix cores; staged (also for a
        // blocked request: no block schedule for orders above 2) or atomic
        const BlockArgs g = block_args(m, p, o.cm0, o.cm1, o.ca, o.v[0], o.v[1], o.v[2]);
        const unsigned grid = static_cast<unsigned>(std::min<int64_t>((m.T + 15) / 16, 4096));
        if (variant == LFEM_SCATTER_ATOMIC) {
            for (int mat = 0; mat < NMAT; ++mat)
                k_fill_zero<<<grid_for(p.nnz, 256), 256, 0, s>>>(o.v[mat], p.nnz);
            with_rule<E>(m.Q, [&](auto qc) {
                k_wave_tri<E, decltype(qc)::value, NM, HA, true><<<grid, 256, 0, s>>>(g, m.T, m.conn, nullptr,
                                                                                    p.row_ptr, p.off8, p.off16, p.kkp);
            });
            LFEM_HIP(hipGetLastError());
            return;
        }
        build_staged(m, p, s);
        const size_t need = static_cast<size_t>(NMAT) * E::np * m.T * sizeof(double);
        if (p.stage_bytes < need) {
            dev_free(p.stage);
            p.stage = nullptr;
            p.stage_bytes = 0;
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&p.stage), need));
            p.stage_bytes = need;
        }
        with_rule<E>(m.Q, [&](auto qc) {
            k_wave_tri<E, decltype(qc)::value, NM, HA, false><<<grid, 256, 0, s>>>(g, m.T, m.conn, p.stage,
                                                                                 p.row_ptr, p.off8, p.off16, p.kkp);
        });
        LFEM_HIP(hipGetLastError());
        k_reduce<E::k, NMAT><<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, p.cptr, p.clist, p.stage, o.v[0],
                                                                   o.v[1], o.v[2]);
        LFEM_HIP(hipGetLastError());
        if (p.nlong > 0) {
            k_reduce_long<E::k, NMAT, 0><<<grid_for(p.nlong, 256), 256, 0, s>>>(p.nlong, p.long_slots, p.cptr,
                                                                                p.clist, p.stage, nullptr, 0, o.v[0],
                                                                                o.v[1], o.v[2]);
            LFEM_HIP(hipGetLastError());
        }
        return;
    } else if constexpr (E::d == 3 && E::p >= 3) {
        // one wave per element; staged (also for a blocked request: no block
        // schedule for orders above 2) or atomic
        const BlockArgs g = block_args(m, p, o.cm0, o.cm1, o.ca, o.v[0], o.v[1], o.v[2]);
        const unsigned grid =
            static_cast<unsigned>(std::min<int64_t>((m.T + kWaveElems - 1) / kWaveElems, 4096));
        if (variant == LFEM_SCATTER_ATOMIC) {
            for (int mat = 0; mat < NMAT; ++mat)
                k_fill_zero<<<grid_for(p.nnz, 256), 256, 0, s>>>(o.v[mat], p.nnz);
            with_rule<E>(m.Q, [&](auto qc) {
                k_wave<E, decltype(qc)::value, NM, HA, true><<<grid, 64 * kWaveElems, 0, s>>>(g, m.T, m.conn, nullptr, p.row_ptr,
                                                                                 p.off16);
            });
            LFEM_HIP(hipGetLastError());
            return;
        }
        build_staged(m, p, s);
        const size_t need = static_cast<size_t>(NMAT) * E::np * m.T * sizeof(double);
        if (p.stage_bytes < need) {
            dev_free(p.stage);
            p.stage = nullptr;
            p.stage_bytes = 0;
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&p.stage), need));
            p.stage_bytes = need;
        }
        with_rule<E>(m.Q, [&](auto qc) {
            k_wave<E, decltype(qc)::value, NM, HA, false><<<grid, 64 * kWaveElems, 0, s>>>(g, m.T, m.conn, p.stage, p.row_ptr,
                                                                              p.off16);
        });
        LFEM_HIP(hipGetLastError());
        k_reduce<E::k, NMAT><<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, p.cptr, p.clist, p.stage, o.v[0],
                                                                   o.v[1], o.v[2]);
        LFEM_HIP(hipGetLastError());
        if (p.nlong > 0) {
            k_reduce_long<E::k, NMAT, 0><<<grid_for(p.nlong, 256), 256, 0, s>>>(p.nlong, p.long_slots, p.cptr,
                                                                                p.clist, p.stage, nullptr, 0, o.v[0],
                                                                                o.v[1], o.v[2]);
            LFEM_HIP(hipGetLastError());
        }
        return;
    } else {
    if (variant == LFEM_SCATTER_ATOMIC) {
        for (int mat = 0; mat < NMAT; ++mat)
            k_fill_zero<<<grid_for(p.nnz, 256), 256, 0, s>>>(o.v[mat], p.nnz);
        const BlockArgs g = block_args(m, p, o.cm0, o.cm1, o.ca, o.v[0], o.v[1], o.v[2]);
        with_rule<E>(m.Q, [&](auto qc) {
            k_atomic<E, decltype(qc)::value, NM, HA><<<grid_for(m.T, 256), 256, 0, s>>>(g, m.T, m.conn, p.row_ptr,
                                                                                       p.off8, p.off16, p.kkp);
        });
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
        const size_t dneed = static_cast<size_t>(NMAT) * (E::d + 1) * m.T * sizeof(double);
        if (p.dstage_bytes < dneed) {
            dev_free(p.dstage);
            p.dstage = nullptr;
            p.dstage_bytes = 0;
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&p.dstage), dneed));
            p.dstage_bytes = dneed;
        }
        const BlockArgs g = block_args(m, p, o.cm0, o.cm1, o.ca, o.v[0], o.v[1], o.v[2]);
        with_rule<E>(m.Q, [&](auto qc) {
            constexpr int Q = decltype(qc)::value;
            auto pick = [] {
                if constexpr (E::d == 3 && Q <= 11) return k_stage2<E, Q, NM, HA>;
                else return k_stage<E, Q, NM, HA>;
            };
            auto ks = pick();
            allow_lds(reinterpret_cast<const void *>(ks), stage_lds_bytes<E, Q, NM>());
            ks<<<grid_for(m.T, 256), 256, stage_lds_bytes<E, Q, NM>(), s>>>(g, m.T, m.conn, p.stage, p.dstage);
        });
        LFEM_HIP(hipGetLastError());
        k_reduce<E::k, NMAT><<<grid_for(p.nnz, 256), 256, 0, s>>>(p.nnz, p.cptr, p.clist, p.stage, o.v[0],
                                                                   o.v[1], o.v[2]);
        LFEM_HIP(hipGetLastError());
        if (p.nlong > 0) {
            k_reduce_long<E::k, NMAT, E::d + 1><<<grid_for(p.nlong, 256), 256, 0, s>>>(
                p.nlong, p.long_slots, p.cptr, p.clist, p.stage, p.dstage, m.T, o.v[0], o.v[1], o.v[2]);
            LFEM_HIP(hipGetLastError());
        }
        return;
    }
    // blocked (block schedules exist for orders 1 and 2 only)
    LFEM_REQUIRE(p.sched.nb > 0, LFEM_EUNSUPPORTED, "pattern has no block schedule");
    if constexpr (E::p > 2) {
        throw Error{LFEM_EUNSUPPORTED, "blocked scatter for orders above 2"};
    } else {
        constexpr int NT = kSideThreads;
        const bool side = p.sched.side_mode;
        const size_t lds = side ? side_lds_bytes(NMAT, p.sched.cap, p.max_row) : block_lds_bytes(p, NMAT);
        LFEM_REQUIRE(lds <= 160 * 1024, LFEM_EUNSUPPORTED, "block schedule exceeds LDS");
        if (side) {
            if constexpr (E::d <= 2) return launch_side<E, NM, HA, NT>(m, p, o, lds, s);
            throw Error{LFEM_EUNSUPPORTED, "side-slot schedule for a tetrahedral mesh"};
        }
        return launch_blocked<E, NM, HA, NT>(m, p, o, lds, s);
    }
    }
}

// allow more than 64 KB of dynamic LDS for kern (once per size increase)
void allow_lds(const void *kern, size_t lds)
{
    static thread_local std::map<const void *, size_t> granted;
    size_t &g = granted[kern];
    if (lds > 64 * 1024 && lds > g) {
        LFEM_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        g = lds;
    }
}

// workgroups of kern that are resident on the device at once
int resident_groups(const void *kern, int nt, size_t lds)
{
    static thread_local std::map<std::tuple<const void *, size_t, int>, int> known;
    int dev = 0;
    LFEM_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(kern, lds, dev);
    auto it = known.find(key);
    if (it != known.end()) return it->second;
    int per_cu = 0, cus = 0;
    LFEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds));
    LFEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LFEM_REQUIRE(per_cu > 0, LFEM_EUNSUPPORTED, "block kernel does not fit on a compute unit");
    const int r = per_cu * cus;
    known.emplace(key, r);
    return r;
}

template <class E, int NM, bool HA, int NT>
void launch_blocked(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s)
{
    auto kern = k_blocked<E, NM, HA, NT>;
    allow_lds(reinterpret_cast<const void *>(kern), lds);
    kern<<<p.sched.nb, NT, lds, s>>>(block_args(m, p, o.cm0, o.cm1, o.ca, o.v[0], o.v[1], o.v[2]));
    LFEM_HIP(hipGetLastError());
}

template <class E, int Q, int NM, bool HA, int CF, int NT, bool MULTI>
void launch_side_q(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s)
{
    auto kern = k_side<E, Q, NM, HA, CF, NT, MULTI>;
    const void *kp = reinterpret_cast<const void *>(kern);
    allow_lds(kp, lds);
    int grid = resident_groups(kp, NT, lds);
    if (grid >= p.sched.nb) grid = p.sched.nb;
    else grid &= ~7;  // keep each workgroup on the XCD its block range belongs to
    kern<<<std::max(grid, 1), NT, lds, s>>>(block_args(m, p, o.cm0, o.cm1, o.ca, o.v[0], o.v[1], o.v[2]),
                                            side_region(p.sched.cap, p.max_row));
    LFEM_HIP(hipGetLastError());
}

// the coefficient set of the selected outputs as a compile-time constant:
// bit 0 / 1: mass-class slot 0 / 1 is weighted, bit 2: the stiffness is
template <int NM, bool HA, class F>
void with_coef(const Outs &o, F &&fn)
{
    const int cf = (o.cm0 ? 1 : 0) | (o.cm1 ? 2 : 0) | (o.ca ? 4 : 0);
    auto pick = [&](auto c) {
        constexpr int C = decltype(c)::value;
        constexpr bool ok = (NM >= 1 || !(C & 1)) && (NM == 2 || !(C & 2)) && (NM != 2 || (C & 3) == 2) &&
                            (HA || !(C & 4));
        if constexpr (ok) fn(c);
        else throw Error{LFEM_EINVAL, "coefficient set does not match the selected matrices"};
    };
    switch (cf) {
    case 0: return pick(std::integral_constant<int, 0>{});
    case 1: return pick(std::integral_constant<int, 1>{});
    case 2: return pick(std::integral_constant<int, 2>{});
    case 4: return pick(std::integral_constant<int, 4>{});
    case 5: return pick(std::integral_constant<int, 5>{});
    case 6: return pick(std::integral_constant<int, 6>{});
    default: throw Error{LFEM_EINVAL, "coefficient set does not match the selected matrices"};
    }
}

template <class E, int NM, bool HA, int NT>
void launch_side(Mesh &m, Pattern &p, const Outs &o, size_t lds, hipStream_t s)
{
    // blocks of more than NT elements (P1 meshes) take the chunk loop and
    // decide coefficients at run time, as do the high-order rules; P2 blocks
    // of one chunk under a default rule get a compile-time coefficient set
    const bool multi = E::p == 1 || p.sched.max_elems > NT;
    with_rule<E>(m.Q, [&](auto qc) {
        constexpr int Q = decltype(qc)::value;
        if constexpr (E::p == 1 || high_order_rule<E>(Q)) {
            launch_side_q<E, Q, NM, HA, kCoefRuntime, NT, true>(m, p, o, lds, s);
        } else {
            if (multi) return launch_side_q<E, Q, NM, HA, kCoefRuntime, NT, true>(m, p, o, lds, s);
            with_coef<NM, HA>(o, [&](auto cc) {
                launch_side_q<E, Q, NM, HA, decltype(cc)::value, NT, false>(m, p, o, lds, s);
            });
        }
    });
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

}  // namespace lfem
