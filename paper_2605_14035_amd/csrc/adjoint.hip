// Energy J(x) = alpha u^T A(x) v + beta w^T M(x) z and its shape derivative.
//
// Per element and quadrature point, with g_u = sum_a u_a grad_hat phi_a,
// K = G^{-1}, G = J^T J (the quadrature forms of section 3.2.2):
//   alpha w mu g_u^T K g_v + beta w mu w_h z_h
// The derivative of that term with respect to node a, coordinate c follows
// from d mu = mu (grad phi_a)_c and d(G^{-1}) = -G^{-1} dG G^{-1} for the
// move dJ = e_c (grad_hat phi_a)^T:
//   w mu [ alpha ((grad u . grad v) grad phi_a - (grad phi_a . grad u) grad v
//                 - (grad phi_a . grad v) grad u) + beta w_h z_h grad phi_a ]_c
// with grad f = J K g_f.  Writing K_a = K g_a, K_u = K g_u, K_v = K g_v this is
//   w mu J [ (alpha g_u.K_v + beta w_h z_h) K_a - alpha (g_a.K_u) K_v
//            - alpha (g_a.K_v) K_u ].
// Element contributions are staged per (local node, component) and gathered
// per node over its ascending incidence list, so the result is bitwise
// reproducible.
//
// The load vector b_j = sum_E sum_q w_q mu f_h(xi_q) phi_j(xi_q) (the
// right-hand side of the paper's assembly, section 6.1) and the non-linear
// terms of the mean-curvature-flow example (section 6.2),
//   f_1[c][j] = sum_E sum_q w mu alpha^2 (nu_h)_c phi_j,
//   f_2[j]    = sum_E sum_q w mu alpha^2 H_h phi_j,
//   alpha^2 = |grad_Gamma_h nu_h|^2 = sum_c g_c^T K g_c, g_c = sum_a nu_{c,a} grad_hat phi_a
// (the Frobenius norm of the tangential gradient: |J K g|^2 = g^T K g), are
// staged and gathered the same way.
#include <cmath>
#include <mutex>

#include "element.hpp"
#include "lfem_internal.hpp"

namespace lfem {

// Fixed device workspace of the allocation-free shape gradient
// (lfem_shape_grad_noalloc): the staged per-(element, local node) contributions,
// k * n_amb * T doubles, at most kNoAllocScratchDoubles (32 MiB).  Every GPU the
// library runs on holds one copy until the process ends.  In host code the
// array's name is not a device address: kernels receive the per-device
// address that noalloc_scratch() obtains with hipGetSymbolAddress.
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 22;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// the address of `scratch` on the current device, looked up once per device
double *noalloc_scratch(const Mesh &m)
{
    int dev = -1;
    LFEM_HIP(hipGetDevice(&dev));
    LFEM_REQUIRE(dev == m.device, LFEM_EINVAL, "the mesh's device must be the current device");
    LFEM_REQUIRE(dev >= 0 && dev < kMaxDevices, LFEM_EUNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        LFEM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        LFEM_REQUIRE(ptr, LFEM_EHIP, "hipGetSymbolAddress returned no address for the workspace");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[dev];
}

// GRAD = false: per-element energy into out[e]
// GRAD = true:  per (local node a, component c) contributions into out[(a*T + e)*n + c]
template <class E, bool GRAD>
__global__ __launch_bounds__(256) void k_adjoint(
    const double *__restrict__ coords, const int32_t *__restrict__ conn,
    const double *__restrict__ tab, int64_t N, int64_t T, int Q, const double *__restrict__ u,
    const double *__restrict__ v, double alpha, const double *__restrict__ w,
    const double *__restrict__ z, double beta, double *__restrict__ out,
    unsigned long long *__restrict__ degenerate)
{
    // contiguous element ranges per XCD: neighbouring elements share nodes,
    // whose gathers then read their staged values from one L2
    const int64_t e = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    const bool has_a = u && v && alpha != 0.0;
    const bool has_m = w && z && beta != 0.0;
    int32_t nid[E::k];
    double x[E::n][E::k], ue[E::k], ve[E::k], we[E::k], ze[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    gather_coords<E>(nid, coords, N, x);
    double J0[E::n][E::d], H[E::n][E::nh > 0 ? E::nh : 1];
    jacobian_setup<E>(x, J0, H);
#pragma unroll
    for (int a = 0; a < E::k; ++a) {
        ue[a] = has_a ? u[nid[a]] : 0.0;
        ve[a] = has_a ? v[nid[a]] : 0.0;
        we[a] = has_m ? w[nid[a]] : 0.0;
        ze[a] = has_m ? z[nid[a]] : 0.0;
    }
    double energy = 0.0;
    double acc[E::k][E::n];
#pragma unroll
    for (int a = 0; a < E::k; ++a)
#pragma unroll
        for (int c = 0; c < E::n; ++c) acc[a][c] = 0.0;
    int bad = 0;
    for (int q = 0; q < Q; ++q) {
        cdouble *t = const_table(tab) + q * E::stride;
        double J[E::n][E::d];
        jacobian_q<E>(x, J0, H, t, J);
        double K[E::d][E::d], mu;
        geometry<E>(J, K, mu);
        bad += !(mu > 0.0 && mu < INFINITY);
        const double wmu = t[0] * mu;
        double gu[E::d], gv[E::d], wh = 0.0, zh = 0.0;
#pragma unroll
        for (int m = 0; m < E::d; ++m) {
            gu[m] = 0.0;
            gv[m] = 0.0;
        }
#pragma unroll
        for (int a = 0; a < E::k; ++a) {
#pragma unroll
            for (int m = 0; m < E::d; ++m) {
                gu[m] = fma(ue[a], t[E::off_g + a * E::d + m], gu[m]);
                gv[m] = fma(ve[a], t[E::off_g + a * E::d + m], gv[m]);
            }
            wh = fma(we[a], t[E::off_phi + a], wh);
            zh = fma(ze[a], t[E::off_phi + a], zh);
        }
        double Ku[E::d], Kv[E::d];
#pragma unroll
        for (int m = 0; m < E::d; ++m) {
            Ku[m] = 0.0;
            Kv[m] = 0.0;
#pragma unroll
            for (int l = 0; l < E::d; ++l) {
                Ku[m] = fma(K[m][l], gu[l], Ku[m]);
                Kv[m] = fma(K[m][l], gv[l], Kv[m]);
            }
        }
        double uv = 0.0;
#pragma unroll
        for (int m = 0; m < E::d; ++m) uv = fma(gu[m], Kv[m], uv);
        const double wz = wh * zh;
        if constexpr (!GRAD) {
            energy += wmu * (alpha * uv + beta * wz);
        } else {
            const double s0 = alpha * uv + beta * wz;
#pragma unroll
            for (int a = 0; a < E::k; ++a) {
                double Ka[E::d], pu = 0.0, pv = 0.0;
#pragma unroll
                for (int m = 0; m < E::d; ++m) {
                    double s = 0.0;
#pragma unroll
                    for (int l = 0; l < E::d; ++l) s = fma(K[m][l], t[E::off_g + a * E::d + l], s);
                    Ka[m] = s;
                    pu = fma(t[E::off_g + a * E::d + m], Ku[m], pu);
                    pv = fma(t[E::off_g + a * E::d + m], Kv[m], pv);
                }
                double r[E::d];
#pragma unroll
                for (int m = 0; m < E::d; ++m) r[m] = s0 * Ka[m] - alpha * (pu * Kv[m] + pv * Ku[m]);
#pragma unroll
                for (int c = 0; c < E::n; ++c) {
                    double s = 0.0;
#pragma unroll
                    for (int m = 0; m < E::d; ++m) s = fma(J[c][m], r[m], s);
                    acc[a][c] = fma(wmu, s, acc[a][c]);
                }
            }
        }
    }
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
    if constexpr (!GRAD) {
        out[e] = energy;
    } else {
#pragma unroll
        for (int a = 0; a < E::k; ++a)
#pragma unroll
            for (int c = 0; c < E::n; ++c) out[(a * T + e) * E::n + c] = acc[a][c];
    }
}

// per (local node a) load contributions into out[a*T + e]; f NULL: f = 1
template <class E>
__global__ __launch_bounds__(256) void k_load(const double *__restrict__ coords, const int32_t *__restrict__ conn,
                                              const double *__restrict__ tab, int64_t N, int64_t T, int Q,
                                              const double *__restrict__ f, double *__restrict__ out,
                                              unsigned long long *__restrict__ degenerate)
{
    // contiguous element ranges per XCD: neighbouring elements share nodes,
    // whose gathers then read their staged values from one L2
    const int64_t e = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    int32_t nid[E::k];
    double x[E::n][E::k], fe[E::k], acc[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    gather_coords<E>(nid, coords, N, x);
    double J0[E::n][E::d], H[E::n][E::nh > 0 ? E::nh : 1];
    jacobian_setup<E>(x, J0, H);
#pragma unroll
    for (int a = 0; a < E::k; ++a) {
        fe[a] = f ? f[nid[a]] : 1.0;
        acc[a] = 0.0;
    }
    int bad = 0;
    for (int q = 0; q < Q; ++q) {
        cdouble *t = const_table(tab) + q * E::stride;
        double J[E::n][E::d];
        jacobian_q<E>(x, J0, H, t, J);
        double K[E::d][E::d], mu;
        geometry<E>(J, K, mu);  // K unused: only the measure is needed
        bad += !(mu > 0.0 && mu < INFINITY);
        double fh = 0.0;
#pragma unroll
        for (int a = 0; a < E::k; ++a) fh = fma(fe[a], t[E::off_phi + a], fh);
        const double wmf = t[0] * mu * fh;
#pragma unroll
        for (int a = 0; a < E::k; ++a) acc[a] = fma(wmf, t[E::off_phi + a], acc[a]);
    }
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
#pragma unroll
    for (int a = 0; a < E::k; ++a) out[a * T + e] = acc[a];
}

// per (local node a, channel c) non-linear load contributions into
// out[(a*T + e)*(n+1) + c]: channels 0..n-1 the field components, n the
// scalar H (NULL: H = 1)
template <class E>
__global__ __launch_bounds__(256) void k_kll(const double *__restrict__ coords, const int32_t *__restrict__ conn,
                                             const double *__restrict__ tab, int64_t N, int64_t T, int Q,
                                             const double *__restrict__ nu, const double *__restrict__ Hs,
                                             double *__restrict__ out, unsigned long long *__restrict__ degenerate)
{
    constexpr int NC = E::n + 1;
    // contiguous element ranges per XCD: neighbouring elements share nodes,
    // whose gathers then read their staged values from one L2
    const int64_t e = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    int32_t nid[E::k];
    double x[E::n][E::k], ul[NC][E::k], acc[NC][E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = conn[a * T + e];
    gather_coords<E>(nid, coords, N, x);
#pragma unroll
    for (int a = 0; a < E::k; ++a) {
#pragma unroll
        for (int c = 0; c < E::n; ++c) ul[c][a] = nu[c * N + nid[a]];
        ul[E::n][a] = Hs ? Hs[nid[a]] : 1.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c][a] = 0.0;
    }
    double J0[E::n][E::d], H[E::n][E::nh > 0 ? E::nh : 1];
    jacobian_setup<E>(x, J0, H);
    int bad = 0;
    for (int q = 0; q < Q; ++q) {
        cdouble *t = const_table(tab) + q * E::stride;
        double J[E::n][E::d];
        jacobian_q<E>(x, J0, H, t, J);
        double K[E::d][E::d], mu;
        geometry<E>(J, K, mu);
        bad += !(mu > 0.0 && mu < INFINITY);
        double alpha2 = 0.0;
#pragma unroll
        for (int c = 0; c < E::n; ++c) {
            double g[E::d];
#pragma unroll
            for (int m = 0; m < E::d; ++m) {
                g[m] = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) g[m] = fma(ul[c][a], t[E::off_g + a * E::d + m], g[m]);
            }
#pragma unroll
            for (int m = 0; m < E::d; ++m) {
                double kg = 0.0;
#pragma unroll
                for (int l = 0; l < E::d; ++l) kg = fma(K[m][l], g[l], kg);
                alpha2 = fma(g[m], kg, alpha2);
            }
        }
        const double wgt = t[0] * mu * alpha2;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double uh = 0.0;
#pragma unroll
            for (int a = 0; a < E::k; ++a) uh = fma(ul[c][a], t[E::off_phi + a], uh);
            const double wu = wgt * uh;
#pragma unroll
            for (int a = 0; a < E::k; ++a) acc[c][a] = fma(wu, t[E::off_phi + a], acc[c][a]);
        }
    }
    if (bad) atomicAdd(degenerate, static_cast<unsigned long long>(bad));
#pragma unroll
    for (int a = 0; a < E::k; ++a)
#pragma unroll
        for (int c = 0; c < NC; ++c) out[(a * T + e) * NC + c] = acc[c][a];
}

// grad[c*N + r] = sum over incidences (e, a) of node r, in ascending order of
// their codes a*T + e, of stage[(a*T + e)*n + c]
// (one plane per local node, the n channels of a contribution side by side:
// one cache line per incidence, coalesced writes by consecutive elements)
template <int NCH>
__global__ __launch_bounds__(256) void k_gather(int64_t N, int64_t T,
                                                const int32_t *__restrict__ ne_ptr,
                                                const int32_t *__restrict__ ne,
                                                const double *__restrict__ stage,
                                                double *__restrict__ grad)
{
    constexpr int U = 8;  // incidences in flight per thread
    // contiguous node ranges per XCD (the staging kernels map elements the same way)
    const int64_t r = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
    const int32_t b1 = ne_ptr[r + 1];
    for (int32_t s0 = ne_ptr[r]; s0 < b1; s0 += U) {
        const int cnt = min(U, b1 - s0);
        int32_t inc[U];
        double v[U][NCH];
#pragma unroll
        for (int i = 0; i < U; ++i) inc[i] = i < cnt ? ne[s0 + i] : 0;
#pragma unroll
        for (int i = 0; i < U; ++i)
            if (i < cnt) {
                const int64_t at = inc[i];  // a * T + e
#pragma unroll
                for (int c = 0; c < NCH; ++c) v[i][c] = stage[at * NCH + c];
            }
        // added in ascending incidence order, as without the batching
#pragma unroll
        for (int i = 0; i < U; ++i)
            if (i < cnt) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) acc[c] += v[i][c];
            }
    }
    // written once, not read again here: non-temporal stores keep the staged
    // contributions that neighbouring nodes still gather in the caches (the
    // staged reads themselves must stay cached: hinting them is far slower)
#pragma unroll
    for (int c = 0; c < NCH; ++c) __builtin_nontemporal_store(acc[c], &grad[c * N + r]);
}

void gather(int64_t N, int64_t T, int n, const int32_t *ne_ptr, const int32_t *ne, const double *stage,
            double *out, hipStream_t s)
{
    if (N == 0) return;
    const unsigned grid = static_cast<unsigned>((N + 255) / 256);
    switch (n) {
    case 1: k_gather<1><<<grid, 256, 0, s>>>(N, T, ne_ptr, ne, stage, out); break;
    case 2: k_gather<2><<<grid, 256, 0, s>>>(N, T, ne_ptr, ne, stage, out); break;
    case 3: k_gather<3><<<grid, 256, 0, s>>>(N, T, ne_ptr, ne, stage, out); break;
    case 4: k_gather<4><<<grid, 256, 0, s>>>(N, T, ne_ptr, ne, stage, out); break;
    default: throw Error{LFEM_EINVAL, "gather channels"};
    }
    LFEM_HIP(hipGetLastError());
}

constexpr int RED_NT = 256;

// fixed-order reduction: block b sums x[b*chunk .. (b+1)*chunk) with a
// strided per-thread loop and an LDS tree
__global__ __launch_bounds__(RED_NT) void k_reduce_sum(const double *__restrict__ x, int64_t n,
                                                       int64_t chunk, double *__restrict__ out)
{
    __shared__ double s[RED_NT];
    const int t = threadIdx.x;
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t b1 = min(b0 + chunk, n);
    double acc = 0.0;
    for (int64_t i = b0 + t; i < b1; i += RED_NT) acc += x[i];
    s[t] = acc;
    __syncthreads();
    for (int w = RED_NT / 2; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    if (t == 0) out[blockIdx.x] = s[0];
}

inline unsigned grid_for(int64_t n, int nt) { return static_cast<unsigned>((n + nt - 1) / nt); }

template <class E>
void run_adj(Mesh &m, bool grad, const double *u, const double *v, double alpha, const double *w,
             const double *z, double beta, double *out, hipStream_t s)
{
    if (m.T == 0) return;
    if (grad)
        k_adjoint<E, true><<<grid_for(m.T, 256), 256, 0, s>>>(m.coords, m.conn, m.tab, m.N, m.T, m.Q,
                                                              u, v, alpha, w, z, beta, out,
                                                              m.degenerate);
    else
        k_adjoint<E, false><<<grid_for(m.T, 256), 256, 0, s>>>(m.coords, m.conn, m.tab, m.N, m.T, m.Q,
                                                               u, v, alpha, w, z, beta, out,
                                                               m.degenerate);
    LFEM_HIP(hipGetLastError());
}

void dispatch(Mesh &m, bool grad, const double *u, const double *v, double alpha, const double *w,
              const double *z, double beta, double *out, hipStream_t s)
{
    switch (m.etype) {
    case S1P1: run_adj<ET<1, 1, 1>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S1P2: run_adj<ET<1, 1, 2>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S2P1: run_adj<ET<1, 2, 1>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S2P2: run_adj<ET<1, 2, 2>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B2P1: run_adj<ET<0, 2, 1>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B2P2: run_adj<ET<0, 2, 2>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S1P3: run_adj<ET<1, 1, 3>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S1P4: run_adj<ET<1, 1, 4>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S2P3: run_adj<ET<1, 2, 3>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case S2P4: run_adj<ET<1, 2, 4>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B2P3: run_adj<ET<0, 2, 3>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B2P4: run_adj<ET<0, 2, 4>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B3P1: run_adj<ET<0, 3, 1>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B3P2: run_adj<ET<0, 3, 2>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B3P3: run_adj<ET<0, 3, 3>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    case B3P4: run_adj<ET<0, 3, 4>>(m, grad, u, v, alpha, w, z, beta, out, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

template <class E>
void run_load(Mesh &m, const double *f, double *out, hipStream_t s)
{
    if (m.T == 0) return;
    k_load<E><<<grid_for(m.T, 256), 256, 0, s>>>(m.coords, m.conn, m.tab, m.N, m.T, m.Q, f, out, m.degenerate);
    LFEM_HIP(hipGetLastError());
}

void dispatch_load(Mesh &m, const double *f, double *out, hipStream_t s)
{
    switch (m.etype) {
    case S1P1: run_load<ET<1, 1, 1>>(m, f, out, s); break;
    case S1P2: run_load<ET<1, 1, 2>>(m, f, out, s); break;
    case S2P1: run_load<ET<1, 2, 1>>(m, f, out, s); break;
    case S2P2: run_load<ET<1, 2, 2>>(m, f, out, s); break;
    case B2P1: run_load<ET<0, 2, 1>>(m, f, out, s); break;
    case B2P2: run_load<ET<0, 2, 2>>(m, f, out, s); break;
    case S1P3: run_load<ET<1, 1, 3>>(m, f, out, s); break;
    case S1P4: run_load<ET<1, 1, 4>>(m, f, out, s); break;
    case S2P3: run_load<ET<1, 2, 3>>(m, f, out, s); break;
    case S2P4: run_load<ET<1, 2, 4>>(m, f, out, s); break;
    case B2P3: run_load<ET<0, 2, 3>>(m, f, out, s); break;
    case B2P4: run_load<ET<0, 2, 4>>(m, f, out, s); break;
    case B3P1: run_load<ET<0, 3, 1>>(m, f, out, s); break;
    case B3P2: run_load<ET<0, 3, 2>>(m, f, out, s); break;
    case B3P3: run_load<ET<0, 3, 3>>(m, f, out, s); break;
    case B3P4: run_load<ET<0, 3, 4>>(m, f, out, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

template <class E>
void run_kll(Mesh &m, const double *nu, const double *H, double *out, hipStream_t s)
{
    if (m.T == 0) return;
    k_kll<E><<<grid_for(m.T, 256), 256, 0, s>>>(m.coords, m.conn, m.tab, m.N, m.T, m.Q, nu, H, out,
                                                m.degenerate);
    LFEM_HIP(hipGetLastError());
}

void dispatch_kll(Mesh &m, const double *nu, const double *H, double *out, hipStream_t s)
{
    switch (m.etype) {
    case S1P1: run_kll<ET<1, 1, 1>>(m, nu, H, out, s); break;
    case S1P2: run_kll<ET<1, 1, 2>>(m, nu, H, out, s); break;
    case S2P1: run_kll<ET<1, 2, 1>>(m, nu, H, out, s); break;
    case S2P2: run_kll<ET<1, 2, 2>>(m, nu, H, out, s); break;
    case B2P1: run_kll<ET<0, 2, 1>>(m, nu, H, out, s); break;
    case B2P2: run_kll<ET<0, 2, 2>>(m, nu, H, out, s); break;
    case S1P3: run_kll<ET<1, 1, 3>>(m, nu, H, out, s); break;
    case S1P4: run_kll<ET<1, 1, 4>>(m, nu, H, out, s); break;
    case S2P3: run_kll<ET<1, 2, 3>>(m, nu, H, out, s); break;
    case S2P4: run_kll<ET<1, 2, 4>>(m, nu, H, out, s); break;
    case B2P3: run_kll<ET<0, 2, 3>>(m, nu, H, out, s); break;
    case B2P4: run_kll<ET<0, 2, 4>>(m, nu, H, out, s); break;
    case B3P1: run_kll<ET<0, 3, 1>>(m, nu, H, out, s); break;
    case B3P2: run_kll<ET<0, 3, 2>>(m, nu, H, out, s); break;
    case B3P3: run_kll<ET<0, 3, 3>>(m, nu, H, out, s); break;
    case B3P4: run_kll<ET<0, 3, 4>>(m, nu, H, out, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

}  // namespace

double *mesh_scratch(Mesh &m, size_t bytes)
{
    if (m.scratch_bytes < bytes) {
        dev_free(m.scratch);
        m.scratch = nullptr;
        m.scratch_bytes = 0;
        LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&m.scratch), bytes));
        m.scratch_bytes = bytes;
    }
    return m.scratch;
}

void launch_energy(Mesh &m, const double *u, const double *v, double alpha, const double *w,
                   const double *z, double beta, double *J, hipStream_t s)
{
    const int64_t chunk = 4096;
    const int64_t nblk = std::max<int64_t>(1, (m.T + chunk - 1) / chunk);
    double *buf = mesh_scratch(m, static_cast<size_t>(m.T + nblk + 1) * sizeof(double));
    double *part = buf + m.T;
    if (m.T == 0) {
        k_reduce_sum<<<1, RED_NT, 0, s>>>(buf, 0, chunk, J);
        LFEM_HIP(hipGetLastError());
        return;
    }
    dispatch(m, false, u, v, alpha, w, z, beta, buf, s);
    k_reduce_sum<<<static_cast<unsigned>(nblk), RED_NT, 0, s>>>(buf, m.T, chunk, part);
    LFEM_HIP(hipGetLastError());
    k_reduce_sum<<<1, RED_NT, 0, s>>>(part, nblk, nblk, J);
    LFEM_HIP(hipGetLastError());
}

void launch_load(Mesh &m, const double *f, double *b, hipStream_t s)
{
    const size_t cnt = static_cast<size_t>(m.k) * m.T;
    double *stage = mesh_scratch(m, std::max<size_t>(cnt, 1) * sizeof(double));
    dispatch_load(m, f, stage, s);
    gather(m.N, m.T, 1, m.ne_ptr, m.ne, stage, b, s);
}

void launch_kll(Mesh &m, const double *nu, const double *H, double *f, hipStream_t s)
{
    const int nc = m.namb + 1;
    const size_t cnt = static_cast<size_t>(m.k) * nc * m.T;
    double *stage = mesh_scratch(m, std::max<size_t>(cnt, 1) * sizeof(double));
    dispatch_kll(m, nu, H, stage, s);
    gather(m.N, m.T, nc, m.ne_ptr, m.ne, stage, f, s);
}

void launch_shape_grad(Mesh &m, const double *u, const double *v, double alpha,
                       const double *w, const double *z, double beta, double *grad,
                       hipStream_t s)
{
    const size_t cnt = static_cast<size_t>(m.k) * m.namb * m.T;
    double *stage = mesh_scratch(m, std::max<size_t>(cnt, 1) * sizeof(double));
    dispatch(m, true, u, v, alpha, w, z, beta, stage, s);
    gather(m.N, m.T, m.namb, m.ne_ptr, m.ne, stage, grad, s);
}

// The same kernels as launch_shape_grad with the staging in the fixed
// workspace.  Every staged entry the gather reads is written by this call's
// k_adjoint first, so nothing needs clearing; calls that overlap on one GPU
// share the workspace and race.
void launch_shape_grad_noalloc(Mesh &m, const double *u, const double *v, double alpha, const double *w,
                               const double *z, double beta, double *grad, hipStream_t s)
{
    const size_t cnt = static_cast<size_t>(m.k) * m.namb * m.T;
    LFEM_REQUIRE(cnt <= kNoAllocScratchDoubles, LFEM_ERANGE,
                 "mesh too large for the fixed workspace of lfem_shape_grad_noalloc "
                 "(k * n_amb * n_elems must not exceed 4194304)");
    double *stage = noalloc_scratch(m);
    dispatch(m, true, u, v, alpha, w, z, beta, stage, s);
    gather(m.N, m.T, m.namb, m.ne_ptr, m.ne, stage, grad, s);
}

}  // namespace lfem
