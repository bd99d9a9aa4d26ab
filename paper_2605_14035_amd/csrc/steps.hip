// Per-step systems of the two mean-curvature-flow schemes of the paper.
//
// Dziuk's algorithm, timed against DUNE (section 6.3): at the current node
// positions x^n, with M = M(x^n) and A = A(x^n),
//   (M + tau A) x^{n+1} = M x^n.
// The algorithm of section 6.2 (evolving-surface finite elements with
// linearly implicit BDF for the coupled system in u = (nu; H)): at the
// extrapolated positions x~ (the mesh's coordinates) and extrapolated u~,
//   (delta_0 M + tau A) u^n = tau f(x~, u~) - M sum_{j>=1} delta_j u^{n-j},
// f the non-linear terms (f_1; f_2) of that section.
// One call assembles M and A into the fixed pattern (the numeric phase of
// the caller's pattern, scatter variant as tuned), for the second scheme
// also f, then one pass over the rows forms S and the right-hand sides of
// every component.  The linear solves are the caller's.  Nothing here
// allocates once the pattern's and the mesh's lazy structures exist, so a
// whole step can be captured in a HIP graph and replayed as the mesh moves
// in place.
#include <algorithm>

#include "element.hpp"
#include "lfem_internal.hpp"

namespace lfem {

namespace {

// one thread per row: S = cm M + ca A in the row's stored order, and per
// component c < NC: rhs[c N + r] = alpha f[c N + r] + beta sum_j M_rj y[c N + j],
// the sum in column order (y or f may be null: that term is left out)
template <int NC>
__global__ __launch_bounds__(256) void k_step_rows(int64_t n_rows, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ m,
                                                   const double *__restrict__ a, double cm, double ca,
                                                   const double *__restrict__ y, double beta,
                                                   const double *__restrict__ f, double alpha,
                                                   double *__restrict__ s, double *__restrict__ rhs)
{
    const int64_t r = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const int32_t k0 = row_ptr[r], k1 = row_ptr[r + 1];
    if (y) {
        for (int32_t k = k0; k < k1; ++k) {
            const double mv = m[k];
            s[k] = fma(ca, a[k], cm * mv);
            const int64_t j = col[k];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = fma(mv, y[c * n_rows + j], acc[c]);
        }
    } else {
        for (int32_t k = k0; k < k1; ++k) s[k] = fma(ca, a[k], cm * m[k]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        rhs[c * n_rows + r] = f ? fma(alpha, f[c * n_rows + r], beta * acc[c]) : beta * acc[c];
}

void step_rows(int nc, const Mesh &m, const Pattern &p, const double *vm, const double *va, double cm, double ca,
               const double *y, double beta, const double *f, double alpha, double *vs, double *rhs, hipStream_t s)
{
    if (m.N == 0) return;
    const unsigned grid = static_cast<unsigned>((m.N + 255) / 256);
    switch (nc) {
    case 2: k_step_rows<2><<<grid, 256, 0, s>>>(m.N, p.row_ptr, p.col_idx, vm, va, cm, ca, y, beta, f, alpha, vs, rhs); break;
    case 3: k_step_rows<3><<<grid, 256, 0, s>>>(m.N, p.row_ptr, p.col_idx, vm, va, cm, ca, y, beta, f, alpha, vs, rhs); break;
    case 4: k_step_rows<4><<<grid, 256, 0, s>>>(m.N, p.row_ptr, p.col_idx, vm, va, cm, ca, y, beta, f, alpha, vs, rhs); break;
    default: throw Error{LFEM_EUNSUPPORTED, "number of right-hand sides"};
    }
    LFEM_HIP(hipGetLastError());
}

// one thread per row and component block: y[c N + r] = alpha sum_j v_rj x[c N + j]
// for c < NC, the sum in column order (bitwise reproducible)
template <int NC>
__global__ __launch_bounds__(256) void k_spmv(int64_t n_rows, const int32_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col, const double *__restrict__ v,
                                              const double *__restrict__ x, double alpha, double *__restrict__ y)
{
    const int64_t r = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    const int32_t k0 = row_ptr[r], k1 = row_ptr[r + 1];
    for (int32_t k = k0; k < k1; ++k) {
        const double a = v[k];
        const int64_t j = col[k];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = fma(a, x[c * n_rows + j], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c * n_rows + r] = alpha * acc[c];
}

}  // namespace

void launch_spmv(const Pattern &p, const double *vals, const double *x, double alpha, double *y, int nvec,
                 hipStream_t s)
{
    const int64_t n = p.mesh->N;
    if (n == 0) return;
    const unsigned grid = static_cast<unsigned>((n + 255) / 256);
    for (int c0 = 0; c0 < nvec; c0 += 4) {
        const int nc = std::min(4, nvec - c0);
        const double *xc = x + c0 * n;
        double *yc = y + c0 * n;
        switch (nc) {
        case 1: k_spmv<1><<<grid, 256, 0, s>>>(n, p.row_ptr, p.col_idx, vals, xc, alpha, yc); break;
        case 2: k_spmv<2><<<grid, 256, 0, s>>>(n, p.row_ptr, p.col_idx, vals, xc, alpha, yc); break;
        case 3: k_spmv<3><<<grid, 256, 0, s>>>(n, p.row_ptr, p.col_idx, vals, xc, alpha, yc); break;
        default: k_spmv<4><<<grid, 256, 0, s>>>(n, p.row_ptr, p.col_idx, vals, xc, alpha, yc); break;
        }
        LFEM_HIP(hipGetLastError());
    }
}

void launch_dziuk(Mesh &m, Pattern &p, double tau, const double *x, double *vals_m, double *vals_a,
                  double *vals_s, double *rhs, int variant, hipStream_t s)
{
    NumericOut o;
    o.what = LFEM_M | LFEM_A;
    o.vals_m = vals_m;
    o.vals_a = vals_a;
    launch_numeric(m, p, o, variant, s);
    step_rows(m.namb, m, p, vals_m, vals_a, 1.0, tau, x ? x : m.coords, 1.0, nullptr, 0.0, vals_s, rhs, s);
}

void launch_kll_system(Mesh &m, Pattern &p, double tau, double delta0, const double *nu, const double *H,
                       const double *hist, double *vals_m, double *vals_a, double *vals_s, double *f, double *rhs,
                       int variant, hipStream_t s)
{
    NumericOut o;
    o.what = LFEM_M | LFEM_A;
    o.vals_m = vals_m;
    o.vals_a = vals_a;
    launch_numeric(m, p, o, variant, s);
    launch_kll(m, nu, H, f, s);
    step_rows(m.namb + 1, m, p, vals_m, vals_a, delta0, tau, hist, -1.0, f, tau, vals_s, rhs, s);
}

}  // namespace lfem
