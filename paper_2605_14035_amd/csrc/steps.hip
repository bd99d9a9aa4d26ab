// Per-step system of the linearly implicit mean-curvature-flow scheme that
// the paper times against DUNE (section 6.3, Dziuk's algorithm): at the
// current node positions x^n, with M = M(x^n) and A = A(x^n),
//   (M + tau A) x^{n+1} = M x^n.
// One call assembles M and A into the fixed pattern (the numeric phase of
// the caller's pattern, scatter variant as tuned), then one pass over the
// rows forms S = M + tau A and rhs[c*N + i] = sum_j M_ij x[c*N + j] for
// every coordinate c.  The linear solve is the caller's.  Nothing here
// allocates once the pattern's lazy structures exist, so the whole step can
// be captured in a HIP graph and replayed as the mesh moves in place.
#include "lfem_internal.hpp"

namespace lfem {

namespace {

// one thread per row: S in the row's stored order, rhs summed in column order
__global__ __launch_bounds__(256) void k_dziuk_rows(int64_t n_rows, int nc, const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ m,
                                                    const double *__restrict__ a, double tau,
                                                    const double *__restrict__ x, double *__restrict__ s,
                                                    double *__restrict__ rhs)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
        const double mv = m[k];
        s[k] = fma(tau, a[k], mv);
        const int64_t j = col[k];
        for (int c = 0; c < nc; ++c) acc[c] = fma(mv, x[c * n_rows + j], acc[c]);
    }
    for (int c = 0; c < nc; ++c) rhs[c * n_rows + r] = acc[c];
}

}  // namespace

void launch_dziuk(Mesh &m, Pattern &p, double tau, const double *x, double *vals_m, double *vals_a,
                  double *vals_s, double *rhs, int variant, hipStream_t s)
{
    NumericOut o;
    o.what = LFEM_M | LFEM_A;
    o.vals_m = vals_m;
    o.vals_a = vals_a;
    launch_numeric(m, p, o, variant, s);
    if (m.N > 0) {
        k_dziuk_rows<<<static_cast<unsigned>((m.N + 255) / 256), 256, 0, s>>>(
            m.N, m.namb, p.row_ptr, p.col_idx, vals_m, vals_a, tau, x ? x : m.coords, vals_s, rhs);
        LFEM_HIP(hipGetLastError());
    }
}

}  // namespace lfem
