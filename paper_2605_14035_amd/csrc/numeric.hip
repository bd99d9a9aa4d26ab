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
#include "lfem_internal.hpp"

namespace lfem {

namespace {

__global__ void k_zero(double *__restrict__ x, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

}  // namespace

void fill_zero(double *x, int64_t n, hipStream_t s)
{
    if (n > 0) k_zero<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(x, n);
    LFEM_HIP(hipGetLastError());
}

void launch_numeric(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    switch (m.etype) {
    case S1P1:
    case S1P2:
    case S1P3:
    case S1P4: numeric_curve(m, p, no, variant, s); break;
    case S2P1:
    case S2P2:
    case S2P3:
    case S2P4: numeric_surface(m, p, no, variant, s); break;
    case B2P1:
    case B2P2:
    case B2P3:
    case B2P4: numeric_planar(m, p, no, variant, s); break;
    case B3P1:
    case B3P2:
    case B3P3:
    case B3P4: numeric_tet(m, p, no, variant, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

}  // namespace lfem
