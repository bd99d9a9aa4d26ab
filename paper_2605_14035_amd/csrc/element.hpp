// Element traits and per-quadrature-point geometry shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace lfem {

// Compile-time nodal Lagrange basis on the reference simplex, in barycentric
// coordinates l_0 = 1 - sum xi, l_i = xi_i (P1: l_i; P2: corners l_i (2 l_i - 1),
// edges 4 l_i l_j; edge order segment (0,1), triangle (0,1) (1,2) (2,0),
// tetrahedron (0,1) (1,2) (0,2) (0,3) (1,3) (2,3)).  For these elements the
// reference gradient is affine in xi:  grad phi_a(xi) = g0_a + Hess_a xi, so the
// Jacobian of an isoparametric element is J(xi) = J0 + sum_l xi_l H_l.
template <int D, int P>
struct RefBasis {
    static constexpr int k = P == 1 ? D + 1 : (D + 1) * (D + 2) / 2;
    static constexpr int edge(int s, int end)
    {
        constexpr int seg[1][2] = {{0, 1}};
        constexpr int tri[3][2] = {{0, 1}, {1, 2}, {2, 0}};
        constexpr int tet[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
        return D == 1 ? seg[s][end] : (D == 2 ? tri[s][end] : tet[s][end]);
    }
    // d l_i / d xi_m and l_i at xi = 0
    static constexpr double dl(int i, int m) { return i == 0 ? -1.0 : (i - 1 == m ? 1.0 : 0.0); }
    static constexpr double l0(int i) { return i == 0 ? 1.0 : 0.0; }
    // d phi_a / d xi_m at xi = 0
    static constexpr double g0(int a, int m)
    {
        if (P == 1) return dl(a, m);
        if (a <= D) return (4.0 * l0(a) - 1.0) * dl(a, m);
        const int i = edge(a - D - 1, 0), j = edge(a - D - 1, 1);
        return 4.0 * (dl(i, m) * l0(j) + l0(i) * dl(j, m));
    }
    // d^2 phi_a / d xi_l d xi_m (constant)
    static constexpr double hess(int a, int l, int m)
    {
        if (P == 1) return 0.0;
        if (a <= D) return 4.0 * dl(a, l) * dl(a, m);
        const int i = edge(a - D - 1, 0), j = edge(a - D - 1, 1);
        return 4.0 * (dl(i, m) * dl(j, l) + dl(i, l) * dl(j, m));
    }
};

template <int SURF, int D, int P>
struct ET {
    static constexpr bool surf = SURF != 0;
    static constexpr int d = D;
    static constexpr int p = P;
    static constexpr int n = SURF ? D + 1 : D;
    static constexpr int k = D == 1 ? P + 1 : (D == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6);
    static constexpr int np = k * (k + 1) / 2;
    static constexpr int nh = P == 2 ? D * (D + 1) / 2 : 0;  // distinct Hessian slots (l <= m)
    // orders 1 and 2: J(xi) = J0 + sum_l xi_l H_l with compile-time basis
    // coefficients; orders 3 and 4: J(xi) from the tabulated reference
    // gradients at the point
    static constexpr bool affine_j = P <= 2;
    // per-quadrature-point table: [w, xi (d), phi (k), grad phi (k*d), phi_a phi_b (np)]
    static constexpr int off_xi = 1;
    static constexpr int off_phi = 1 + D;
    static constexpr int off_g = 1 + D + k;
    static constexpr int off_pp = 1 + D + k + k * D;
    // reference stiffness tensor: for pair p and the symmetric slots (m <= n) of K,
    // g_am g_bn + g_an g_bm (m < n) or g_am g_bm (m = n), so that
    // g_a^T K g_b = sum_s K_s R_{p,s}
    static constexpr int nsym = D * (D + 1) / 2;
    static constexpr int off_ra = off_pp + np;
    static constexpr int stride = 1 + D + k + k * D + np + np * nsym;
    using B = RefBasis<D, (P <= 2 ? P : 1)>;  // used only when affine_j
};

// Workgroup i runs on XCD i % 8; give each XCD a contiguous range of blocks so
// that neighbouring blocks (which share halo elements and nodes) share an L2.
__device__ __forceinline__ int xcd_block(int bid, int nb)
{
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = bid & 7, local = bid >> 3;
    return xcd * per + min(xcd, rem) + local;
}

// Read-only tables are read through the constant address space: uniform loads
// from it become scalar loads.
using cdouble = const __attribute__((address_space(4))) double;
__device__ __forceinline__ cdouble *const_table(const double *p)
{
    return (cdouble *)(p);
}

template <class E>
__device__ __forceinline__ void gather_coords(const int32_t (&nid)[E::k],
                                              const double *__restrict__ coords, int64_t N,
                                              double (&x)[E::n][E::k])
{
#pragma unroll
    for (int a = 0; a < E::k; ++a)
#pragma unroll
        for (int c = 0; c < E::n; ++c) x[c][a] = coords[c * N + nid[a]];
}

// J0[c][m] = sum_a x_a g0_a;  H[c][h] = sum_a x_a Hess_a for the slots l <= m
// (zero basis coefficients are skipped at compile time after unrolling)
template <class E>
__device__ __forceinline__ void jacobian_setup(const double (&x)[E::n][E::k],
                                               double (&J0)[E::n][E::d],
                                               double (&H)[E::n][E::nh > 0 ? E::nh : 1])
{
    if constexpr (!E::affine_j) return;
#pragma unroll
    for (int c = 0; c < E::n; ++c) {
#pragma unroll
        for (int m = 0; m < E::d; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < E::k; ++a) {
                const double g = E::B::g0(a, m);
                if (g != 0.0) acc = fma(x[c][a], g, acc);
            }
            J0[c][m] = acc;
        }
        int h = 0;
#pragma unroll
        for (int l = 0; l < E::d; ++l)
#pragma unroll
            for (int m = l; m < E::d; ++m) {
                if constexpr (E::nh > 0) {
                    double acc = 0.0;
#pragma unroll
                    for (int a = 0; a < E::k; ++a) {
                        const double g = E::B::hess(a, l, m);
                        if (g != 0.0) acc = fma(x[c][a], g, acc);
                    }
                    H[c][h] = acc;
                }
                ++h;
            }
    }
}

// J(xi) = J0 + sum_l xi_l H_l  (column m of H_l is Hess slot (min(l,m), max(l,m)))
template <class E>
__device__ __forceinline__ void jacobian_at(const double (&J0)[E::n][E::d],
                                            const double (&H)[E::n][E::nh > 0 ? E::nh : 1],
                                            cdouble *xi, double (&J)[E::n][E::d])
{
#pragma unroll
    for (int c = 0; c < E::n; ++c)
#pragma unroll
        for (int m = 0; m < E::d; ++m) {
            double acc = J0[c][m];
            if constexpr (E::nh > 0) {
#pragma unroll
                for (int l = 0; l < E::d; ++l) {
                    const int lo = l < m ? l : m, hi = l < m ? m : l;
                    const int slot = lo * E::d - lo * (lo - 1) / 2 + (hi - lo);
                    acc = fma(xi[l], H[c][slot], acc);
                }
            }
            J[c][m] = acc;
        }
}

// J at quadrature point q whose table row is t: the affine form for orders 1
// and 2, else sum_a x_a (grad_hat phi_a(xi_q))^T from the table
template <class E>
__device__ __forceinline__ void jacobian_q(const double (&x)[E::n][E::k], const double (&J0)[E::n][E::d],
                                           const double (&H)[E::n][E::nh > 0 ? E::nh : 1], cdouble *t,
                                           double (&J)[E::n][E::d])
{
    if constexpr (E::affine_j) {
        jacobian_at<E>(J0, H, t + E::off_xi, J);
    } else {
#pragma unroll
        for (int c = 0; c < E::n; ++c)
#pragma unroll
            for (int m = 0; m < E::d; ++m) {
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a < E::k; ++a) acc = fma(x[c][a], t[E::off_g + a * E::d + m], acc);
                J[c][m] = acc;
            }
    }
}

// K = G^{-1} and the measure from J (n x d).  Every fused multiply-add is
// written out (the library is built without floating-point contraction), so
// the rounding is the same wherever this is inlined.
template <class E>
__device__ __forceinline__ void geometry(const double (&J)[E::n][E::d], double (&K)[E::d][E::d],
                                         double &mu)
{
    if constexpr (E::surf && E::d == 1) {
        // one reciprocal square root gives both: mu = g / sqrt(g), 1/g = (1/sqrt(g))^2
        const double g = fma(J[0][0], J[0][0], J[1][0] * J[1][0]);
        const double rr = rsqrt(g);
        mu = g * rr;
        K[0][0] = rr * rr;
    } else if constexpr (E::surf && E::d == 2) {
        const double nx = fma(J[1][0], J[2][1], -(J[2][0] * J[1][1]));
        const double ny = fma(J[2][0], J[0][1], -(J[0][0] * J[2][1]));
        const double nz = fma(J[0][0], J[1][1], -(J[1][0] * J[0][1]));
        const double det = fma(nx, nx, fma(ny, ny, nz * nz));  // det G = |t1 x t2|^2
        const double rr = rsqrt(det);  // mu = det / sqrt(det), 1/det = rr^2
        mu = det * rr;
        const double g11 = fma(J[0][0], J[0][0], fma(J[1][0], J[1][0], J[2][0] * J[2][0]));
        const double g12 = fma(J[0][0], J[0][1], fma(J[1][0], J[1][1], J[2][0] * J[2][1]));
        const double g22 = fma(J[0][1], J[0][1], fma(J[1][1], J[1][1], J[2][1] * J[2][1]));
        const double inv = rr * rr;
        K[0][0] = g22 * inv;
        K[0][1] = -g12 * inv;
        K[1][0] = K[0][1];
        K[1][1] = g11 * inv;
    } else if constexpr (!E::surf && E::d == 2) {
        const double det = fma(J[0][0], J[1][1], -(J[0][1] * J[1][0]));
        mu = fabs(det);
        const double g11 = fma(J[0][0], J[0][0], J[1][0] * J[1][0]);
        const double g12 = fma(J[0][0], J[0][1], J[1][0] * J[1][1]);
        const double g22 = fma(J[0][1], J[0][1], J[1][1] * J[1][1]);
        const double inv = 1.0 / (det * det);
        K[0][0] = g22 * inv;
        K[0][1] = -g12 * inv;
        K[1][0] = K[0][1];
        K[1][1] = g11 * inv;
    } else {
        // cofactors C[r][m] of J; J^{-1} = C^T / det, K = J^{-1} J^{-T} = C^T C / det^2
        double C[3][3];
        C[0][0] = fma(J[1][1], J[2][2], -(J[1][2] * J[2][1]));
        C[0][1] = fma(J[1][2], J[2][0], -(J[1][0] * J[2][2]));
        C[0][2] = fma(J[1][0], J[2][1], -(J[1][1] * J[2][0]));
        C[1][0] = fma(J[0][2], J[2][1], -(J[0][1] * J[2][2]));
        C[1][1] = fma(J[0][0], J[2][2], -(J[0][2] * J[2][0]));
        C[1][2] = fma(J[0][1], J[2][0], -(J[0][0] * J[2][1]));
        C[2][0] = fma(J[0][1], J[1][2], -(J[0][2] * J[1][1]));
        C[2][1] = fma(J[0][2], J[1][0], -(J[0][0] * J[1][2]));
        C[2][2] = fma(J[0][0], J[1][1], -(J[0][1] * J[1][0]));
        const double det = fma(J[0][0], C[0][0], fma(J[0][1], C[0][1], J[0][2] * C[0][2]));
        mu = fabs(det);
        const double inv = 1.0 / (det * det);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                const double v = fma(C[0][a], C[0][b], fma(C[1][a], C[1][b], C[2][a] * C[2][b])) * inv;
                K[a][b] = v;
                K[b][a] = v;
            }
    }
}

}  // namespace lfem
