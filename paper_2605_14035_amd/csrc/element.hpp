// Element traits and per-quadrature-point geometry shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace lfem {

template <int SURF, int D, int P>
struct ET {
    static constexpr bool surf = SURF != 0;
    static constexpr int d = D;
    static constexpr int n = SURF ? D + 1 : D;
    static constexpr int k = P == 1 ? D + 1 : (D + 1) * (D + 2) / 2;
    static constexpr int np = k * (k + 1) / 2;
    static constexpr int stride = 1 + k + k * D + np;
    static constexpr int off_g = 1 + k;
    static constexpr int off_pp = 1 + k + k * D;
};

// K = G^{-1} and the measure from J (n x d)
template <class E>
__device__ __forceinline__ void geometry(const double (&J)[E::n][E::d], double (&K)[E::d][E::d],
                                         double &mu)
{
    if constexpr (E::surf && E::d == 1) {
        const double g = J[0][0] * J[0][0] + J[1][0] * J[1][0];
        mu = sqrt(g);
        K[0][0] = 1.0 / g;
    } else if constexpr (E::surf && E::d == 2) {
        const double nx = J[1][0] * J[2][1] - J[2][0] * J[1][1];
        const double ny = J[2][0] * J[0][1] - J[0][0] * J[2][1];
        const double nz = J[0][0] * J[1][1] - J[1][0] * J[0][1];
        const double det = nx * nx + ny * ny + nz * nz;  // det G = |t1 x t2|^2
        mu = sqrt(det);
        const double g11 = J[0][0] * J[0][0] + J[1][0] * J[1][0] + J[2][0] * J[2][0];
        const double g12 = J[0][0] * J[0][1] + J[1][0] * J[1][1] + J[2][0] * J[2][1];
        const double g22 = J[0][1] * J[0][1] + J[1][1] * J[1][1] + J[2][1] * J[2][1];
        const double inv = 1.0 / det;
        K[0][0] = g22 * inv;
        K[0][1] = -g12 * inv;
        K[1][0] = K[0][1];
        K[1][1] = g11 * inv;
    } else if constexpr (!E::surf && E::d == 2) {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        mu = fabs(det);
        const double g11 = J[0][0] * J[0][0] + J[1][0] * J[1][0];
        const double g12 = J[0][0] * J[0][1] + J[1][0] * J[1][1];
        const double g22 = J[0][1] * J[0][1] + J[1][1] * J[1][1];
        const double inv = 1.0 / (det * det);
        K[0][0] = g22 * inv;
        K[0][1] = -g12 * inv;
        K[1][0] = K[0][1];
        K[1][1] = g11 * inv;
    } else {
        // cofactors C[r][m] of J; J^{-1} = C^T / det, K = J^{-1} J^{-T} = C^T C / det^2
        double C[3][3];
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        mu = fabs(det);
        const double inv = 1.0 / (det * det);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                const double v = (C[0][a] * C[0][b] + C[1][a] * C[1][b] + C[2][a] * C[2][b]) * inv;
                K[a][b] = v;
                K[b][a] = v;
            }
    }
}

}  // namespace lfem
