/*
 * Plain FP64 CPU oracle for isoparametric P1/P2 finite-element assembly.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code
 * with the GPU library (no headers, tables or helpers in common).
 *
 * It follows the paper's derivation literally, one element and one
 * quadrature point at a time:
 *
 *   reference map       F(xi) = sum_a x_a phi_a(xi)                (eq. F_map)
 *   tangents            t_m = sum_a x_a d_m phi_a(xi_q)            (Listing 1 (c))
 *   L_E                 surface d=2: [t1 t2 t1 x t2]; curve: [t t_perp];
 *                       bulk: DF itself                              (eq. jacobian_inv)
 *   measure             |t1 x t2|, |t|, |det DF|                     (Listing 1 (c),
 *                                                                    eq. basic integral formula)
 *   C_E = L_E^{-1}      explicit adjugate / determinant
 *   grad phi_a          C_E^T [grad_hat phi_a ; 0]                   (section 3.2.1)
 *   M_loc[a][b]         sum_q w_q mu_q c_h phi_a phi_b               (eq. quadrature mass)
 *   A_loc[a][b]         sum_q w_q mu_q a_h grad phi_a . grad phi_b   (eq. quadrature stiffness)
 *   global matrix       sum of local contributions; COO triples in element
 *                       order, stably sorted by (row, col), duplicates summed
 *                       (eqs. M matrix / A matrix; the sparse() step of Listing 1)
 *
 * Readings of the paper used here:
 *  - the printed P2 triangle basis is the hierarchical set, which is not
 *    nodal; the nodal P2 Lagrange basis (corners l(2l-1), edges 4 l_i l_j) is
 *    used, consistent with phi_j(x_i) = delta_ij (section 3.1);
 *  - C_E^T multiplies the reference gradient (the listing's convention):
 *    grad phi = L^{-T} [g; 0];
 *  - the normal column is the unnormalised t1 x t2; it does not change the
 *    tangential gradient, and the measure is |t1 x t2|, never det L;
 *  - the CSR pattern is structural: no entry is dropped for being zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Internal arithmetic type.  The oracle is built with double.  The same
 * source built with -DORACLE_LONG_DOUBLE serves only as a finite-difference
 * reference for the shape-derivative pins: its energy rounds ~2^11 times
 * less, so a central difference with h = 1e-6 is not dominated by round-off. */
#ifdef ORACLE_LONG_DOUBLE
typedef long double real;
#define r_sqrt sqrtl
#define r_fabs fabsl
#else
typedef double real;
#define r_sqrt sqrt
#define r_fabs fabs
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2
#define OR_EDEGENERATE 3

#define KMAX 35
#define DMAX 3

/* ---------------------------------------------------------------------- */
/* reference element: nodal Lagrange basis in barycentric coordinates      */
/* ---------------------------------------------------------------------- */
static const int SEG_E[1][2] = {{0, 1}};
static const int TRI_E[3][2] = {{0, 1}, {1, 2}, {2, 0}};
static const int TET_E[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

static const int TET_F[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

int oracle_nodes_per_element(int d, int p)
{
    if (p == 1) return d + 1;
    if (p == 2) return (d + 1) * (d + 2) / 2;
    if ((p == 3 || p == 4) && d == 1) return p + 1;
    if ((p == 3 || p == 4) && d == 2) return (p + 1) * (p + 2) / 2;
    if ((p == 3 || p == 4) && d == 3) return (p + 1) * (p + 2) * (p + 3) / 6;
    return -1;
}

/* Orders 3 and 4 (the paper notes that its assembly extends to degree 3 and
 * up, section 1; its mesh utility builds orders 2 to 4 in one to three
 * dimensions, section 5.4).  Node a has the multi-index alpha (|alpha| = p)
 * of its barycentric position alpha / p, in the order: vertices; then for each
 * edge (u -> v) of the edge list its p - 1 nodes from u to v (alpha_u = p - i,
 * alpha_v = i, i = 1..p-1); then the nodes inside the faces of a tetrahedron,
 * face by face in the order (0,1,2), (0,1,3), (0,2,3), (1,2,3) (p = 3: its
 * centroid (1,1,1); p = 4: (2,1,1), (1,2,1), (1,1,2) on the face's vertices
 * in that order); then the interior nodes (triangle, p = 3: (1,1,1); p = 4:
 * (2,1,1), (1,2,1), (1,1,2); tetrahedron, p = 4: (1,1,1,1)).  The Lagrange
 * function of node alpha is
 *   phi_alpha = prod_j prod_{m < alpha_j} (p lambda_j - m) / (m + 1),
 * which is 1 at its node and 0 at every other node of the lattice. */
static void node_alpha(int d, int p, int a, int *alpha)
{
    int j, nv = d + 1;
    for (j = 0; j <= d; j++) alpha[j] = 0;
    if (a < nv) {
        alpha[a] = p;
        return;
    }
    a -= nv;
    {
        int ne = (d == 1) ? 1 : (d == 2 ? 3 : 6);
        const int(*E)[2] = (d == 1) ? SEG_E : (d == 2 ? TRI_E : TET_E);
        if (a < ne * (p - 1)) {
            int e = a / (p - 1), i = a % (p - 1) + 1;
            alpha[E[e][0]] = p - i;
            alpha[E[e][1]] = i;
            return;
        }
        a -= ne * (p - 1);
    }
    if (d == 3) {
        int nf = (p == 3) ? 1 : 3; /* nodes inside one face */
        if (a < 4 * nf) {
            const int *F = TET_F[a / nf];
            alpha[F[0]] = alpha[F[1]] = alpha[F[2]] = 1;
            if (p == 4) alpha[F[a % nf]] = 2;
            return;
        }
        /* interior (p == 4) */
        alpha[0] = alpha[1] = alpha[2] = alpha[3] = 1;
        return;
    }
    /* interior (d == 2) */
    alpha[0] = alpha[1] = alpha[2] = 1;
    if (p == 4) alpha[a] = 2;
}

static void basis_lattice(int d, int p, const real *lam, const real (*dlam)[DMAX], real *phi,
                          real *dphi)
{
    int k = oracle_nodes_per_element(d, p), a, j, m, r;
    for (a = 0; a < k; a++) {
        int alpha[DMAX + 1];
        real f[DMAX + 1], df[DMAX + 1], val = 1.0;
        node_alpha(d, p, a, alpha);
        /* factor j and its derivative with respect to lambda_j */
        for (j = 0; j <= d; j++) {
            real fj = 1.0, dfj = 0.0;
            for (r = 0; r < alpha[j]; r++) {
                real t = (p * lam[j] - r) / (r + 1);
                dfj = dfj * t + fj * (real)p / (r + 1);
                fj *= t;
            }
            f[j] = fj;
            df[j] = dfj;
            val *= fj;
        }
        phi[a] = val;
        for (m = 0; m < d; m++) {
            real g = 0.0;
            for (j = 0; j <= d; j++) {
                real others = 1.0;
                for (r = 0; r <= d; r++)
                    if (r != j) others *= f[r];
                g += df[j] * dlam[j][m] * others;
            }
            dphi[a * d + m] = g;
        }
    }
}

/* phi[a], dphi[a*d + m] = d phi_a / d xi_m at reference point xi[0..d-1] */
static int basis_r(int d, int p, const real *xi, real *phi, real *dphi)
{
    real lam[DMAX + 1], dlam[DMAX + 1][DMAX];
    int i, m;
    if (d < 1 || d > 3 || p < 1 || p > 4) return OR_EINVAL;
    lam[0] = 1.0;
    for (m = 0; m < d; m++) {
        lam[0] -= xi[m];
        dlam[0][m] = -1.0;
    }
    for (i = 1; i <= d; i++) {
        lam[i] = xi[i - 1];
        for (m = 0; m < d; m++) dlam[i][m] = (m == i - 1) ? 1.0 : 0.0;
    }
    if (p == 1) {
        for (i = 0; i <= d; i++) {
            phi[i] = lam[i];
            for (m = 0; m < d; m++) dphi[i * d + m] = dlam[i][m];
        }
        return OR_OK;
    }
    if (p > 2) {
        basis_lattice(d, p, lam, (const real(*)[DMAX])dlam, phi, dphi);
        return OR_OK;
    }
    /* p == 2: corners lambda (2 lambda - 1), then edges 4 lambda_i lambda_j */
    for (i = 0; i <= d; i++) {
        phi[i] = lam[i] * (2.0 * lam[i] - 1.0);
        for (m = 0; m < d; m++) dphi[i * d + m] = (4.0 * lam[i] - 1.0) * dlam[i][m];
    }
    {
        int ne = (d == 1) ? 1 : (d == 2 ? 3 : 6);
        const int(*E)[2] = (d == 1) ? SEG_E : (d == 2 ? TRI_E : TET_E);
        int e;
        for (e = 0; e < ne; e++) {
            int a = E[e][0], b = E[e][1], r = d + 1 + e;
            phi[r] = 4.0 * lam[a] * lam[b];
            for (m = 0; m < d; m++)
                dphi[r * d + m] = 4.0 * (dlam[a][m] * lam[b] + lam[a] * dlam[b][m]);
        }
    }
    return OR_OK;
}

int oracle_basis(int d, int p, const double *xi, double *phi, double *dphi)
{
    real x[DMAX], f[KMAX], g[KMAX * DMAX];
    int i, st;
    if (oracle_nodes_per_element(d, p) < 0 || d > 3) return OR_EINVAL;
    for (i = 0; i < d; i++) x[i] = xi[i];
    st = basis_r(d, p, x, f, g);
    for (i = 0; i < oracle_nodes_per_element(d, p); i++) phi[i] = (double)f[i];
    for (i = 0; i < oracle_nodes_per_element(d, p) * d; i++) dphi[i] = (double)g[i];
    return st;
}

/* ---------------------------------------------------------------------- */
/* small dense linear algebra                                              */
/* ---------------------------------------------------------------------- */
/* inverse of an n x n matrix (n = 1, 2, 3) stored row-major; returns det */
static real inverse_small(int n, const real *L, real *C)
{
    real det;
    if (n == 1) {
        det = L[0];
        C[0] = 1.0 / det;
        return det;
    }
    if (n == 2) {
        det = L[0] * L[3] - L[1] * L[2];
        C[0] = L[3] / det;
        C[1] = -L[1] / det;
        C[2] = -L[2] / det;
        C[3] = L[0] / det;
        return det;
    }
    /* 3 x 3: C = adj(L) / det(L), adj = transpose of the cofactor matrix */
    {
        real c00 = L[4] * L[8] - L[5] * L[7];
        real c01 = -(L[3] * L[8] - L[5] * L[6]);
        real c02 = L[3] * L[7] - L[4] * L[6];
        real c10 = -(L[1] * L[8] - L[2] * L[7]);
        real c11 = L[0] * L[8] - L[2] * L[6];
        real c12 = -(L[0] * L[7] - L[1] * L[6]);
        real c20 = L[1] * L[5] - L[2] * L[4];
        real c21 = -(L[0] * L[5] - L[2] * L[3]);
        real c22 = L[0] * L[4] - L[1] * L[3];
        det = L[0] * c00 + L[1] * c01 + L[2] * c02;
        C[0] = c00 / det; C[1] = c10 / det; C[2] = c20 / det;
        C[3] = c01 / det; C[4] = c11 / det; C[5] = c21 / det;
        C[6] = c02 / det; C[7] = c12 / det; C[8] = c22 / det;
        return det;
    }
}

/* ---------------------------------------------------------------------- */
/* per quadrature point geometry, the paper's route                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    int surface; /* 1 surface (n = d + 1), 0 bulk (n = d) */
    int d, p, n, k;
    int Q;
    const double *qp; /* [Q][d] */
    const double *qw; /* [Q] */
} etype;

/* For element e at quadrature point q: phi[k], grad[k][n] (physical / tangential
   gradients) and mu.  Returns 0, or OR_EDEGENERATE when mu is not positive
   and finite. */
static int point_geometry(const etype *t, const real *x /*[k][n]*/, int q, real *phi,
                          real *grad, real *mu_out)
{
    real dphi[KMAX * DMAX];
    real L[9], C[9], tm[DMAX][DMAX]; /* tm[m][c] = tangent m, component c */
    int a, c, m, r, s, n = t->n, d = t->d;
    real mu;
    {
        real xi[DMAX];
        for (m = 0; m < d; m++) xi[m] = t->qp[q * d + m];
        basis_r(d, t->p, xi, phi, dphi);
    }
    for (m = 0; m < d; m++)
        for (c = 0; c < n; c++) {
            real acc = 0.0;
            for (a = 0; a < t->k; a++) acc += x[a * n + c] * dphi[a * d + m];
            tm[m][c] = acc;
        }
    /* L has the tangents as its first d columns (row-major L[row*n + col]) */
    for (c = 0; c < n; c++)
        for (m = 0; m < d; m++) L[c * n + m] = tm[m][c];
    if (t->surface) {
        if (d == 2) { /* third column t1 x t2 */
            real nx = tm[0][1] * tm[1][2] - tm[0][2] * tm[1][1];
            real ny = tm[0][2] * tm[1][0] - tm[0][0] * tm[1][2];
            real nz = tm[0][0] * tm[1][1] - tm[0][1] * tm[1][0];
            L[0 * 3 + 2] = nx;
            L[1 * 3 + 2] = ny;
            L[2 * 3 + 2] = nz;
            mu = r_sqrt(nx * nx + ny * ny + nz * nz);
        } else { /* curve in R^2: second column t_perp */
            L[0 * 2 + 1] = -tm[0][1];
            L[1 * 2 + 1] = tm[0][0];
            mu = r_sqrt(tm[0][0] * tm[0][0] + tm[0][1] * tm[0][1]);
        }
        inverse_small(n, L, C);
    } else {
        mu = r_fabs(inverse_small(n, L, C));
    }
    /* grad phi_a = C^T [g_a ; 0]: component r = sum_s C[s][r] g_ext[s] */
    for (a = 0; a < t->k; a++)
        for (r = 0; r < n; r++) {
            real acc = 0.0;
            for (s = 0; s < d; s++) acc += C[s * n + r] * dphi[a * d + s];
            grad[a * n + r] = acc;
        }
    *mu_out = mu;
    return (mu > 0.0 && isfinite(mu)) ? OR_OK : OR_EDEGENERATE;
}

static int make_type(etype *t, int surface, int d, int p, int Q, const double *qp,
                     const double *qw)
{
    if (d < 1 || d > 3 || p < 1 || p > 4 || Q < 1) return OR_EINVAL;
    if (surface && d == 3) return OR_EINVAL;
    if (!surface && d == 1) return OR_EINVAL;
    t->surface = surface;
    t->d = d;
    t->p = p;
    t->n = surface ? d + 1 : d;
    t->k = oracle_nodes_per_element(d, p);
    t->Q = Q;
    t->qp = qp;
    t->qw = qw;
    return OR_OK;
}

static void gather(const etype *t, int64_t N, const double *coords, int64_t T,
                   const int32_t *conn, int64_t e, real *x)
{
    int a, c;
    for (a = 0; a < t->k; a++) {
        int64_t g = conn[(int64_t)a * T + e];
        for (c = 0; c < t->n; c++) x[a * t->n + c] = coords[(int64_t)c * N + g];
    }
}

/* Test hook, never defined in the oracle proper: a build with
 * -DORACLE_PLANTED_COEF_MISTAKE pairs the nodal coefficient of local node r
 * with the basis function of node r + 1, so that the tests can show that
 * their pins of the coefficient branch catch such a mistake. */
#ifdef ORACLE_PLANTED_COEF_MISTAKE
#define COEF_NODE(r, k) (((r) + 1) % (k))
#else
#define COEF_NODE(r, k) (r)
#endif

/* kind: 0 mass, 1 stiffness.  coef: nodal coefficient interpolated with the
   basis (c_h = sum_r c_r phi_r), or NULL for 1.  out: k*k row-major. */
static int element_matrix(const etype *t, int64_t N, const double *coords, int64_t T,
                          const int32_t *conn, const double *coef, int kind, int64_t e,
                          real *out)
{
    real x[KMAX * DMAX], phi[KMAX], grad[KMAX * DMAX], ce[KMAX];
    int q, a, b, r, k = t->k, n = t->n, status = OR_OK;
    gather(t, N, coords, T, conn, e, x);
    if (coef)
        for (a = 0; a < k; a++) ce[a] = coef[conn[(int64_t)a * T + e]];
    for (a = 0; a < k * k; a++) out[a] = 0;
    for (q = 0; q < t->Q; q++) {
        real mu, f = 1.0, wmu;
        if (point_geometry(t, x, q, phi, grad, &mu)) status = OR_EDEGENERATE;
        if (coef) {
            f = 0.0;
            for (a = 0; a < k; a++) f += ce[COEF_NODE(a, k)] * phi[a];
        }
        wmu = t->qw[q] * mu * f;
        for (a = 0; a < k; a++)
            for (b = 0; b < k; b++) {
                real v;
                if (kind == 0) {
                    v = phi[a] * phi[b];
                } else {
                    v = 0.0;
                    for (r = 0; r < n; r++) v += grad[a * n + r] * grad[b * n + r];
                }
                out[a * k + b] += wmu * v;
            }
    }
    return status;
}

int oracle_element_matrices(int surface, int d, int p, int Q, const double *qp,
                            const double *qw, int64_t N, const double *coords, int64_t T,
                            const int32_t *conn, const double *coef, int kind, int64_t e0,
                            int64_t e1, double *out)
{
    etype t;
    int64_t e;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    if (st) return st;
    for (e = e0; e < e1; e++) {
        real loc[KMAX * KMAX];
        int i;
        if (element_matrix(&t, N, coords, T, conn, coef, kind, e, loc)) bad = 1;
        for (i = 0; i < t.k * t.k; i++) out[(e - e0) * t.k * t.k + i] = (double)loc[i];
    }
    return bad ? OR_EDEGENERATE : OR_OK;
}

/* ---------------------------------------------------------------------- */
/* COO -> CSR: stable sort of (row, col) keys, duplicates summed in order   */
/* ---------------------------------------------------------------------- */
/* Two stable counting sorts (by column, then by row) give the (row, col)
   lexicographic order while keeping element order among equal keys. */
static int coo_to_csr(int64_t N, int64_t m, const int32_t *I, const int32_t *J,
                      const real *V, int64_t *row_ptr, int32_t *col_idx, double *vals,
                      int64_t *nnz_out)
{
    int64_t *cnt = calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *p1 = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int64_t *p2 = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int64_t i, s, nnz = 0;
    if (!cnt || !p1 || !p2) {
        free(cnt); free(p1); free(p2);
        return OR_ENOMEM;
    }
    for (i = 0; i < m; i++) cnt[J[i] + 1]++;
    for (i = 0; i < N; i++) cnt[i + 1] += cnt[i];
    for (i = 0; i < m; i++) p1[cnt[J[i]]++] = i;
    memset(cnt, 0, sizeof(int64_t) * ((size_t)N + 1));
    for (i = 0; i < m; i++) cnt[I[i] + 1]++;
    for (i = 0; i < N; i++) cnt[i + 1] += cnt[i];
    for (i = 0; i < m; i++) {
        int64_t src = p1[i];
        p2[cnt[I[src]]++] = src;
    }
    /* walk the sorted triples, summing runs of equal (row, col) */
    for (i = 0; i <= N; i++) row_ptr[i] = 0;
    for (s = 0; s < m;) {
        int64_t src = p2[s], t = s + 1;
        real acc = V[src];
        while (t < m && I[p2[t]] == I[src] && J[p2[t]] == J[src]) {
            acc += V[p2[t]];
            t++;
        }
        col_idx[nnz] = J[src];
        vals[nnz] = (double)acc;
        row_ptr[I[src] + 1]++;
        nnz++;
        s = t;
    }
    for (i = 0; i < N; i++) row_ptr[i + 1] += row_ptr[i];
    *nnz_out = nnz;
    free(cnt);
    free(p1);
    free(p2);
    return OR_OK;
}

/*
 * Assemble the global matrix.  If row_mask is non-NULL only rows with
 * row_mask[i] != 0 are produced (the other rows come out empty), which lets
 * the tests check single rows of very large meshes.  The caller sizes
 * col_idx / vals for at most k*k*T entries (or the masked subset); pass
 * cap = their capacity.
 */
int oracle_assemble(int surface, int d, int p, int Q, const double *qp, const double *qw,
                    int64_t N, const double *coords, int64_t T, const int32_t *conn,
                    const double *coef, int kind, const uint8_t *row_mask, int64_t cap,
                    int64_t *row_ptr, int32_t *col_idx, double *vals, int64_t *nnz_out)
{
    etype t;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    int64_t e, m = 0, k2;
    int32_t *I, *J;
    real *V, loc[KMAX * KMAX];
    if (st) return st;
    k2 = (int64_t)t.k * t.k;
    /* count the triples to keep */
    for (e = 0; e < T; e++) {
        int a;
        for (a = 0; a < t.k; a++) {
            int32_t g = conn[(int64_t)a * T + e];
            if (g < 0 || g >= N) return OR_EINVAL;
            if (!row_mask || row_mask[g]) m += t.k;
        }
    }
    I = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    J = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    V = malloc(sizeof(real) * (size_t)(m ? m : 1));
    if (!I || !J || !V) {
        free(I); free(J); free(V);
        return OR_ENOMEM;
    }
    m = 0;
    for (e = 0; e < T; e++) {
        int a, b, need = 0;
        for (a = 0; a < t.k; a++)
            if (!row_mask || row_mask[conn[(int64_t)a * T + e]]) need = 1;
        if (!need) continue;
        if (element_matrix(&t, N, coords, T, conn, coef, kind, e, loc)) bad = 1;
        for (a = 0; a < t.k; a++) {
            int32_t gi = conn[(int64_t)a * T + e];
            if (row_mask && !row_mask[gi]) continue;
            for (b = 0; b < t.k; b++) {
                I[m] = gi;
                J[m] = conn[(int64_t)b * T + e];
                V[m] = loc[a * t.k + b];
                m++;
            }
        }
    }
    (void)k2;
    if (m > cap) {
        free(I); free(J); free(V);
        return OR_EINVAL;
    }
    st = coo_to_csr(N, m, I, J, V, row_ptr, col_idx, vals, nnz_out);
    free(I);
    free(J);
    free(V);
    if (st) return st;
    return bad ? OR_EDEGENERATE : OR_OK;
}

/*
 * Numeric phase alone, into a CSR pattern built beforehand (the structural
 * pattern of the same element array, as oracle_assemble returns it): vals is
 * set to zero, then every element's local matrix is added entry by entry in
 * element order, the slot of (i, j) found by binary search in row i.  The sums
 * are those of oracle_assemble (element order per entry).  This is the CPU
 * counterpart of assembling into a precomputed sparsity pattern, which the
 * paper names as the way FEM packages avoid the sort (section 4.2).
 * Returns OR_EINVAL if an element pair is missing from the pattern.
 */
int oracle_assemble_numeric(int surface, int d, int p, int Q, const double *qp,
                            const double *qw, int64_t N, const double *coords, int64_t T,
                            const int32_t *conn, const double *coef, int kind,
                            const int64_t *row_ptr, const int32_t *col_idx, double *vals)
{
    etype t;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    int64_t e, s;
    real loc[KMAX * KMAX];
    if (st) return st;
    for (s = 0; s < row_ptr[N]; s++) vals[s] = 0.0;
    for (e = 0; e < T; e++) {
        int a, b;
        if (element_matrix(&t, N, coords, T, conn, coef, kind, e, loc)) bad = 1;
        for (a = 0; a < t.k; a++) {
            int32_t gi = conn[(int64_t)a * T + e];
            for (b = 0; b < t.k; b++) {
                int32_t gj = conn[(int64_t)b * T + e];
                int64_t lo = row_ptr[gi], hi = row_ptr[gi + 1];
                while (lo < hi) {
                    int64_t mid = lo + (hi - lo) / 2;
                    if (col_idx[mid] < gj)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo >= row_ptr[gi + 1] || col_idx[lo] != gj) return OR_EINVAL;
                vals[lo] = (double)((real)vals[lo] + loc[a * t.k + b]);
            }
        }
    }
    return bad ? OR_EDEGENERATE : OR_OK;
}

/* ---------------------------------------------------------------------- */
/* energy and its shape derivative                                          */
/* ---------------------------------------------------------------------- */
/* J(x) = alpha u^T A(x) v + beta w^T M(x) z, straight from the local matrices. */
int oracle_energy(int surface, int d, int p, int Q, const double *qp, const double *qw,
                  int64_t N, const double *coords, int64_t T, const int32_t *conn,
                  const double *u, const double *v, double alpha, const double *w,
                  const double *z, double beta, double *J_out)
{
    etype t;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    int64_t e;
    real loc[KMAX * KMAX], J = 0.0;
    if (st) return st;
    for (e = 0; e < T; e++) {
        int a, b;
        real ea = 0.0, em = 0.0;
        if (u && v && alpha != 0.0) {
            if (element_matrix(&t, N, coords, T, conn, NULL, 1, e, loc)) bad = 1;
            for (a = 0; a < t.k; a++)
                for (b = 0; b < t.k; b++)
                    ea += u[conn[(int64_t)a * T + e]] * loc[a * t.k + b] *
                          v[conn[(int64_t)b * T + e]];
        }
        if (w && z && beta != 0.0) {
            if (element_matrix(&t, N, coords, T, conn, NULL, 0, e, loc)) bad = 1;
            for (a = 0; a < t.k; a++)
                for (b = 0; b < t.k; b++)
                    em += w[conn[(int64_t)a * T + e]] * loc[a * t.k + b] *
                          z[conn[(int64_t)b * T + e]];
        }
        J += alpha * ea + beta * em;
    }
    *J_out = (double)J;
    return bad ? OR_EDEGENERATE : OR_OK;
}

/*
 * grad[c*N + r] = d J / d x_{r,c}, overwritten.  Closed form, per element and
 * quadrature point, with grad_phi_r the tangential/physical gradient,
 * grad u = sum u_a grad_phi_a, u_h = sum u_a phi_a:
 *   d/dx_r [u^T A v]: w mu [ (grad u . grad v) grad_phi_r
 *                            - (grad_phi_r . grad u) grad v
 *                            - (grad_phi_r . grad v) grad u ]
 *   d/dx_r [w^T M z]: w mu (w_h z_h) grad_phi_r
 * It follows from d mu = mu (grad_phi_r)_c for a move of node r along e_c and
 * from d(G^{-1}) = -G^{-1} dG G^{-1}, G = DF^T DF.
 */
int oracle_shape_grad(int surface, int d, int p, int Q, const double *qp, const double *qw,
                      int64_t N, const double *coords, int64_t T, const int32_t *conn,
                      const double *u, const double *v, double alpha, const double *w,
                      const double *z, double beta, double *grad)
{
    etype t;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    int64_t e;
    if (st) return st;
    memset(grad, 0, sizeof(double) * (size_t)(t.n * N));
    for (e = 0; e < T; e++) {
        real x[KMAX * DMAX], phi[KMAX], gp[KMAX * DMAX];
        real ue[KMAX], ve[KMAX], we[KMAX], ze[KMAX];
        int a, q, c, k = t.k, n = t.n;
        gather(&t, N, coords, T, conn, e, x);
        for (a = 0; a < k; a++) {
            int64_t g = conn[(int64_t)a * T + e];
            ue[a] = u ? u[g] : 0.0;
            ve[a] = v ? v[g] : 0.0;
            we[a] = w ? w[g] : 0.0;
            ze[a] = z ? z[g] : 0.0;
        }
        for (q = 0; q < t.Q; q++) {
            real mu, gu[DMAX] = {0}, gv[DMAX] = {0}, wh = 0.0, zh = 0.0, uv = 0.0;
            if (point_geometry(&t, x, q, phi, gp, &mu)) bad = 1;
            for (a = 0; a < k; a++) {
                for (c = 0; c < n; c++) {
                    gu[c] += ue[a] * gp[a * n + c];
                    gv[c] += ve[a] * gp[a * n + c];
                }
                wh += we[a] * phi[a];
                zh += ze[a] * phi[a];
            }
            for (c = 0; c < n; c++) uv += gu[c] * gv[c];
            for (a = 0; a < k; a++) {
                real pu = 0.0, pv = 0.0;
                int64_t g = conn[(int64_t)a * T + e];
                for (c = 0; c < n; c++) {
                    pu += gp[a * n + c] * gu[c];
                    pv += gp[a * n + c] * gv[c];
                }
                for (c = 0; c < n; c++) {
                    real dA = uv * gp[a * n + c] - pu * gv[c] - pv * gu[c];
                    real dM = wh * zh * gp[a * n + c];
                    grad[(int64_t)c * N + g] += (double)(t.qw[q] * mu * (alpha * dA + beta * dM));
                }
            }
        }
    }
    return bad ? OR_EDEGENERATE : OR_OK;
}

/* ---------------------------------------------------------------------- */
/* load vector                                                              */
/* ---------------------------------------------------------------------- */
/*
 * b[j] = sum_E sum_q w_q mu_E(xi_q) f_h(xi_q) phi_j(xi_q), the right-hand side
 * that the paper's assembly returns beside M and A (section 6.1; summed node
 * by node like the accumarray step of Listing 1).  f_h = sum_r f_r phi_r is
 * the nodal data interpolated with the element basis; f NULL means f = 1.
 * Contributions are added in element order.  b has N entries, overwritten.
 */
int oracle_load(int surface, int d, int p, int Q, const double *qp, const double *qw, int64_t N,
                const double *coords, int64_t T, const int32_t *conn, const double *f, double *b)
{
    etype t;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    int64_t e, i;
    real *acc;
    if (st) return st;
    acc = (real *)calloc((size_t)(N > 0 ? N : 1), sizeof(real));
    if (!acc) return OR_ENOMEM;
    for (e = 0; e < T; e++) {
        real x[KMAX * DMAX], phi[KMAX], gp[KMAX * DMAX], fe[KMAX];
        int a, q;
        gather(&t, N, coords, T, conn, e, x);
        for (a = 0; a < t.k; a++) fe[a] = f ? f[conn[(int64_t)a * T + e]] : 1.0;
        for (q = 0; q < t.Q; q++) {
            real mu, fh = 0.0;
            if (point_geometry(&t, x, q, phi, gp, &mu)) bad = 1;
            for (a = 0; a < t.k; a++) fh += fe[a] * phi[a];
            for (a = 0; a < t.k; a++) acc[conn[(int64_t)a * T + e]] += t.qw[q] * mu * fh * phi[a];
        }
    }
    for (i = 0; i < N; i++) b[i] = (double)acc[i];
    free(acc);
    return bad ? OR_EDEGENERATE : OR_OK;
}

/* Non-linear terms of the mean-curvature-flow example (section 6.2, the
 * vector f = (f_1; f_2)): for a nodal vector field nu (n components,
 * nu[c*N + r]) and a nodal scalar H (NULL: H = 1),
 *   alpha^2 = |grad_Gamma_h nu_h|^2  (Frobenius norm of the tangential
 *             gradient; row c is grad_Gamma_h (nu_h)_c = sum_a nu_{c,a} grad phi_a)
 *   f[c*N + j] = sum_E sum_q w mu alpha^2 (nu_h)_c phi_j      c < n  (f_1)
 *   f[n*N + j] = sum_E sum_q w mu alpha^2 H_h phi_j                  (f_2)
 * The steps follow the listing of that section: local nodal values, the
 * gradient from the tangential basis gradients C^T [grad_hat phi; 0], its
 * Frobenius norm squared, the weighted point values, then the products with
 * phi_j summed over the points.  Contributions are added in element order. */
int oracle_kll(int surface, int d, int p, int Q, const double *qp, const double *qw, int64_t N,
               const double *coords, int64_t T, const int32_t *conn, const double *nu,
               const double *H, double *f)
{
    etype t;
    int st = make_type(&t, surface, d, p, Q, qp, qw), bad = 0;
    int64_t e, i;
    real *acc;
    if (st) return st;
    acc = (real *)calloc((size_t)(N > 0 ? N : 1) * (size_t)(t.n + 1), sizeof(real));
    if (!acc) return OR_ENOMEM;
    for (e = 0; e < T; e++) {
        real x[KMAX * DMAX], phi[KMAX], gp[KMAX * DMAX], ul[KMAX][DMAX + 1];
        int a, c, r, q;
        gather(&t, N, coords, T, conn, e, x);
        for (a = 0; a < t.k; a++) {
            int64_t g = conn[(int64_t)a * T + e];
            for (c = 0; c < t.n; c++) ul[a][c] = nu[(int64_t)c * N + g];
            ul[a][t.n] = H ? H[g] : 1.0;
        }
        for (q = 0; q < t.Q; q++) {
            real mu, alpha2 = 0.0, uh[DMAX + 1], wgt;
            if (point_geometry(&t, x, q, phi, gp, &mu)) bad = 1;
            for (c = 0; c < t.n; c++)
                for (r = 0; r < t.n; r++) {
                    real gcr = 0.0; /* d (nu_h)_c / d x_r, tangential */
                    for (a = 0; a < t.k; a++) gcr += ul[a][c] * gp[a * t.n + r];
                    alpha2 += gcr * gcr;
                }
            for (c = 0; c <= t.n; c++) {
                uh[c] = 0.0;
                for (a = 0; a < t.k; a++) uh[c] += ul[a][c] * phi[a];
            }
            wgt = t.qw[q] * mu * alpha2;
            for (a = 0; a < t.k; a++) {
                int64_t g = conn[(int64_t)a * T + e];
                for (c = 0; c <= t.n; c++) acc[(int64_t)c * N + g] += wgt * uh[c] * phi[a];
            }
        }
    }
    for (i = 0; i < N * (t.n + 1); i++) f[i] = (double)acc[i];
    free(acc);
    return bad ? OR_EDEGENERATE : OR_OK;
}
