/*
 * Test infrastructure: a stand-alone driver that runs every entry point of
 * the CPU oracle (lfem_oracle.c) on one mesh read from a file, so the oracle
 * can be built and exercised under AddressSanitizer and
 * UndefinedBehaviorSanitizer (gcc, host code only).  It is never part of the
 * library's path.
 *
 * Input (native little-endian binary):
 *   int64 surface, d, p, Q, N, T
 *   double qp[Q * d], qw[Q], coords[n_amb * N]   (n_amb = d + surface)
 *   int32  conn[k * T]                           (k nodes per element)
 *   double coef[N], u[N], v[N], w[N], z[N], nu[n_amb * N], H[N]
 * Output (doubles):
 *   for each of M, A, M_c (coef), A_a (coef): nnz, then the values in CSR
 *   order; the values of A_a again from the numeric-only entry point on the
 *   pattern just built; J = 1.0 u^T A v + 0.5 w^T M z; the shape gradient
 *   [n_amb * N]; the load vector with f = coef [N]; the mean-curvature-flow
 *   terms [(n_amb + 1) * N].
 * Exit status 0 on success, 2 on bad input, 3 when an oracle call fails.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_nodes_per_element(int d, int p);
int oracle_assemble(int surface, int d, int p, int Q, const double *qp, const double *qw,
                    int64_t N, const double *coords, int64_t T, const int32_t *conn,
                    const double *coef, int kind, const uint8_t *row_mask, int64_t cap,
                    int64_t *row_ptr, int32_t *col_idx, double *vals, int64_t *nnz_out);
int oracle_assemble_numeric(int surface, int d, int p, int Q, const double *qp,
                            const double *qw, int64_t N, const double *coords, int64_t T,
                            const int32_t *conn, const double *coef, int kind,
                            const int64_t *row_ptr, const int32_t *col_idx, double *vals);
int oracle_energy(int surface, int d, int p, int Q, const double *qp, const double *qw,
                  int64_t N, const double *coords, int64_t T, const int32_t *conn,
                  const double *u, const double *v, double alpha, const double *w,
                  const double *z, double beta, double *J_out);
int oracle_shape_grad(int surface, int d, int p, int Q, const double *qp, const double *qw,
                      int64_t N, const double *coords, int64_t T, const int32_t *conn,
                      const double *u, const double *v, double alpha, const double *w,
                      const double *z, double beta, double *grad);
int oracle_load(int surface, int d, int p, int Q, const double *qp, const double *qw, int64_t N,
                const double *coords, int64_t T, const int32_t *conn, const double *f, double *b);
int oracle_kll(int surface, int d, int p, int Q, const double *qp, const double *qw, int64_t N,
               const double *coords, int64_t T, const int32_t *conn, const double *nu,
               const double *H, double *f);

static void *read_block(FILE *fp, size_t count, size_t size)
{
    void *p = malloc(count * size > 0 ? count * size : 1);
    if (!p || fread(p, size, count, fp) != count) {
        free(p);
        return NULL;
    }
    return p;
}

static int put(FILE *fp, const double *x, int64_t n)
{
    return fwrite(x, sizeof(double), (size_t)n, fp) == (size_t)n ? 0 : 1;
}

int main(int argc, char **argv)
{
    int64_t h[6];
    FILE *in, *out;
    double *qp, *qw, *coords, *coef, *u, *v, *w, *z, *nu, *H;
    int32_t *conn;
    int surface, d, p, Q, k, n_amb, kind, st = 0, err = 0;
    int64_t N, T, cap, nnz = 0;
    int64_t *row_ptr;
    int32_t *col_idx;
    double *vals, *again, *grad, *b, *f, J = 0.0, dn;
    if (argc != 3) return 2;
    in = fopen(argv[1], "rb");
    if (!in || fread(h, sizeof(int64_t), 6, in) != 6) return 2;
    surface = (int)h[0];
    d = (int)h[1];
    p = (int)h[2];
    Q = (int)h[3];
    N = h[4];
    T = h[5];
    k = oracle_nodes_per_element(d, p);
    n_amb = d + surface;
    if (k <= 0 || Q <= 0 || N <= 0 || T < 0) return 2;
    qp = read_block(in, (size_t)Q * d, sizeof(double));
    qw = read_block(in, (size_t)Q, sizeof(double));
    coords = read_block(in, (size_t)n_amb * N, sizeof(double));
    conn = read_block(in, (size_t)k * T, sizeof(int32_t));
    coef = read_block(in, (size_t)N, sizeof(double));
    u = read_block(in, (size_t)N, sizeof(double));
    v = read_block(in, (size_t)N, sizeof(double));
    w = read_block(in, (size_t)N, sizeof(double));
    z = read_block(in, (size_t)N, sizeof(double));
    nu = read_block(in, (size_t)n_amb * N, sizeof(double));
    H = read_block(in, (size_t)N, sizeof(double));
    fclose(in);
    if (!qp || !qw || !coords || !conn || !coef || !u || !v || !w || !z || !nu || !H) return 2;
    cap = (int64_t)k * k * T;
    if (cap < 1) cap = 1;
    row_ptr = malloc((size_t)(N + 1) * sizeof(int64_t));
    col_idx = malloc((size_t)cap * sizeof(int32_t));
    vals = malloc((size_t)cap * sizeof(double));
    again = malloc((size_t)cap * sizeof(double));
    grad = malloc((size_t)n_amb * N * sizeof(double));
    b = malloc((size_t)N * sizeof(double));
    f = malloc((size_t)(n_amb + 1) * N * sizeof(double));
    out = fopen(argv[2], "wb");
    if (!row_ptr || !col_idx || !vals || !again || !grad || !b || !f || !out) return 2;
    /* M, A, M_c, A_a */
    for (kind = 0; kind < 4 && !st; ++kind) {
        st = oracle_assemble(surface, d, p, Q, qp, qw, N, coords, T, conn, kind >= 2 ? coef : NULL,
                             kind & 1, NULL, cap, row_ptr, col_idx, vals, &nnz);
        if (st) break;
        dn = (double)nnz;
        err |= put(out, &dn, 1) | put(out, vals, nnz);
    }
    /* A_a again into the pattern of the last call */
    if (!st) st = oracle_assemble_numeric(surface, d, p, Q, qp, qw, N, coords, T, conn, coef, 1, row_ptr,
                                          col_idx, again);
    if (!st) err |= put(out, again, nnz);
    if (!st) st = oracle_energy(surface, d, p, Q, qp, qw, N, coords, T, conn, u, v, 1.0, w, z, 0.5, &J);
    if (!st) err |= put(out, &J, 1);
    if (!st) st = oracle_shape_grad(surface, d, p, Q, qp, qw, N, coords, T, conn, u, v, 1.0, w, z, 0.5, grad);
    if (!st) err |= put(out, grad, (int64_t)n_amb * N);
    if (!st) st = oracle_load(surface, d, p, Q, qp, qw, N, coords, T, conn, coef, b);
    if (!st) err |= put(out, b, N);
    if (!st) st = oracle_kll(surface, d, p, Q, qp, qw, N, coords, T, conn, nu, H, f);
    if (!st) err |= put(out, f, (int64_t)(n_amb + 1) * N);
    fclose(out);
    free(qp);
    free(qw);
    free(coords);
    free(conn);
    free(coef);
    free(u);
    free(v);
    free(w);
    free(z);
    free(nu);
    free(H);
    free(row_ptr);
    free(col_idx);
    free(vals);
    free(again);
    free(grad);
    free(b);
    free(f);
    if (st) {
        fprintf(stderr, "oracle call failed with status %d\n", st);
        return 3;
    }
    return err ? 2 : 0;
}
