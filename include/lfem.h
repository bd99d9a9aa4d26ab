/*
 * lfem.h -- C ABI of the MI355X (gfx950) isoparametric finite-element
 * assembly library (liblfem.so).
 *
 * What it computes.  For a mesh of linear (P1) or quadratic (P2)
 * isoparametric simplices -- curves in R^2, surfaces in R^3, bulk domains in
 * R^2 and R^3 (the element types of the paper's table of supported elements,
 * section 5) -- and of orders 3 and 4 on segments, triangles and tetrahedra
 * (the paper notes its assembly extends to degree 3 and up, section 1, and
 * its mesh utility builds orders 2 to 4 in one to three dimensions, section
 * 5.4) -- it assembles in FP64:
 *
 *   mass              M_ij   = sum_E sum_q w_q mu_E(xi_q) phi_i phi_j
 *   stiffness         A_ij   = sum_E sum_q w_q mu_E(xi_q) grad phi_i . grad phi_j
 *   weighted mass     Mc_ij  = sum_E sum_q w_q mu_E(xi_q) c_h(xi_q) phi_i phi_j
 *   coefficient stiffness: A with the factor a_h(xi_q) inside the sum
 *
 * (section 3.2: elementwise splitting of M and A, the local mass and
 * stiffness matrices, and their quadrature forms).  grad is the tangential
 * gradient on curves and surfaces (section 2.1, discrete tangential
 * gradient) and the ordinary gradient in bulk; mu is the surface/curve
 * measure |t1 x t2| or |t|, or |det DF| in bulk (section 3.2.1 and
 * Listing 1 (c)).  Nodal coefficients are interpolated with the element
 * basis: c_h = sum_r c_r phi_r.  Results are summed into a CSR matrix whose
 * pattern is structural: every (i, j) that share an element, diagonal
 * included, columns ascending, no entry dropped for being zero.
 *
 * Conventions for every entry point.
 *  - Indices are 0-based int32.  Coordinates are structure-of-arrays:
 *    coords[c * N + i] is coordinate c of node i (the paper's node array N,
 *    section 4).  Connectivity is structure-of-arrays: conn[a * T + e] is
 *    local node a of element e (the paper's element array E), corners first
 *    in anticlockwise order, then edge nodes: segment (0,1); triangle
 *    (0,1), (1,2), (2,0); tetrahedron (0,1), (1,2), (0,2), (0,3), (1,3), (2,3).
 *    Orders 3 and 4: the p - 1 nodes of each edge from its first corner to
 *    its second; on tetrahedra then the nodes inside the faces (0,1,2),
 *    (0,1,3), (0,2,3), (1,2,3), face by face (order 3: the face centroid;
 *    order 4: (2,1,1)/4, (1,2,1)/4, (1,1,2)/4 over the face's corners in
 *    that order); then the interior nodes (triangle, order 3: the centroid,
 *    order 4: (2,1,1)/4, (1,2,1)/4, (1,1,2)/4; tetrahedron, order 4: the
 *    centroid) in barycentric coordinates.
 *  - Every array argument is a DEVICE pointer owned by the caller; the
 *    library never frees it.  A mesh keeps the coords / conn pointers it was
 *    given (no copy): they must stay valid, and conn unchanged, for the
 *    mesh's lifetime.  Handles own their internal device buffers and release
 *    them in the matching *_destroy call.
 *  - stream is a hipStream_t passed as void* (NULL: the default stream).
 *    Calls enqueue work and return without waiting, except where a call says
 *    that it synchronises.
 *  - Every call returns an lfem_status; no exception crosses the ABI.  On an
 *    error lfem_last_error() returns a thread-local message.
 *  - Calls that share a handle must not overlap on different streams.
 */
#ifndef LFEM_H
#define LFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int lfem_status;
#define LFEM_OK 0
#define LFEM_EINVAL 1          /* bad argument (null pointer, bad size, index out of range) */
#define LFEM_ENOMEM 2          /* device or host allocation failed */
#define LFEM_EHIP 3            /* a HIP runtime call failed */
#define LFEM_ERANGE 4          /* nnz or an index would not fit in int32 */
#define LFEM_EDEGENERATE 5     /* degenerate elements were found */
#define LFEM_EUNSUPPORTED 6    /* element type / rule / option not supported */

/* domains */
#define LFEM_SURFACE 0         /* d-manifold in R^(d+1): curve (d=1) or surface (d=2) */
#define LFEM_BULK 1            /* d-dimensional domain in R^d, d = 2 or 3 */

/* matrix selection bits */
#define LFEM_M 1u              /* mass */
#define LFEM_A 2u              /* stiffness (optionally with a nodal coefficient) */
#define LFEM_MC 4u             /* weighted mass with a nodal coefficient */

/* numeric scatter variants (how local matrices are summed into CSR values) */
#define LFEM_SCATTER_AUTO 0     /* the pattern's tuned choice (blocked unless tuned otherwise) */
#define LFEM_SCATTER_BLOCKED 1  /* deterministic: row blocks accumulated in LDS (order-free adds
                                   where at most two contributions meet, fixed order elsewhere) */
#define LFEM_SCATTER_STAGED 2   /* deterministic: local matrices staged, slot-sorted segmented sum */
#define LFEM_SCATTER_ATOMIC 3   /* FP64 atomics into zeroed values; summation order not fixed */

/* flags of lfem_pattern_autotune_ex */
#define LFEM_TUNE_ALLOW_ATOMIC 1u /* also time the atomic scatter (its summation order is not fixed) */
#define LFEM_TUNE_NO_CACHE 2u     /* time the candidates even when the cache holds a result; refresh it */

typedef struct lfem_mesh_s *lfem_mesh_t;
typedef struct lfem_pattern_s *lfem_pattern_t;
typedef struct lfem_batch_s *lfem_batch_t;

/*
 * Create a mesh handle.  domain: LFEM_SURFACE or LFEM_BULK; dim: manifold
 * dimension d (surface: 1 or 2; bulk: 2 or 3); order: 1, 2, 3 or 4 (orders 3
 * and 4 take the high-order rules and the staged scatter).  The ambient
 * dimension is n_amb = d + 1 (surface) or d (bulk), so coords has
 * n_amb * n_nodes entries and conn has k * n_elems entries, k = C(order+d, d).
 * quad_points selects the quadrature rule on the reference simplex by its
 * number of points (0: the default for the element type):
 *   segment: 2 (Gauss, degree 3, P1 default), 3 (Gauss, degree 5, P2 default),
 *            5, 6 (Gauss, degree 9, 11)
 *   triangle: 3 (interior orbit, degree 2, P1 default), 6 (degree 4, P2 default),
 *            16 (Dunavant, degree 8)
 *   tetrahedron: 4 (degree 2, P1 default), 11 (degree 4, P2 default),
 *            35 (fully symmetric, degree 7, positive weights)
 * The rules are those of the paper's quadrature forms (section 3.2.2) and the
 * high-order rules of its precomputations (section 5.2: Gauss of degree 10 or
 * more on segments, Dunavant of degree 8 on triangles, degree 7 on
 * tetrahedra), with the weights summing to the reference measure.
 * Orders 3 and 4 take only the high-order rules (defaults: segment 5 points
 * for order 3 and 6 for order 4; triangle 16; tetrahedron 35).
 * Uploads the reference tables and builds the node -> element incidence
 * asynchronously on stream (device buffers are allocated with hipMalloc
 * first); use the handle on the same stream, or synchronise it before using
 * the handle on another.
 * Errors: LFEM_EINVAL (sizes, nulls), LFEM_ERANGE (n_elems * k >= 2^31),
 * LFEM_EUNSUPPORTED (type/rule), LFEM_ENOMEM, LFEM_EHIP.
 */
lfem_status lfem_mesh_create(int domain, int dim, int order, int64_t n_nodes,
                             const double *coords, int64_t n_elems, const int32_t *conn,
                             int quad_points, void *stream, lfem_mesh_t *out);

/* Point the mesh at new coordinates (moving mesh, same topology).  The next
 * assembly reads them, also through a batch that holds the mesh (its next
 * lfem_assemble_batch call re-uploads its descriptors); nothing is recomputed
 * eagerly.  The new array must stay valid while the mesh may read it. */
lfem_status lfem_mesh_set_coords(lfem_mesh_t m, const double *coords);

/*
 * Symbolic phase (once per topology): build the CSR pattern, the
 * element -> CSR slot map (one byte per local pair: the column offset inside
 * the row; two bytes for elements of more than 15 nodes, the cubic and
 * quartic tetrahedra, and for any mesh with a row of more than 255 entries, a
 * node of very high valence) and, except for P2 tetrahedra (whose default
 * is the staged scatter), the row-block schedule of the blocked
 * scatter.  A pattern with two-byte slots has no block schedule: its
 * LFEM_SCATTER_AUTO choice is the staged scatter, lfem_assemble runs a
 * blocked request staged, and lfem_pattern_schedule refuses the blocked
 * scatter with LFEM_EUNSUPPORTED.  The pattern is
 * the structural sparsity of the element array (the paper's sparse() step
 * without its value-dependent dropping).  SYNCHRONISES stream once to learn
 * nnz and to build the block schedule on the host.
 * Errors: LFEM_EINVAL (a conn entry outside [0, N) or repeated inside an
 * element), LFEM_ERANGE (nnz >= 2^31, or a row with more than 1023 entries),
 * LFEM_ENOMEM, LFEM_EHIP.
 */
lfem_status lfem_pattern_build(lfem_mesh_t m, void *stream, lfem_pattern_t *out);

/* Pattern sizes and device pointers (owned by the pattern): row_ptr has
 * n_rows + 1 entries, col_idx has nnz entries.  Any output may be NULL. */
lfem_status lfem_pattern_get(lfem_pattern_t p, int64_t *n_rows, int64_t *nnz,
                             const int32_t **row_ptr, const int32_t **col_idx);

/* Statistics of a pattern and of its blocked-scatter schedule. */
typedef struct {
    int64_t n_rows, nnz;
    int32_t max_row;          /* longest CSR row */
    int32_t blocks;           /* row blocks of the blocked scatter (0: none) */
    int32_t block_cap;        /* max values per block and matrix */
    int32_t max_block_rows;
    int32_t max_block_elems;
    int32_t max_colors;       /* colours used inside one block */
    double halo;              /* element evaluations per element (>= 1) */
    int32_t scatter;          /* variant used by LFEM_SCATTER_AUTO */
    int32_t slot_bytes;       /* bytes per local pair in the slot map: 1 or 2 */
} lfem_pattern_info_t;

lfem_status lfem_pattern_info(lfem_pattern_t p, lfem_pattern_info_t *info);

/*
 * Numeric phase, any subset of matrices in one pass over the elements.
 * what: bitwise OR of LFEM_M, LFEM_A, LFEM_MC.  coef_a: nodal coefficient
 * [N] inside the stiffness (NULL: 1).  coef_c: nodal coefficient [N] of the
 * weighted mass (required with LFEM_MC).  vals_m / vals_a / vals_mc: outputs
 * of nnz doubles each, overwritten (required for the selected matrices).
 * scatter: LFEM_SCATTER_*.  The blocked and staged scatters are bitwise
 * reproducible run to run; the atomic one is not.  Orders 3 and 4, and
 * patterns with rows of more than 255 entries, have no block schedule: a
 * blocked request takes the staged scatter.  P2 tetrahedra default to the
 * staged scatter; the first blocked request on such a pattern builds its
 * block schedule (colour mode) and SYNCHRONISES stream.
 * The first
 * staged call on a pattern builds its contribution lists and SYNCHRONISES
 * stream once (LFEM_EUNSUPPORTED if k^2 * n_elems >= 2^31); later calls are
 * asynchronous and allocate nothing while the staging buffer suffices.
 * Degenerate elements (measure not positive and finite) still produce values
 * and increment the mesh's counter (lfem_status_get).
 */
lfem_status lfem_assemble(lfem_mesh_t m, lfem_pattern_t p, unsigned what, const double *coef_a,
                          const double *coef_c, double *vals_m, double *vals_a, double *vals_mc,
                          int scatter, void *stream);

/* Single-matrix shorthands of lfem_assemble with LFEM_SCATTER_AUTO. */
lfem_status lfem_assemble_mass(lfem_mesh_t m, lfem_pattern_t p, double *vals, void *stream);
lfem_status lfem_assemble_stiffness(lfem_mesh_t m, lfem_pattern_t p, const double *coef,
                                    double *vals, void *stream);
lfem_status lfem_assemble_weighted(lfem_mesh_t m, lfem_pattern_t p, const double *coef,
                                   double *vals, void *stream);

/*
 * Product of an assembled matrix with nvec nodal vectors:
 *     y[c * N + i] = alpha * sum_j vals_ij x[c * N + j],   c < nvec,
 * vals: nnz doubles on pattern p (any matrix this library assembled on it);
 * x, y: nvec * N doubles, component-major, must not overlap.  Each row is
 * summed in column order (bitwise reproducible).  The operation the
 * paper's schemes apply to assembled matrices (the right-hand side M x^n of
 * Dziuk's scheme, section 6.3), and the partial derivatives of
 * u^T A v with respect to u and v (A v and A^T u = A u).
 * Errors: LFEM_EINVAL (null pattern or buffers, nvec < 1, x == y), LFEM_EHIP.
 */
lfem_status lfem_spmv(lfem_pattern_t p, const double *vals, const double *x, double alpha, double *y,
                      int nvec, void *stream);

/*
 * Per-step system of the linearly implicit mean-curvature-flow scheme the
 * paper times against DUNE (section 6.3, Dziuk's algorithm):
 *     (M(x^n) + tau A(x^n)) x^{n+1} = M(x^n) x^n.
 * Assembles M and A at the mesh's current coordinates into vals_m, vals_a
 * (nnz doubles each, the pattern's tuned scatter variant), then forms
 * vals_s = vals_m + tau * vals_a and rhs[c * N + i] = sum_j M_ij x[c * N + j]
 * for c < n_amb (each row summed in column order: deterministic).  x: n_amb *
 * N doubles, component-major, or NULL for the mesh's own coordinates.  The
 * linear solve is the caller's.  After one call (which builds the pattern's
 * lazy structures) a call allocates nothing, so it can be captured in a HIP
 * graph and replayed while the coordinates change in place.  A captured graph
 * keeps the pattern's staging buffers: an assembly on the same pattern that
 * needs larger ones (more matrices, staged) reallocates them, after which the
 * graph must be captured again.
 * Errors: LFEM_EINVAL (handles, null buffers, non-finite tau), LFEM_EHIP.
 */
lfem_status lfem_dziuk_system(lfem_mesh_t m, lfem_pattern_t p, double tau, const double *x,
                              double *vals_m, double *vals_a, double *vals_s, double *rhs,
                              void *stream);

/*
 * Per-step system of the paper's mean-curvature-flow algorithm of section 6.2
 * (evolving-surface finite elements, linearly implicit BDF time stepping of
 * the coupled system for u = (nu; H), nu the unit normal and H the mean
 * curvature).  With the BDF derivative u_dot^n = (1/tau) sum_{j>=0}
 * delta_j u^{n-j}, the equation M u_dot^n + A u^n = f(x~, u~) at the
 * extrapolated surface x~ and extrapolated u~ reads, per component,
 *     (delta0 M(x~) + tau A(x~)) u^n = tau f(x~, u~) - M(x~) hist,
 *     hist = sum_{j>=1} delta_j u^{n-j}.
 * The mesh's current coordinates are x~.  Assembles M and A into vals_m,
 * vals_a (nnz doubles each, the pattern's tuned scatter variant), the
 * non-linear terms f = (f_1; f_2) of nu = nu~, H = H~ exactly as
 * lfem_assemble_kll into f ((n_amb + 1) * N doubles), then forms
 * vals_s = delta0 * vals_m + tau * vals_a and, for c <= n_amb,
 *     rhs[c * N + i] = tau * f[c * N + i] - sum_j M_ij hist[c * N + j]
 * (each row summed in column order: deterministic).  nu: n_amb * N doubles
 * and hist, rhs: (n_amb + 1) * N doubles, all component-major with the
 * normal components first and H last; H: N doubles; hist may be NULL (zero
 * history).  The velocity v = -H^n nu^n and the position update are the
 * caller's, as are the linear solves.  After one call a call allocates
 * nothing (HIP-graph capturable, as lfem_dziuk_system); it uses the mesh's
 * scratch buffer: calls on one mesh must not overlap.
 * Errors: LFEM_EINVAL (handles, null buffers, non-finite tau or delta0),
 * LFEM_EHIP.
 */
lfem_status lfem_kll_system(lfem_mesh_t m, lfem_pattern_t p, double tau, double delta0, const double *nu,
                            const double *H, const double *hist, double *vals_m, double *vals_a,
                            double *vals_s, double *f, double *rhs, void *stream);

/*
 * Autotune the scatter variant and row-block size of pattern p for the
 * matrix set `what` (LFEM_M, LFEM_A or both) by timing the candidates on
 * stream (SYNCHRONISES): the blocked scatter at block capacities 2048 to
 * 8192 value entries (those the longest row and the LDS admit), the staged
 * scatter, and the atomic one only with LFEM_TUNE_ALLOW_ATOMIC.  The choice
 * is kept in the pattern and used by LFEM_SCATTER_AUTO (and by batches and
 * the step calls).  Results are cached for the life of the process, keyed by
 * device, element type, rule, `what`, size bucket (bit length of the element
 * count) and the atomic flag: a later call for a mesh with the same key
 * applies the cached choice without timing (unless LFEM_TUNE_NO_CACHE, which
 * times and refreshes the entry, or the cached capacity does not fit the new
 * pattern's longest row).  Tuning rebuilds the block schedule, which any
 * batch holding the pattern notices at its next run.  *variant_out and
 * *block_cap_out (either may be NULL) receive the choice (the capacity 0
 * unless blocked).  Scratch outputs are allocated and freed inside.
 */
lfem_status lfem_pattern_autotune_ex(lfem_mesh_t m, lfem_pattern_t p, unsigned what, unsigned flags,
                                     void *stream, int *variant_out, int *block_cap_out);

/* lfem_pattern_autotune_ex with flags 0 (deterministic candidates, cache on). */
lfem_status lfem_pattern_autotune(lfem_mesh_t m, lfem_pattern_t p, unsigned what, void *stream,
                                  int *variant_out);

/* Empty the autotuner's result cache (the patterns keep their choices). */
void lfem_tune_cache_clear(void);

/*
 * Manual schedule knob: make `variant` (LFEM_SCATTER_BLOCKED, _STAGED or
 * _ATOMIC) the pattern's LFEM_SCATTER_AUTO choice.  For the blocked scatter,
 * block_cap is the number of CSR value entries one workgroup holds in LDS per
 * matrix (0: the default, 4992 clamped to the longest row); the rows of a
 * block, and with them the elements one workgroup assembles, follow from it
 * (lfem_pattern_info reports max_block_rows and max_block_elems).  block_cap
 * must lie in [longest row, 20480] and hold one row with its side slots
 * (else LFEM_EINVAL); a capacity whose LDS
 * for the requested matrices exceeds 160 KiB fails at assembly with
 * LFEM_EUNSUPPORTED.  Orders 3 and 4 have no block schedule
 * (LFEM_EUNSUPPORTED for a blocked request; their blocked requests run
 * staged anyway).  Rebuilding the schedule is asynchronous on stream apart
 * from its host part (the block partition is built on the host).
 */
lfem_status lfem_pattern_schedule(lfem_mesh_t m, lfem_pattern_t p, int variant, int block_cap, void *stream);

/*
 * Batched assembly (section 6.1's many-meshes workload): n meshes of uneven
 * size assembled by one HIP graph replay.  Any mesh and rule the library
 * assembles may be a member:
 *   - curves, surfaces and planar domains of order 1 or 2 under their two
 *     default rules (segment 2 or 3 points, triangle 3 or 6 points), whose
 *     patterns carry a side-slot block schedule, without coefficients and
 *     without LFEM_MC, share one persistent launch (work items = (mesh, row
 *     block) pairs, largest first, pulled from an atomic counter);
 *   - every other member (tetrahedra, orders 3 and 4, high-order rules, a
 *     coefficient, the weighted mass) is assembled by its own numeric launch
 *     with its pattern's tuned scatter, recorded into the same graph.
 * Results equal lfem_assemble with LFEM_SCATTER_AUTO on each mesh bitwise.
 * what: matrices per mesh, any non-empty combination of LFEM_M, LFEM_A,
 * LFEM_MC.  autotune != 0 times the candidate block capacities of the
 * persistent kernel's members once at creation and rebuilds their schedules
 * (SYNCHRONISES stream).  Creation also runs each other member once on
 * scratch outputs to build its lazily created structures (SYNCHRONISES).
 * The handle keeps the mesh and pattern handles (which must outlive it).
 */
lfem_status lfem_batch_create(int n, const lfem_mesh_t *meshes, const lfem_pattern_t *pats,
                              unsigned what, int autotune, void *stream, lfem_batch_t *out);

/*
 * lfem_batch_create with nodal coefficients: coef_a[i] (may be NULL, or the
 * whole array NULL) is mesh i's device array of N_i doubles, the coefficient
 * a_h inside A (section 3.2); coef_c[i] the weight c_h of M_c, required for
 * every mesh with elements when what contains LFEM_MC (else LFEM_EINVAL).
 * The pointers are kept by the batch and read at every replay (their values
 * may change between calls; the arrays must outlive the batch).
 */
lfem_status lfem_batch_create_ex(int n, const lfem_mesh_t *meshes, const lfem_pattern_t *pats,
                                 unsigned what, const double *const *coef_a, const double *const *coef_c,
                                 int autotune, void *stream, lfem_batch_t *out);

/*
 * Run the batch.  vals[i * nmat + j] is the output of matrix j of mesh i,
 * nmat = number of bits in `what`, ordered M, A, MC; each has that mesh's
 * nnz doubles and is overwritten.  Each call reads every mesh's current
 * coordinates (lfem_mesh_set_coords).  When the output or coordinate pointers
 * of a persistent-kernel member differ from the previous call the library
 * waits for the previous descriptor upload before updating its device-side
 * pointer table; when those of another member (or its pattern's staging
 * buffer) differ from the graph's, the call SYNCHRONISES stream and captures
 * the graph again.  If a pattern's block schedule was rebuilt since the batch
 * was set up (lfem_pattern_autotune, another batch's autotuning), the call
 * SYNCHRONISES stream and rebuilds the work list and graph first; a member
 * whose new schedule the persistent kernel does not run gets a launch of its
 * own.  Calls of one batch that overlap on different streams race.
 */
lfem_status lfem_assemble_batch(lfem_batch_t b, double *const *vals, void *stream);

/*
 * Shape derivative (adjoint) of
 *     J(x) = alpha u^T A(x) v + beta w^T M(x) z
 * with respect to every node coordinate: grad[c * N + r] = dJ / dx_{r,c}
 * (n_amb * N doubles, overwritten).  u, v, w, z: nodal vectors [N]; the A
 * term is skipped when u or v is NULL, the M term when w or z is NULL.
 * Deterministic (fixed summation order).  Plain A and M only (no coefficients).
 */
lfem_status lfem_shape_grad(lfem_mesh_t m, const double *u, const double *v, double alpha,
                            const double *w, const double *z, double beta, double *grad,
                            void *stream);

/*
 * lfem_shape_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and result (bit for bit) as lfem_shape_grad, but
 * the staged per-element contributions live in a fixed 32 MiB workspace
 * inside the library (one per GPU, held until the process ends), so the
 * call makes no hipMalloc / hipFree or other allocating call.  Limit:
 * k * n_amb * n_elems <= 4194304 doubles (e.g. 233,016 P2 surface
 * triangles); larger meshes get LFEM_ERANGE before anything is launched.
 * The mesh's device must be current.  Calls on one GPU share the
 * workspace: calls that overlap on one GPU (different streams, or other
 * threads) race; serialise them.  Errors: LFEM_EINVAL (null mesh or grad,
 * wrong current device), LFEM_ERANGE (mesh too large), LFEM_EHIP.
 */
lfem_status lfem_shape_grad_noalloc(lfem_mesh_t m, const double *u, const double *v, double alpha,
                                    const double *w, const double *z, double beta, double *grad,
                                    void *stream);

/* Matrix-free value of the same J(x) into the device scalar *J_out. */
lfem_status lfem_energy(lfem_mesh_t m, const double *u, const double *v, double alpha,
                        const double *w, const double *z, double beta, double *J_out,
                        void *stream);

/*
 * Load vector (the right-hand side the paper's assembly returns beside M and
 * A, section 6.1):
 *     b[j] = sum_E sum_q w_q mu_E(xi_q) f_h(xi_q) phi_j(xi_q),
 * f_h = sum_r f_r phi_r the nodal data coef_f [N] interpolated with the
 * element basis (NULL: f = 1, so b = M 1).  b: N doubles, overwritten.  Each
 * element's contributions are staged and summed per node in ascending
 * element order (bitwise reproducible).  Uses the mesh's scratch buffer:
 * calls on one mesh must not overlap.
 */
lfem_status lfem_assemble_load(lfem_mesh_t m, const double *coef_f, double *b, void *stream);

/*
 * Non-linear terms of the paper's mean-curvature-flow example (section 6.2,
 * the vector f = (f_1; f_2)): for a nodal vector field nu and a nodal scalar H,
 *     alpha^2 = |grad_Gamma_h nu_h|^2   (Frobenius norm of the tangential
 *               gradient of nu_h = sum_r nu_r phi_r),
 *     f[c * N + j]     = sum_E sum_q w_q mu alpha^2 (nu_h)_c phi_j,  c < n_amb (f_1)
 *     f[n_amb * N + j] = sum_E sum_q w_q mu alpha^2 H_h phi_j                  (f_2)
 * nu: n_amb * N doubles, component-major (nu[c * N + r]); H: N doubles, or
 * NULL for H = 1; f: (n_amb + 1) * N doubles, overwritten.  Any element type
 * (in the bulk the gradient is the full gradient).  Deterministic like the
 * load vector; uses the mesh's scratch buffer: calls on one mesh must not
 * overlap.  Errors: LFEM_EINVAL (null mesh, nu or f with N > 0), LFEM_EHIP.
 */
lfem_status lfem_assemble_kll(lfem_mesh_t m, const double *nu, const double *H, double *f,
                              void *stream);

/*
 * Host query of the reference data the library builds for an element type
 * (no device is touched): the quadrature rule of quad_points points (0: the
 * default of the type) and the nodal basis at its points, the precomputed
 * quantities of the paper's assembly (section 5.2).  *q_out and *k_out get
 * the number of points Q and of element nodes k; each non-NULL array gets
 * w[Q] (weights, summing to the reference measure), xi[Q * dim] (points),
 * phi[Q * k] (phi_a(xi_q) at q * k + a) and dphi[Q * k * dim]
 * (d phi_a / d xi_m at (q * k + a) * dim + m).  Call with NULL arrays to
 * learn the sizes.  Errors: LFEM_EINVAL (null q_out or k_out),
 * LFEM_EUNSUPPORTED (type or rule).
 */
lfem_status lfem_reference_table(int dim, int order, int quad_points, int *q_out, int *k_out,
                                 double *w, double *xi, double *phi, double *dphi);

/* Number of degenerate (element, quadrature point) evaluations seen by this
 * mesh since creation or the last reset.  SYNCHRONISES the whole device
 * (hipDeviceSynchronize: the counter may be written from any stream the mesh
 * was used on), then reads the counter. */
lfem_status lfem_status_get(lfem_mesh_t m, int64_t *n_degenerate);
lfem_status lfem_status_reset(lfem_mesh_t m, void *stream);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *lfem_last_error(void);

/* Library version string. */
const char *lfem_version(void);

/*
 * Debug mode (a development aid; off unless the environment
 * variable LFEM_DEBUG=1 is set when the library loads, or this call turns it
 * on).  While on, every call that reads a mesh's connectivity (the assembly,
 * step, load, mean-curvature-flow, energy and shape-gradient calls, autotuning
 * and batches at creation and at every run) first runs a bounds check on the
 * GPU: each node id in [0, N), and, for calls that assemble into a pattern,
 * the slot of every local pair (a, b) inside row conn[a] holding column
 * conn[b] (catches a connectivity edited after the pattern was built).  The
 * first failing element is reported as LFEM_EINVAL, naming the element and
 * the reason (lfem_last_error), and nothing is launched.  The check
 * SYNCHRONISES the stream and must not be captured into a graph; checks from
 * several threads are serialised.  Returns the previous setting.
 */
int lfem_set_debug(int on);

/* Release a handle and its device buffers.  Each destroy call first waits
 * for all work on the device (hipDeviceSynchronize), since work on any stream
 * may still read the buffers.  NULL is ignored. */
void lfem_mesh_destroy(lfem_mesh_t m);
void lfem_pattern_destroy(lfem_pattern_t p);
void lfem_batch_destroy(lfem_batch_t b);

#ifdef __cplusplus
}
#endif

#endif /* LFEM_H */
