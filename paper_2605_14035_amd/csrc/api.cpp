// The extern "C" boundary of liblfem.so: argument checks, handle lifetime and
// error translation.  No exception crosses this file's functions.
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "lfem_internal.hpp"

namespace lfem {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char *last_error() { return g_last_error.c_str(); }

// rows per block of the blocked scatter's default schedule
constexpr int kMaxRows = kBlockMaxRows;
// largest block capacity: one matrix region filling a compute unit's LDS
constexpr int kMaxBlockCap = 160 * 1024 / 8;

}  // namespace lfem

using namespace lfem;

struct lfem_mesh_s : Mesh {};
struct lfem_pattern_s : Pattern {};

namespace lfem {
// batch.hip
lfem_status batch_create(int n, Mesh *const *meshes, Pattern *const *pats, unsigned what,
                         const double *const *coef_a, const double *const *coef_c, int autotune,
                         hipStream_t s, lfem_batch_t *out);
void batch_run(lfem_batch_t b, double *const *vals, hipStream_t s);
void batch_destroy(lfem_batch_t b);
void batch_debug_check(lfem_batch_t b, hipStream_t s);
// tune.cpp
int autotune_pattern(Mesh &m, Pattern &p, unsigned what, unsigned flags, hipStream_t s);
void tune_cache_clear();
}  // namespace lfem

namespace {

template <class F>
lfem_status guarded(F &&f)
{
    try {
        clear_error();
        f();
        return LFEM_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return LFEM_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LFEM_EINVAL;
    } catch (...) {
        set_error("unknown error");
        return LFEM_EINVAL;
    }
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

void release_mesh(Mesh &m)
{
    dev_free(m.tab);
    dev_free(m.tabp);
    dev_free(m.ne_ptr);
    dev_free(m.ne);
    dev_free(m.flags);
    dev_free(m.degenerate);
    dev_free(m.scratch);
}

void release_pattern(Pattern &p)
{
    dev_free(p.row_ptr);
    dev_free(p.col_idx);
    dev_free(p.off8);
    dev_free(p.off16);
    dev_free(p.cptr);
    dev_free(p.clist);
    dev_free(p.long_slots);
    dev_free(p.stage);
    dev_free(p.dstage);
    free_schedule(p.sched);
}

void check_numeric_args(const Mesh *m, const Pattern *p, unsigned what, const double *coef_c,
                        double *vm, double *va, double *vmc)
{
    LFEM_REQUIRE(m && p, LFEM_EINVAL, "null mesh or pattern handle");
    LFEM_REQUIRE(p->mesh == m, LFEM_EINVAL, "pattern was built for another mesh");
    LFEM_REQUIRE(what != 0 && (what & ~(LFEM_M | LFEM_A | LFEM_MC)) == 0, LFEM_EINVAL,
                 "what must be a non-empty combination of LFEM_M, LFEM_A, LFEM_MC");
    // with nnz == 0 (no elements) there is nothing to write and null outputs are fine
    const bool need = p->nnz > 0;
    LFEM_REQUIRE(!(what & LFEM_M) || vm || !need, LFEM_EINVAL, "vals_m is null");
    LFEM_REQUIRE(!(what & LFEM_A) || va || !need, LFEM_EINVAL, "vals_a is null");
    LFEM_REQUIRE(!(what & LFEM_MC) || ((vmc && coef_c) || !need), LFEM_EINVAL,
                 "weighted mass needs coef_c and vals_mc");
    LFEM_REQUIRE(m->coords || m->N == 0, LFEM_EINVAL, "mesh has no coordinates");
}

}  // namespace

extern "C" {

const char *lfem_last_error(void) { return last_error(); }

int lfem_set_debug(int on) { return set_debug(on); }

const char *lfem_version(void) { return "lfem-mi355x 0.1 (gfx950, fp64)"; }

lfem_status lfem_mesh_create(int domain, int dim, int order, int64_t n_nodes,
                             const double *coords, int64_t n_elems, const int32_t *conn,
                             int quad_points, void *stream, lfem_mesh_t *out)
{
    return guarded([&] {
        LFEM_REQUIRE(out, LFEM_EINVAL, "out is null");
        *out = nullptr;
        const int et = etype_of(domain, dim, order);
        LFEM_REQUIRE(order >= 1 && order <= 4, LFEM_EUNSUPPORTED, "order must be 1, 2, 3 or 4");
        LFEM_REQUIRE(et >= 0, LFEM_EUNSUPPORTED, "unsupported (domain, dim)");
        LFEM_REQUIRE(n_nodes >= 0 && n_elems >= 0, LFEM_EINVAL, "negative size");
        LFEM_REQUIRE(n_nodes < (int64_t(1) << 31) - 1, LFEM_ERANGE, "n_nodes >= 2^31 - 1");
        const int k = nodes_per_elem(dim, order);
        LFEM_REQUIRE(n_elems * k < (int64_t(1) << 31), LFEM_ERANGE,
                     "too many element nodes for int32 incidence codes (k * n_elems >= 2^31)");
        LFEM_REQUIRE(n_nodes == 0 || coords, LFEM_EINVAL, "coords is null");
        LFEM_REQUIRE(n_elems == 0 || conn, LFEM_EINVAL, "conn is null");
        RefTable tab;
        LFEM_REQUIRE(build_ref_table(dim, order, quad_points, tab), LFEM_EUNSUPPORTED,
                     "no quadrature rule with that number of points for this simplex");
        LFEM_REQUIRE(order <= 2 || tab.Q >= (dim == 1 ? 5 : (dim == 2 ? 16 : 35)), LFEM_EUNSUPPORTED,
                     "orders 3 and 4 take the high-order rules (segment 5 or 6, triangle 16, "
                     "tetrahedron 35 points)");
        auto *m = new lfem_mesh_s();
        try {
            m->domain = domain;
            m->d = dim;
            m->p = order;
            m->namb = domain == LFEM_SURFACE ? dim + 1 : dim;
            m->k = k;
            m->etype = et;
            m->Q = tab.Q;
            m->tab_stride = tab.stride;
            m->N = n_nodes;
            m->T = n_elems;
            m->coords = coords;
            m->conn = conn;
            LFEM_HIP(hipGetDevice(&m->device));
            // the uploads read the mesh's own copy of the tables, which lives
            // as long as the handle, so nothing here waits for the stream
            m->host_tab = std::move(tab);
            const RefTable &ht = m->host_tab;
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&m->tab), ht.data.size() * sizeof(double)));
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&m->flags), 4 * sizeof(int32_t)));
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&m->degenerate), sizeof(unsigned long long)));
            LFEM_HIP(hipMemcpyAsync(m->tab, ht.data.data(), ht.data.size() * sizeof(double),
                                    hipMemcpyHostToDevice, S(stream)));
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&m->tabp), ht.pairs.size() * sizeof(double)));
            LFEM_HIP(hipMemcpyAsync(m->tabp, ht.pairs.data(), ht.pairs.size() * sizeof(double),
                                    hipMemcpyHostToDevice, S(stream)));
            LFEM_HIP(hipMemsetAsync(m->degenerate, 0, sizeof(unsigned long long), S(stream)));
            build_incidence(*m, S(stream));
        } catch (...) {
            (void)hipStreamSynchronize(S(stream));
            release_mesh(*m);
            delete m;
            throw;
        }
        *out = m;
    });
}

lfem_status lfem_mesh_set_coords(lfem_mesh_t m, const double *coords)
{
    return guarded([&] {
        LFEM_REQUIRE(m, LFEM_EINVAL, "null mesh");
        LFEM_REQUIRE(coords || m->N == 0, LFEM_EINVAL, "coords is null");
        m->coords = coords;
    });
}

lfem_status lfem_pattern_build(lfem_mesh_t m, void *stream, lfem_pattern_t *out)
{
    return guarded([&] {
        LFEM_REQUIRE(m && out, LFEM_EINVAL, "null argument");
        *out = nullptr;
        auto *p = new lfem_pattern_s();
        try {
            build_pattern(*m, *p, S(stream));
            if (m->N > 0 && m->T > 0) {
                if (m->d == 3 && m->p == 2) {
                    // P2 tetrahedra take the staged scatter by default (1.9 ms
                    // against 6.5 ms for the colour-blocked one, M + A on the
                    // 1.57 M-element cube; P1 tetrahedra the other way round,
                    // 0.15 against 0.43 ms); their block schedule is built when
                    // a blocked scatter is requested or timed
                    p->tuned_variant = LFEM_SCATTER_STAGED;
                } else {
                    try {
                        build_schedule(*m, *p, default_block_cap(p->max_row), kMaxRows, S(stream));
                    } catch (const Error &e) {
                        if (e.code != LFEM_EUNSUPPORTED) throw;
                        p->tuned_variant = LFEM_SCATTER_STAGED;  // no block schedule possible
                    }
                }
            }
        } catch (...) {
            release_pattern(*p);
            delete p;
            throw;
        }
        *out = p;
    });
}

lfem_status lfem_pattern_get(lfem_pattern_t p, int64_t *n_rows, int64_t *nnz,
                             const int32_t **row_ptr, const int32_t **col_idx)
{
    return guarded([&] {
        LFEM_REQUIRE(p, LFEM_EINVAL, "null pattern");
        if (n_rows) *n_rows = p->mesh->N;
        if (nnz) *nnz = p->nnz;
        if (row_ptr) *row_ptr = p->row_ptr;
        if (col_idx) *col_idx = p->col_idx;
    });
}

lfem_status lfem_pattern_info(lfem_pattern_t p, lfem_pattern_info_t *info)
{
    return guarded([&] {
        LFEM_REQUIRE(p && info, LFEM_EINVAL, "null argument");
        info->n_rows = p->mesh->N;
        info->nnz = p->nnz;
        info->max_row = p->max_row;
        info->blocks = p->sched.nb;
        info->block_cap = p->sched.cap;
        info->max_block_rows = p->sched.max_rows;
        info->max_block_elems = p->sched.max_elems;
        info->max_colors = p->sched.max_colors;
        info->halo = p->sched.halo;
        info->scatter = p->tuned_variant;
        info->slot_bytes = p->off16 ? 2 : 1;
    });
}

lfem_status lfem_assemble(lfem_mesh_t m, lfem_pattern_t p, unsigned what, const double *coef_a,
                          const double *coef_c, double *vals_m, double *vals_a, double *vals_mc,
                          int scatter, void *stream)
{
    return guarded([&] {
        check_numeric_args(m, p, what, coef_c, vals_m, vals_a, vals_mc);
        LFEM_REQUIRE(scatter >= LFEM_SCATTER_AUTO && scatter <= LFEM_SCATTER_ATOMIC, LFEM_EINVAL,
                     "unknown scatter variant");
        int variant = scatter == LFEM_SCATTER_AUTO ? p->tuned_variant : scatter;
        if (variant == LFEM_SCATTER_BLOCKED && p->sched.nb == 0 && m->T > 0) {
            // no block schedule yet: build the default one where one can exist
            // (orders 1 and 2 with byte slot maps), else take the staged scatter
            variant = LFEM_SCATTER_STAGED;
            if (m->p <= 2 && p->off8) {
                try {
                    build_schedule(*m, *p, default_block_cap(p->max_row), kMaxRows, S(stream));
                    variant = LFEM_SCATTER_BLOCKED;
                } catch (const Error &e) {
                    if (e.code != LFEM_EUNSUPPORTED) throw;
                }
            }
        }
        NumericOut o;
        o.what = what;
        o.coef_a = coef_a;
        o.coef_c = coef_c;
        o.vals_m = vals_m;
        o.vals_a = vals_a;
        o.vals_mc = vals_mc;
        debug_check(*m, p, S(stream));
        launch_numeric(*m, *p, o, variant, S(stream));
    });
}

lfem_status lfem_dziuk_system(lfem_mesh_t m, lfem_pattern_t p, double tau, const double *x,
                              double *vals_m, double *vals_a, double *vals_s, double *rhs, void *stream)
{
    return guarded([&] {
        check_numeric_args(m, p, LFEM_M | LFEM_A, nullptr, vals_m, vals_a, nullptr);
        LFEM_REQUIRE(vals_s || p->nnz == 0, LFEM_EINVAL, "vals_s is null");
        LFEM_REQUIRE(rhs || m->N == 0, LFEM_EINVAL, "rhs is null");
        LFEM_REQUIRE(std::isfinite(tau), LFEM_EINVAL, "tau is not finite");
        int variant = p->tuned_variant;
        if (variant == LFEM_SCATTER_BLOCKED && p->sched.nb == 0 && m->T > 0) variant = LFEM_SCATTER_STAGED;
        debug_check(*m, p, S(stream));
        launch_dziuk(*m, *p, tau, x, vals_m, vals_a, vals_s, rhs, variant, S(stream));
    });
}

lfem_status lfem_kll_system(lfem_mesh_t m, lfem_pattern_t p, double tau, double delta0, const double *nu,
                            const double *H, const double *hist, double *vals_m, double *vals_a, double *vals_s,
                            double *f, double *rhs, void *stream)
{
    return guarded([&] {
        check_numeric_args(m, p, LFEM_M | LFEM_A, nullptr, vals_m, vals_a, nullptr);
        LFEM_REQUIRE(vals_s || p->nnz == 0, LFEM_EINVAL, "vals_s is null");
        LFEM_REQUIRE((nu && H && f && rhs) || m->N == 0, LFEM_EINVAL, "nu, H, f or rhs is null");
        LFEM_REQUIRE(std::isfinite(tau) && std::isfinite(delta0), LFEM_EINVAL, "tau or delta0 is not finite");
        int variant = p->tuned_variant;
        if (variant == LFEM_SCATTER_BLOCKED && p->sched.nb == 0 && m->T > 0) variant = LFEM_SCATTER_STAGED;
        debug_check(*m, p, S(stream));
        launch_kll_system(*m, *p, tau, delta0, nu, H, hist, vals_m, vals_a, vals_s, f, rhs, variant, S(stream));
    });
}

lfem_status lfem_spmv(lfem_pattern_t p, const double *vals, const double *x, double alpha, double *y,
                      int nvec, void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(p, LFEM_EINVAL, "null pattern");
        LFEM_REQUIRE(nvec >= 1, LFEM_EINVAL, "nvec must be at least 1");
        const int64_t n = p->mesh->N;
        LFEM_REQUIRE(n == 0 || (x && y), LFEM_EINVAL, "x or y is null");
        LFEM_REQUIRE(p->nnz == 0 || vals, LFEM_EINVAL, "vals is null");
        LFEM_REQUIRE(x != y || n == 0, LFEM_EINVAL, "x and y must not alias");
        launch_spmv(*p, vals, x, alpha, y, nvec, S(stream));
    });
}

lfem_status lfem_assemble_mass(lfem_mesh_t m, lfem_pattern_t p, double *vals, void *stream)
{
    return lfem_assemble(m, p, LFEM_M, nullptr, nullptr, vals, nullptr, nullptr,
                         LFEM_SCATTER_AUTO, stream);
}

lfem_status lfem_assemble_stiffness(lfem_mesh_t m, lfem_pattern_t p, const double *coef,
                                    double *vals, void *stream)
{
    return lfem_assemble(m, p, LFEM_A, coef, nullptr, nullptr, vals, nullptr, LFEM_SCATTER_AUTO,
                         stream);
}

lfem_status lfem_assemble_weighted(lfem_mesh_t m, lfem_pattern_t p, const double *coef,
                                   double *vals, void *stream)
{
    return lfem_assemble(m, p, LFEM_MC, nullptr, coef, nullptr, nullptr, vals, LFEM_SCATTER_AUTO,
                         stream);
}

lfem_status lfem_pattern_autotune_ex(lfem_mesh_t m, lfem_pattern_t p, unsigned what, unsigned flags,
                                     void *stream, int *variant_out, int *block_cap_out)
{
    return guarded([&] {
        LFEM_REQUIRE(m && p && p->mesh == m, LFEM_EINVAL, "bad mesh/pattern");
        LFEM_REQUIRE(what != 0 && (what & ~(LFEM_M | LFEM_A)) == 0, LFEM_EINVAL,
                     "autotune supports LFEM_M | LFEM_A");
        LFEM_REQUIRE((flags & ~(LFEM_TUNE_ALLOW_ATOMIC | LFEM_TUNE_NO_CACHE)) == 0, LFEM_EINVAL,
                     "unknown autotune flag");
        debug_check(*m, p, S(stream));
        const int v = autotune_pattern(*m, *p, what, flags, S(stream));
        if (variant_out) *variant_out = v;
        if (block_cap_out) *block_cap_out = v == LFEM_SCATTER_BLOCKED ? p->sched.cap : 0;
    });
}

lfem_status lfem_pattern_autotune(lfem_mesh_t m, lfem_pattern_t p, unsigned what, void *stream,
                                  int *variant_out)
{
    return lfem_pattern_autotune_ex(m, p, what, 0, stream, variant_out, nullptr);
}

void lfem_tune_cache_clear(void) { tune_cache_clear(); }

lfem_status lfem_pattern_schedule(lfem_mesh_t m, lfem_pattern_t p, int variant, int block_cap, void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m && p && p->mesh == m, LFEM_EINVAL, "bad mesh/pattern");
        LFEM_REQUIRE(variant >= LFEM_SCATTER_BLOCKED && variant <= LFEM_SCATTER_ATOMIC, LFEM_EINVAL,
                     "unknown scatter variant");
        if (variant == LFEM_SCATTER_BLOCKED && m->T > 0) {
            LFEM_REQUIRE(block_cap == 0 || (block_cap >= p->max_row && block_cap <= kMaxBlockCap), LFEM_EINVAL,
                         "block capacity outside [longest row, LDS limit]");
            build_schedule(*m, *p, block_cap == 0 ? default_block_cap(p->max_row) : block_cap, kMaxRows,
                           S(stream));
        }
        p->tuned_variant = variant;
    });
}

lfem_status lfem_batch_create_ex(int n, const lfem_mesh_t *meshes, const lfem_pattern_t *pats,
                                 unsigned what, const double *const *coef_a, const double *const *coef_c,
                                 int autotune, void *stream, lfem_batch_t *out)
{
    lfem_status st = LFEM_OK;
    lfem_status g = guarded([&] {
        LFEM_REQUIRE(out && n > 0 && meshes && pats, LFEM_EINVAL, "bad batch arguments");
        *out = nullptr;
        std::vector<Mesh *> ms(n);
        std::vector<Pattern *> ps(n);
        for (int i = 0; i < n; ++i) {
            LFEM_REQUIRE(meshes[i] && pats[i] && pats[i]->mesh == meshes[i], LFEM_EINVAL,
                         "batch entry with a null or mismatched mesh/pattern");
            LFEM_REQUIRE(meshes[i]->coords || meshes[i]->N == 0, LFEM_EINVAL, "mesh has no coordinates");
            ms[i] = meshes[i];
            ps[i] = pats[i];
        }
        for (int i = 0; i < n; ++i) debug_check(*ms[i], ps[i], S(stream));
        st = batch_create(n, ms.data(), ps.data(), what, coef_a, coef_c, autotune, S(stream), out);
    });
    return g != LFEM_OK ? g : st;
}

lfem_status lfem_batch_create(int n, const lfem_mesh_t *meshes, const lfem_pattern_t *pats,
                              unsigned what, int autotune, void *stream, lfem_batch_t *out)
{
    return lfem_batch_create_ex(n, meshes, pats, what, nullptr, nullptr, autotune, stream, out);
}

lfem_status lfem_assemble_batch(lfem_batch_t b, double *const *vals, void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(b && vals, LFEM_EINVAL, "null batch or vals");
        batch_debug_check(b, S(stream));
        batch_run(b, vals, S(stream));
    });
}

lfem_status lfem_shape_grad(lfem_mesh_t m, const double *u, const double *v, double alpha,
                            const double *w, const double *z, double beta, double *grad,
                            void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m && grad, LFEM_EINVAL, "null mesh or grad");
        debug_check(*m, nullptr, S(stream));
        launch_shape_grad(*m, u, v, alpha, w, z, beta, grad, S(stream));
    });
}

lfem_status lfem_shape_grad_noalloc(lfem_mesh_t m, const double *u, const double *v, double alpha,
                                    const double *w, const double *z, double beta, double *grad,
                                    void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m && grad, LFEM_EINVAL, "null mesh or grad");
        debug_check(*m, nullptr, S(stream));
        launch_shape_grad_noalloc(*m, u, v, alpha, w, z, beta, grad, S(stream));
    });
}

lfem_status lfem_energy(lfem_mesh_t m, const double *u, const double *v, double alpha,
                        const double *w, const double *z, double beta, double *J_out,
                        void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m && J_out, LFEM_EINVAL, "null mesh or J_out");
        debug_check(*m, nullptr, S(stream));
        launch_energy(*m, u, v, alpha, w, z, beta, J_out, S(stream));
    });
}

lfem_status lfem_assemble_load(lfem_mesh_t m, const double *coef_f, double *b, void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m && (b || m->N == 0), LFEM_EINVAL, "null mesh or b");
        debug_check(*m, nullptr, S(stream));
        launch_load(*m, coef_f, b, S(stream));
    });
}

lfem_status lfem_assemble_kll(lfem_mesh_t m, const double *nu, const double *H, double *f, void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m && ((nu && f) || m->N == 0), LFEM_EINVAL, "null mesh, nu or f");
        debug_check(*m, nullptr, S(stream));
        launch_kll(*m, nu, H, f, S(stream));
    });
}

lfem_status lfem_reference_table(int dim, int order, int quad_points, int *q_out, int *k_out,
                                 double *w, double *xi, double *phi, double *dphi)
{
    return guarded([&] {
        LFEM_REQUIRE(q_out && k_out, LFEM_EINVAL, "null q_out or k_out");
        LFEM_REQUIRE(dim >= 1 && dim <= 3 && order >= 1 && order <= 4, LFEM_EUNSUPPORTED,
                     "no element of that dimension and order");
        RefTable tab;
        LFEM_REQUIRE(build_ref_table(dim, order, quad_points, tab), LFEM_EUNSUPPORTED,
                     "no quadrature rule with that number of points for this simplex");
        *q_out = tab.Q;
        *k_out = tab.k;
        const int d = dim, k = tab.k;
        for (int q = 0; q < tab.Q; ++q) {
            const double *t = tab.data.data() + static_cast<size_t>(q) * tab.stride;
            if (w) w[q] = t[0];
            for (int m = 0; m < d; ++m)
                if (xi) xi[q * d + m] = t[1 + m];
            for (int a = 0; a < k; ++a) {
                if (phi) phi[q * k + a] = t[1 + d + a];
                for (int m = 0; m < d; ++m)
                    if (dphi) dphi[(q * k + a) * d + m] = t[1 + d + k + a * d + m];
            }
        }
    });
}

lfem_status lfem_status_get(lfem_mesh_t m, int64_t *n_degenerate)
{
    return guarded([&] {
        LFEM_REQUIRE(m && n_degenerate, LFEM_EINVAL, "null argument");
        unsigned long long v = 0;
        LFEM_HIP(hipDeviceSynchronize());
        LFEM_HIP(hipMemcpy(&v, m->degenerate, sizeof(v), hipMemcpyDeviceToHost));
        *n_degenerate = static_cast<int64_t>(v);
    });
}

lfem_status lfem_status_reset(lfem_mesh_t m, void *stream)
{
    return guarded([&] {
        LFEM_REQUIRE(m, LFEM_EINVAL, "null mesh");
        LFEM_HIP(hipMemsetAsync(m->degenerate, 0, sizeof(unsigned long long), S(stream)));
    });
}

void lfem_mesh_destroy(lfem_mesh_t m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();
    release_mesh(*m);
    delete m;
}

void lfem_pattern_destroy(lfem_pattern_t p)
{
    if (!p) return;
    (void)hipDeviceSynchronize();
    release_pattern(*p);
    delete p;
}

void lfem_batch_destroy(lfem_batch_t b)
{
    if (!b) return;
    batch_destroy(b);
}

}  // extern "C"
