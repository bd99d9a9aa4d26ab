// Internal declarations shared by the translation units of liblfem.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lfem.h"

namespace lfem {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
void clear_error();

struct Error {
    lfem_status code;
    std::string msg;
};

#define LFEM_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::lfem::Error{e_ == hipErrorOutOfMemory ? LFEM_ENOMEM : LFEM_EHIP,     \
                                std::string(#call) + ": " + hipGetErrorString(e_)};      \
    } while (0)

inline void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

#define LFEM_REQUIRE(cond, code, msg)                                                    \
    do {                                                                                 \
        if (!(cond)) throw ::lfem::Error{(code), (msg)};                                 \
    } while (0)

// ---------------------------------------------------------------------------
// element types: (surface?, manifold dimension d, order p)
// ---------------------------------------------------------------------------
// orders 3 and 4 (segments, triangles, then tetrahedra) follow the eight
// original types
enum EType : int {
    S1P1 = 0, S1P2, S2P1, S2P2, B2P1, B2P2, B3P1, B3P2,
    S1P3, S1P4, S2P3, S2P4, B2P3, B2P4, B3P3, B3P4, NUM_ETYPES
};

inline int etype_of(int domain, int d, int p)
{
    if (p < 1 || p > 4) return -1;
    if (p <= 2) {
        if (domain == LFEM_SURFACE && d == 1) return p == 1 ? S1P1 : S1P2;
        if (domain == LFEM_SURFACE && d == 2) return p == 1 ? S2P1 : S2P2;
        if (domain == LFEM_BULK && d == 2) return p == 1 ? B2P1 : B2P2;
        if (domain == LFEM_BULK && d == 3) return p == 1 ? B3P1 : B3P2;
        return -1;
    }
    if (domain == LFEM_SURFACE && d == 1) return p == 3 ? S1P3 : S1P4;
    if (domain == LFEM_SURFACE && d == 2) return p == 3 ? S2P3 : S2P4;
    if (domain == LFEM_BULK && d == 2) return p == 3 ? B2P3 : B2P4;
    if (domain == LFEM_BULK && d == 3) return p == 3 ? B3P3 : B3P4;
    return -1;
}

// largest element (quartic tetrahedron); elements of up to kMaxNodes8 nodes
// keep a byte slot map (rows of at most 255 entries), larger ones a 16-bit
// map (rows of at most kMaxRowWide entries)
constexpr int kMaxNodes = 35;
constexpr int kMaxNodes8 = 15;
constexpr int kMaxRowWide = 1023;
// contributions of one CSR value loaded at once by the staged reduction; the
// values with longer lists (diagonals of well-connected nodes) are summed by
// a second, small launch so that the main one needs a single round of loads
constexpr int kReduceBatch = 8;
constexpr int kMaxSlotWords = (kMaxNodes8 * kMaxNodes8 + 3) / 4;

// nodes of the order-p Lagrange element: (p + d choose d)
inline int nodes_per_elem(int d, int p)
{
    return d == 1 ? p + 1 : (d == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6);
}

// Reference data per quadrature point q, `stride` doubles each:
//   [0]                         weight w_q (weights sum to the reference measure)
//   [1, 1+d)                    the point xi_q
//   [1+d, 1+d+k)                phi_a(xi_q)
//   [1+d+k, 1+d+k+k*d)          d phi_a / d xi_m at xi_q, index a*d + m
//   [1+d+k+k*d, ... + np)       phi_a phi_b for the np = k(k+1)/2 pairs a <= b
//                               (upper triangle, row-major)
//   [..., ... + np*nsym)        reference stiffness tensor R[p][s] over the
//                               nsym = d(d+1)/2 slots m <= n of a symmetric d x d K
struct RefTable {
    int Q = 0, k = 0, d = 0, stride = 0;
    std::vector<double> data;
    // pair-major copy of the reference tensors: for each pair p (a <= b) the Q values
    // phi_a phi_b (xi_q), then the Q*nsym values R[q][p][s]
    int pstride = 0;
    std::vector<double> pairs;
};

// Builds the table of element type (d, p) with the rule of `npts` points
// (0 = default).  Returns false if the rule does not exist.
bool build_ref_table(int d, int p, int npts, RefTable &out);
int default_rule(int d, int p);

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct Mesh {
    int domain = 0, d = 0, p = 0, namb = 0, k = 0, etype = -1, Q = 0, tab_stride = 0;
    int64_t N = 0, T = 0;
    const double *coords = nullptr;
    const int32_t *conn = nullptr;
    int device = 0;
    double *tab = nullptr;           // device reference table
    double *tabp = nullptr;          // device pair-major reference tensors
    RefTable host_tab;
    int32_t *ne_ptr = nullptr;       // [N+1] node -> incidence offsets
    int32_t *ne = nullptr;           // [k*T] incidences a*T + e (position in conn), ascending per node
    int32_t *flags = nullptr;        // [4] device flags: [0] bad index, [1] repeated node
    unsigned long long *degenerate = nullptr;
    double *scratch = nullptr;       // adjoint staging, grown on demand
    size_t scratch_bytes = 0;
};

struct BlockSchedule {
    int cap = 0;          // max CSR values per block and matrix (LDS capacity)
    int nb = 0;           // number of blocks
    int max_rows = 0;     // max rows in one block
    int max_elems = 0;    // max elements in one block
    int max_colors = 0;   // colours used inside one block
    int nthreads = 256;
    double halo = 0.0;    // sum of block element counts / T
    int64_t len = 0;      // total length of the block element lists
    int32_t *row_begin = nullptr;  // [nb+1]
    int32_t *elem_ptr = nullptr;   // [nb+1] list offsets; lists sorted by colour, then element
    uint8_t *colors = nullptr;     // [len] colour of each list entry
    int32_t *bconn = nullptr;      // [k][len] node ids of each list entry
    uint8_t *boff = nullptr;       // [len][kkp] slot offsets of each list entry
    int mw = 0;                    // mask words per list entry
    uint32_t *bmask = nullptr;     // [len][mw] bit a*k+b: target entry has >= 3 contributions
    bool diag_only = false;        // only diagonal entries have >= 3 contributions
    bool side_mode = false;        // ordered entries summed from LDS side slots (no colours)
    int max_side = 0;              // side slots in the largest block
    int max_ord = 0;               // ordered entries in the largest block
    // side mode: per list entry and node a, (row start of node a inside the
    // block, 0xffff if the row is outside) | (side slot of contribution (a, a),
    // 0xffff: none) << 16
    uint32_t *bnode = nullptr;     // [len][k]
    uint32_t *bord = nullptr;      // per ordered entry: (LDS index | count << 16, first slot)
    int32_t *bord_ptr = nullptr;   // [nb+1] offsets into bord (in records)
    // side mode: per block {e0, e1, r0, r1, first CSR value, values, o0, o1}
    // (element list range, row range, value range, ordered-entry range)
    int32_t *brec = nullptr;       // [nb][8]
};

// threads of a side-slot workgroup; side-mode blocks hold at most
// kSideThreads elements for P2 and four times as many for P1
constexpr int kSideThreads = 256;

struct Pattern {
    Mesh *mesh = nullptr;
    int64_t nnz = 0;
    int32_t *row_ptr = nullptr;
    int32_t *col_idx = nullptr;
    uint8_t *off8 = nullptr;   // [T][kkp] column offset of (a,b) in row conn[a] (k <= kMaxNodes8)
    uint16_t *off16 = nullptr; // [T][k*k] the same, 16 bits (k > kMaxNodes8)
    int kkp = 0;               // bytes per element (k*k rounded up to 4)
    int max_row = 0;
    // staged scatter (built on first use)
    int32_t *cptr = nullptr;   // [nnz+1]
    int32_t *clist = nullptr;  // [k*k*T] contributions e*k*k + a*k + b, ascending per slot
    int32_t *long_slots = nullptr;  // [nlong] slots with more than kReduceBatch contributions, ascending
    int64_t nlong = 0;
    double *stage = nullptr;
    size_t stage_bytes = 0;
    // the vertices' diagonal values of every element, [d + 1][T][NMAT] (orders
    // 1 and 2): the long lists read these instead of the full records
    double *dstage = nullptr;
    size_t dstage_bytes = 0;
    // blocked scatter
    BlockSchedule sched;
    uint64_t sched_gen = 0;    // incremented by every schedule (re)build
    // host copies kept for rebuilding the schedule
    std::vector<int32_t> h_row_ptr, h_ne_ptr, h_ne, h_conn;
    int tuned_variant = LFEM_SCATTER_BLOCKED;
};

// most rows of one block (row offsets are staged in LDS; the side-slot kernels
// hold (kBlockMaxRows + 1) / nthreads of them per thread)
constexpr int kBlockMaxRows = 1024;
// default values per block and matrix of the blocked scatter: the largest
// capacity up to kBlockCapDefault at which two M + A workgroups of the
// side-slot kernel (2 x (cap + dump entries) doubles each) fit in one CU's
// 160 KB of LDS.  On the 655,360-element P2 ellipsoid 4992 leaves fewer
// blocks than seven rounds of 512 workgroups take (3550), where 4864 left
// 13 blocks for an eighth round (about 2 % slower).
constexpr int kBlockCapDefault = 4992;
constexpr int kTwoGroupLdsDoubles = 160 * 1024 / 2 / 2 / 8;  // per matrix
int default_block_cap(int max_row);

// ---------------------------------------------------------------------------
// symbolic phase (symbolic.hip)
// ---------------------------------------------------------------------------
void build_incidence(Mesh &m, hipStream_t s);
void build_pattern(Mesh &m, Pattern &p, hipStream_t s);
void build_staged(Mesh &m, Pattern &p, hipStream_t s);
void build_schedule(Mesh &m, Pattern &p, int cap, int max_rows, hipStream_t s);
void free_schedule(BlockSchedule &b);
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *d_total,
                        hipStream_t s);

// ---------------------------------------------------------------------------
// numeric phase (numeric.hip)
// ---------------------------------------------------------------------------
struct NumericOut {
    unsigned what = 0;
    const double *coef_a = nullptr;
    const double *coef_c = nullptr;
    double *vals_m = nullptr, *vals_a = nullptr, *vals_mc = nullptr;
};
void launch_numeric(Mesh &m, Pattern &p, const NumericOut &o, int variant, hipStream_t s);
// debug mode (debug.hip): validate the connectivity (and, with a pattern,
// its slot maps) before a launch; throws LFEM_EINVAL, synchronises s
void debug_check(const Mesh &m, const Pattern *p, hipStream_t s);
int set_debug(int on);
// per element family (numeric_<family>.hip)
void numeric_curve(Mesh &m, Pattern &p, const NumericOut &o, int variant, hipStream_t s);
void numeric_surface(Mesh &m, Pattern &p, const NumericOut &o, int variant, hipStream_t s);
void numeric_planar(Mesh &m, Pattern &p, const NumericOut &o, int variant, hipStream_t s);
void numeric_tet(Mesh &m, Pattern &p, const NumericOut &o, int variant, hipStream_t s);
void fill_zero(double *x, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// adjoint (adjoint.hip)
// ---------------------------------------------------------------------------
void launch_energy(Mesh &m, const double *u, const double *v, double alpha, const double *w,
                   const double *z, double beta, double *J, hipStream_t s);
void launch_shape_grad(Mesh &m, const double *u, const double *v, double alpha,
                       const double *w, const double *z, double beta, double *grad,
                       hipStream_t s);
void launch_shape_grad_noalloc(Mesh &m, const double *u, const double *v, double alpha, const double *w,
                               const double *z, double beta, double *grad, hipStream_t s);
double *mesh_scratch(Mesh &m, size_t bytes);
void launch_load(Mesh &m, const double *f, double *b, hipStream_t s);
void launch_kll(Mesh &m, const double *nu, const double *H, double *f, hipStream_t s);
void launch_spmv(const Pattern &p, const double *vals, const double *x, double alpha, double *y, int nvec,
                 hipStream_t s);
void launch_dziuk(Mesh &m, Pattern &p, double tau, const double *x, double *vals_m, double *vals_a,
                  double *vals_s, double *rhs, int variant, hipStream_t s);
void launch_kll_system(Mesh &m, Pattern &p, double tau, double delta0, const double *nu, const double *H,
                       const double *hist, double *vals_m, double *vals_a, double *vals_s, double *f, double *rhs,
                       int variant, hipStream_t s);

}  // namespace lfem
