// Batched assembly of many meshes of uneven size, replayed from one HIP graph.
//
// Meshes of the persistent kernel's family (curves, surfaces and planar meshes
// of order 1 or 2 under their default rules, whose patterns carry a side-slot
// block schedule, assembling plain M and A) share one persistent launch: every
// (mesh, row block) pair is a work item, items are sorted by cost (block
// element count, largest first), and a grid of as many workgroups as fit on
// the device at once pulls items from an atomic counter, so large and small
// meshes share the machine without a launch per mesh.  Their per-mesh
// arguments (output and coordinate pointers included) live in a device
// descriptor table rewritten only when those pointers change.
//
// Every other member (nodal coefficients, the weighted mass, the high-order
// rules, orders 3 and 4, tetrahedra) is assembled by its own numeric launch
// with its pattern's tuned scatter, recorded into the same graph after the
// persistent kernel.  The graph is captured again when an output, coordinate
// or staging pointer of such a member changes.  One replay assembles the
// whole batch.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "side.hpp"

struct lfem_batch_s {
    int n = 0;
    unsigned what = 0;
    int nmat = 0;
    std::vector<lfem::Mesh *> meshes;
    std::vector<lfem::Pattern *> pats;
    std::vector<const double *> coef_a, coef_c;  // per mesh, null for none
    std::vector<char> fast;                      // assembled by the persistent kernel
    int nfast = 0;
    // persistent kernel
    std::vector<lfem::BlockArgs> host_desc;
    lfem::BlockArgs *pinned = nullptr;  // staging for descriptor uploads
    lfem::BlockArgs *desc = nullptr;    // device descriptors
    int2 *items = nullptr;              // device work items (mesh, block)
    int n_items = 0;
    int *counter = nullptr;
    size_t lds = 0;
    int dump = 0;  // first LDS dump entry (= largest block capacity)
    int rs = 0;    // doubles of one LDS matrix region
    int grid = 0;
    hipEvent_t upload_done = nullptr;
    bool uploaded = false;
    std::vector<double *> last_vals;
    std::vector<const double *> last_coords;
    std::vector<uint64_t> gens;  // schedule generation of each pattern at prepare()
    int cap = 0;
    // the graph and the pointers its per-member launches were captured with
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
    std::vector<double *> cap_vals;
    std::vector<const double *> cap_coords;
    std::vector<const double *> cap_stage, cap_dstage;
};

namespace lfem {

namespace {

constexpr int BATCH_NT = kSideThreads;

// one work item; thread 0 claims the workgroup's next item once this item's
// loads are issued, so the claim's round trip overlaps the item's compute
template <class E, int NM, bool HA>
__device__ __forceinline__ void batch_item(const BlockArgs &g, int blk, double *lds, int dump, int rs,
                                           int *__restrict__ counter, int &next)
{
    constexpr int QA = E::d == 1 ? 2 : 3, QB = E::d == 1 ? 3 : 6;
    SideBlock<E> s;
    side_load_rec<E>(g, blk, s);
    side_load_first<E, true>(g, s);
    side_load_coords<E>(g, s);
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    if (g.Q == QA) side_block<E, QA, NM, HA, 0, BATCH_NT>(g, s, lds, dump, rs);
    else side_block<E, QB, NM, HA, 0, BATCH_NT>(g, s, lds, dump, rs);
}

// LDS: one region of rs doubles per matrix: value entries up to the largest
// block capacity of the batch (`dump`), then the dump entries
template <int NM, bool HA>
__global__ __launch_bounds__(BATCH_NT) void k_batch(const BlockArgs *__restrict__ desc,
                                                    const int2 *__restrict__ items, int n_items,
                                                    int *__restrict__ counter, int dump, int rs)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    extern __shared__ double lds[];
    __shared__ int cur;
    for (int i = threadIdx.x; i < NMAT * rs; i += BATCH_NT) lds[i] = 0.0;
    int next = 0;  // thread 0: the claimed next item
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    for (;;) {
        if (threadIdx.x == 0) cur = next;
        __syncthreads();
        const int it = cur;
        __syncthreads();
        // uniform: every workgroup leaves once its claim is past the list (each
        // item below n_items is claimed once and processed by its claimer)
        if (it >= n_items) break;
        const int2 w = items[it];
        const BlockArgs g = desc[w.x];
        switch (g.etype) {
        case S1P1: batch_item<ET<1, 1, 1>, NM, HA>(g, w.y, lds, dump, rs, counter, next); break;
        case S1P2: batch_item<ET<1, 1, 2>, NM, HA>(g, w.y, lds, dump, rs, counter, next); break;
        case S2P1: batch_item<ET<1, 2, 1>, NM, HA>(g, w.y, lds, dump, rs, counter, next); break;
        case S2P2: batch_item<ET<1, 2, 2>, NM, HA>(g, w.y, lds, dump, rs, counter, next); break;
        case B2P1: batch_item<ET<0, 2, 1>, NM, HA>(g, w.y, lds, dump, rs, counter, next); break;
        case B2P2: batch_item<ET<0, 2, 2>, NM, HA>(g, w.y, lds, dump, rs, counter, next); break;
        default:
            if (threadIdx.x == 0) next = atomicAdd(counter, 1);
            break;
        }
    }
}

__global__ void k_zero_int(int *p) { *p = 0; }

using BatchKernel = void (*)(const BlockArgs *, const int2 *, int, int *, int, int);

BatchKernel pick_kernel(unsigned what)
{
    if (what == LFEM_M) return k_batch<1, false>;
    if (what == LFEM_A) return k_batch<0, true>;
    return k_batch<1, true>;
}

// a mesh the persistent kernel runs: orders 1 and 2 of curves, surfaces and
// planar meshes under the two default rules of each dimension, with a
// side-slot block schedule
bool batch_eligible(const Mesh &m, const Pattern &p)
{
    const bool rule_ok = m.Q == (m.d == 1 ? 2 : 3) || m.Q == (m.d == 1 ? 3 : 6);
    return m.d <= 2 && m.p <= 2 && rule_ok && (m.T == 0 || (p.sched.nb > 0 && p.sched.side_mode));
}

void release_graph(lfem_batch_s &b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.captured = false;
}

// (re)build the persistent kernel's descriptors, work list and launch shape
// over the members it runs; drops the graph (captured again before the next
// replay)
void prepare(lfem_batch_s &b)
{
    release_graph(b);
    dev_free(b.desc);
    dev_free(b.items);
    b.desc = nullptr;
    b.items = nullptr;
    b.host_desc.clear();
    b.n_items = 0;
    b.uploaded = false;
    b.last_vals.clear();
    b.last_coords.clear();
    b.gens.resize(b.n);
    for (int i = 0; i < b.n; ++i) b.gens[i] = b.pats[i]->sched_gen;
    if (b.nfast == 0) return;
    std::vector<std::pair<int, int2>> work;  // (cost, item)
    int max_cap = 1, max_row = 0;
    for (int i = 0; i < b.n; ++i) {
        Mesh &m = *b.meshes[i];
        Pattern &p = *b.pats[i];
        b.host_desc.push_back(b.fast[i] ? block_args(m, p, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr)
                                        : BlockArgs{});
        if (!b.fast[i] || m.T == 0) continue;
        max_cap = std::max(max_cap, p.sched.cap);
        max_row = std::max(max_row, p.max_row);
        std::vector<int32_t> ep(p.sched.nb + 1);
        LFEM_HIP(hipMemcpy(ep.data(), p.sched.elem_ptr, ep.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost));
        for (int blk = 0; blk < p.sched.nb; ++blk)
            work.push_back({ep[blk + 1] - ep[blk], make_int2(i, blk)});
    }
    // value entries of the largest block capacity, then the dump entries
    b.dump = max_cap;
    b.rs = side_region(max_cap, max_row);
    const size_t lds = side_lds_bytes(b.nmat, max_cap, max_row);
    LFEM_REQUIRE(lds <= 160 * 1024, LFEM_EUNSUPPORTED, "batch block schedule exceeds LDS");
    std::stable_sort(work.begin(), work.end(),
                     [](const std::pair<int, int2> &x, const std::pair<int, int2> &y) {
                         return x.first > y.first;
                     });
    std::vector<int2> items;
    items.reserve(work.size());
    for (auto &w : work) items.push_back(w.second);
    b.n_items = static_cast<int>(items.size());
    b.lds = lds;
    LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&b.desc), sizeof(BlockArgs) * b.n));
    LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&b.items), sizeof(int2) * std::max(1, b.n_items)));
    if (!items.empty())
        LFEM_HIP(hipMemcpy(b.items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
    BatchKernel kern = pick_kernel(b.what);
    if (b.lds > 64 * 1024)
        LFEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(b.lds)));
    int per_cu = 0, dev = 0;
    LFEM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    LFEM_HIP(hipGetDeviceProperties(&prop, dev));
    LFEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern),
                                                          BATCH_NT, b.lds));
    LFEM_REQUIRE(per_cu > 0, LFEM_EUNSUPPORTED, "batch kernel does not fit on a compute unit");
    b.grid = std::max(1, std::min(per_cu * prop.multiProcessorCount, std::max(1, b.n_items)));
}

// numeric launch arguments of member i writing into vals[i * nmat ...]
// (ordered M, A, MC)
NumericOut member_out(const lfem_batch_s &b, int i, double *const *vals)
{
    NumericOut o;
    o.what = b.what;
    o.coef_a = b.coef_a[i];
    o.coef_c = b.coef_c[i];
    double *const *v = vals + static_cast<size_t>(i) * b.nmat;
    int j = 0;
    if (b.what & LFEM_M) o.vals_m = v[j++];
    if (b.what & LFEM_A) o.vals_a = v[j++];
    if (b.what & LFEM_MC) o.vals_mc = v[j++];
    return o;
}

// the scatter a member is launched with: its pattern's tuned variant (staged
// when it has no block schedule)
int member_variant(const lfem_batch_s &b, int i)
{
    const Pattern &p = *b.pats[i];
    int v = p.tuned_variant;
    if (v == LFEM_SCATTER_BLOCKED && p.sched.nb == 0 && b.meshes[i]->T > 0) v = LFEM_SCATTER_STAGED;
    return v;
}

// one launch of every member outside the persistent kernel, on scratch
// outputs, outside any capture: builds the structures a launch creates on
// first use (contribution lists, staging buffer), which must not be
// allocated while the graph is being captured (SYNCHRONISES s)
void warm_members(lfem_batch_s &b, hipStream_t s)
{
    std::vector<double *> scratch;
    try {
        for (int i = 0; i < b.n; ++i) {
            if (b.fast[i] || b.meshes[i]->T == 0) continue;
            std::vector<double *> all(static_cast<size_t>(b.n) * b.nmat, nullptr);
            for (int j = 0; j < b.nmat; ++j) {
                double *v = nullptr;
                LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&v), std::max<int64_t>(b.pats[i]->nnz, 1) * 8));
                scratch.push_back(v);
                all[static_cast<size_t>(i) * b.nmat + j] = v;
            }
            launch_numeric(*b.meshes[i], *b.pats[i], member_out(b, i, all.data()), member_variant(b, i), s);
        }
        LFEM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        for (double *v : scratch) dev_free(v);
        throw;
    }
    for (double *v : scratch) dev_free(v);
}

// capture the graph: counter reset (a kernel, not a memset node) and the
// persistent kernel, then, unless fast_only, one numeric launch per other
// member with the given outputs and its current coordinates
void capture_graph(lfem_batch_s &b, double *const *vals, bool fast_only)
{
    release_graph(b);
    LFEM_HIP(hipStreamBeginCapture(b.capture, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
        if (b.nfast > 0) {
            k_zero_int<<<1, 1, 0, b.capture>>>(b.counter);
            pick_kernel(b.what)<<<b.grid, BATCH_NT, b.lds, b.capture>>>(b.desc, b.items, b.n_items, b.counter,
                                                                        b.dump, b.rs);
            LFEM_HIP(hipGetLastError());
        }
        if (!fast_only)
            for (int i = 0; i < b.n; ++i)
                if (!b.fast[i])
                    launch_numeric(*b.meshes[i], *b.pats[i], member_out(b, i, vals), member_variant(b, i),
                                   b.capture);
    } catch (...) {
        (void)hipStreamEndCapture(b.capture, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    LFEM_HIP(hipStreamEndCapture(b.capture, &g));
    b.graph = g;
    LFEM_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    if (fast_only) return;
    b.captured = true;
    b.cap_vals.assign(vals, vals + static_cast<size_t>(b.n) * b.nmat);
    b.cap_coords.resize(b.n);
    b.cap_stage.resize(b.n);
    b.cap_dstage.resize(b.n);
    for (int i = 0; i < b.n; ++i) {
        b.cap_coords[i] = b.meshes[i]->coords;
        b.cap_stage[i] = b.pats[i]->stage;
        b.cap_dstage[i] = b.pats[i]->dstage;
    }
}

// true when the graph must be captured again: none yet, or an output,
// coordinate or staging-buffer pointer of a member outside the persistent
// kernel differs from the captured one (another assembly on the same
// pattern may have reallocated its staging buffers)
bool members_moved(const lfem_batch_s &b, double *const *vals)
{
    if (!b.captured) return true;
    for (int i = 0; i < b.n; ++i) {
        if (b.fast[i]) continue;
        if (b.meshes[i]->coords != b.cap_coords[i] || b.pats[i]->stage != b.cap_stage[i] ||
            b.pats[i]->dstage != b.cap_dstage[i])
            return true;
        for (int j = 0; j < b.nmat; ++j) {
            const size_t k = static_cast<size_t>(i) * b.nmat + j;
            if (vals[k] != b.cap_vals[k]) return true;
        }
    }
    return false;
}

// The descriptor table holds the output pointers and each mesh's current
// coordinate pointer (lfem_mesh_set_coords may have moved it); it is rewritten
// when either set differs from the last upload.
void upload_descriptors(lfem_batch_s &b, double *const *vals, hipStream_t s)
{
    if (b.nfast == 0) return;
    std::vector<double *> cur(vals, vals + static_cast<size_t>(b.n) * b.nmat);
    std::vector<const double *> xs(b.n);
    for (int i = 0; i < b.n; ++i) xs[i] = b.meshes[i]->coords;
    if (b.uploaded && cur == b.last_vals && xs == b.last_coords) return;
    // the staging buffer may still feed the previous upload
    if (b.uploaded) LFEM_HIP(hipEventSynchronize(b.upload_done));
    for (int i = 0; i < b.n; ++i) {
        BlockArgs g = b.host_desc[i];
        g.coords = xs[i];
        g.v[0] = g.v[1] = g.v[2] = nullptr;
        for (int j = 0; j < b.nmat; ++j) g.v[j] = cur[static_cast<size_t>(i) * b.nmat + j];
        b.pinned[i] = g;
    }
    LFEM_HIP(hipMemcpyAsync(b.desc, b.pinned, sizeof(BlockArgs) * b.n, hipMemcpyHostToDevice, s));
    LFEM_HIP(hipEventRecord(b.upload_done, s));
    b.last_vals = cur;
    b.last_coords = xs;
    b.uploaded = true;
}

float time_batch(lfem_batch_s &b, const std::vector<double *> &vals, hipStream_t s)
{
    hipEvent_t e0, e1;
    LFEM_HIP(hipEventCreate(&e0));
    LFEM_HIP(hipEventCreate(&e1));
    upload_descriptors(b, vals.data(), s);
    capture_graph(b, vals.data(), true);
    LFEM_HIP(hipGraphLaunch(b.exec, s));
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
        LFEM_HIP(hipEventRecord(e0, s));
        LFEM_HIP(hipGraphLaunch(b.exec, s));
        LFEM_HIP(hipEventRecord(e1, s));
        LFEM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        LFEM_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

void rebuild_all(lfem_batch_s &b, int cap, hipStream_t s)
{
    for (int i = 0; i < b.n; ++i)
        if (b.fast[i] && b.meshes[i]->T > 0) build_schedule(*b.meshes[i], *b.pats[i], std::max(cap, b.pats[i]->max_row), kBlockMaxRows, s);
}

void autotune_batch(lfem_batch_s &b, hipStream_t s)
{
    const char *env = std::getenv("LFEM_TUNE_VERBOSE");
    const bool verbose = env && env[0] == '1';
    std::vector<double *> vals(static_cast<size_t>(b.n) * b.nmat, nullptr);
    std::vector<double *> owned;
    for (int i = 0; i < b.n; ++i)
        for (int j = 0; j < b.nmat && b.fast[i]; ++j) {
            double *v = nullptr;
            LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&v), std::max<int64_t>(b.pats[i]->nnz, 1) * 8));
            owned.push_back(v);
            vals[static_cast<size_t>(i) * b.nmat + j] = v;
        }
    float best = 1e30f;
    int best_cap = 4096;
    try {
        const int caps[] = {2048, 3072, 4096, 4864, 4992};
        for (int cap : caps) {
            rebuild_all(b, cap, s);
            bool ok = true;
            for (int i = 0; i < b.n; ++i) ok = ok && (!b.fast[i] || batch_eligible(*b.meshes[i], *b.pats[i]));
            if (!ok) continue;
            prepare(b);
            const float t = time_batch(b, vals, s);
            if (verbose) std::fprintf(stderr, "[lfem tune] batch cap %d: %.1f us\n", cap, t * 1e3);
            if (t < best) {
                best = t;
                best_cap = cap;
            }
        }
    } catch (...) {
        for (double *v : owned) dev_free(v);
        throw;
    }
    LFEM_HIP(hipStreamSynchronize(s));
    for (double *v : owned) dev_free(v);
    rebuild_all(b, best_cap, s);
    b.cap = best_cap;
}

}  // namespace

void batch_destroy(lfem_batch_t b);

lfem_status batch_create(int n, Mesh *const *meshes, Pattern *const *pats, unsigned what,
                         const double *const *coef_a, const double *const *coef_c, int autotune,
                         hipStream_t s, lfem_batch_t *out)
{
    LFEM_REQUIRE(what != 0 && (what & ~(LFEM_M | LFEM_A | LFEM_MC)) == 0, LFEM_EINVAL,
                 "what must be a non-empty combination of LFEM_M, LFEM_A, LFEM_MC");
    auto *b = new lfem_batch_s();
    try {
        b->n = n;
        b->what = what;
        b->nmat = (what & LFEM_M ? 1 : 0) + (what & LFEM_A ? 1 : 0) + (what & LFEM_MC ? 1 : 0);
        b->meshes.assign(meshes, meshes + n);
        b->pats.assign(pats, pats + n);
        b->coef_a.assign(n, nullptr);
        b->coef_c.assign(n, nullptr);
        b->fast.assign(n, 0);
        for (int i = 0; i < n; ++i) {
            if (coef_a) b->coef_a[i] = coef_a[i];
            if (coef_c) b->coef_c[i] = coef_c[i];
            LFEM_REQUIRE(!(what & LFEM_MC) || b->coef_c[i] || pats[i]->nnz == 0, LFEM_EINVAL,
                         "the weighted mass needs a nodal coefficient for every mesh");
            b->fast[i] = batch_eligible(*meshes[i], *pats[i]) && !b->coef_a[i] && !(what & LFEM_MC);
            b->nfast += b->fast[i];
        }
        LFEM_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        LFEM_HIP(hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming));
        LFEM_HIP(hipMalloc(reinterpret_cast<void **>(&b->counter), sizeof(int)));
        LFEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&b->pinned), sizeof(BlockArgs) * n,
                               hipHostMallocDefault));
        if (autotune && b->nfast > 0) autotune_batch(*b, s);
        prepare(*b);
        warm_members(*b, s);
    } catch (...) {
        batch_destroy(b);
        throw;
    }
    *out = b;
    return LFEM_OK;
}

void batch_run(lfem_batch_t b, double *const *vals, hipStream_t s)
{
    for (int i = 0; i < b->n; ++i)
        for (int j = 0; j < b->nmat; ++j)
            LFEM_REQUIRE(vals[static_cast<size_t>(i) * b->nmat + j] || b->pats[i]->nnz == 0,
                         LFEM_EINVAL, "null output in batch");
    // a pattern whose block schedule was rebuilt since the batch was set up
    // (lfem_pattern_autotune, another batch's tuning) has freed the schedule the
    // graph and descriptors point at: wait for earlier replays, then rebuild
    // the work list, descriptors and graph from the current schedules
    bool stale = false;
    for (int i = 0; i < b->n; ++i) stale = stale || b->pats[i]->sched_gen != b->gens[i];
    if (stale) {
        LFEM_HIP(hipStreamSynchronize(s));
        // a member rescheduled into a form the persistent kernel does not run
        // (staged only) gets a launch of its own
        for (int i = 0; i < b->n; ++i)
            if (b->fast[i] && !batch_eligible(*b->meshes[i], *b->pats[i])) {
                b->fast[i] = 0;
                --b->nfast;
            }
        prepare(*b);
        warm_members(*b, s);
    }
    upload_descriptors(*b, vals, s);
    if (members_moved(*b, vals)) {
        // earlier replays of the graph being replaced may still run
        LFEM_HIP(hipStreamSynchronize(s));
        capture_graph(*b, vals, false);
    }
    LFEM_HIP(hipGraphLaunch(b->exec, s));
}

void batch_debug_check(lfem_batch_t b, hipStream_t s)
{
    for (int i = 0; i < b->n; ++i) debug_check(*b->meshes[i], b->pats[i], s);
}

void batch_destroy(lfem_batch_t b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    release_graph(*b);
    dev_free(b->desc);
    dev_free(b->items);
    dev_free(b->counter);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->upload_done) (void)hipEventDestroy(b->upload_done);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

}  // namespace lfem
