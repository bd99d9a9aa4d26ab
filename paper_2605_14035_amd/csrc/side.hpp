// Side-slot form of the blocked scatter (curves, surfaces and planar meshes:
// every CSR entry that receives three or more contributions is a diagonal).
//
// Per element the geometry is evaluated once per quadrature point (Jacobian,
// measure, inverse metric K = (J^T J)^{-1}, section 3.3) and kept as Q-point
// data: the weighted measure f_q = w_q mu_q c_h(xi_q) of each mass-class
// output and the scaled inverse metric w_q mu_q a_h(xi_q) K_q of the stiffness
// output.  The local matrices of section 3.4 are then formed one pair (a, b),
// a <= b, at a time from the pair-major reference tensors,
//     M_ab = sum_q f_q phi_a phi_b (xi_q),   A_ab = sum_q sum_s K'_{q,s} R_{ab,q,s},
// and each value goes to LDS as soon as it is known, so no local matrix is
// held in registers.
//
// Determinism: LDS starts at +0 and an entry with at most two contributions
// gets the same bits in either order (0 + a = a, a + b = b + a), so those are
// added by all threads at once; a diagonal contribution to an entry with more
// contributions is stored in its own side slot and the slots of one entry are
// summed in element order after a barrier.
//
// LDS of one block: one region of `rs` doubles per matrix (entry e of matrix
// m at lds[m * rs + e]); in each region, entries [0, cap) hold the block's
// values followed by its side slots, and `dump` entries from index `dump` on
// take the contributions to rows outside the block (one per lane and column
// offset, never read), so the scatter needs no branch.  (Separate regions
// spread one matrix's scattered 8-byte adds over all LDS banks.)  Value
// entries are all zero between blocks: the ordered reduction clears the side
// slots it reads and the write-out clears the values it stores, so no
// separate clearing pass runs per block.
//
// Memory latency dominates a block's life, so its dependent loads are kept
// short: one scalar load of the block record (element, row, value and
// ordered-entry ranges), then per thread its element's schedule words (node
// ids, column offsets, node words: row start in the block and side slot) and
// its ordered-entry record, then the coordinates.  No row offsets are staged
// and the compute starts without a barrier.  The single-mesh kernel is
// persistent (each workgroup walks a fixed sequence of blocks, all in the
// range of its XCD) and loads the next block's record before it starts on
// the current block.
#pragma once

#include <type_traits>

#include "blocked.hpp"

namespace lfem {

template <class E>
struct SideLayout {
    static constexpr int KKP = (E::k * E::k + 3) / 4 * 4;  // slot-offset bytes per element
    static constexpr int KW = KKP / 4;                     // ... as 32-bit words
};

using cint32 = const __attribute__((address_space(4))) int32_t;

// one block: its record (uniform) and this thread's first element and first
// ordered-entry record
template <class E>
struct SideBlock {
    int32_t blk, e0, e1, r0, r1, base, nloc, o0, o1;
    int32_t nid[E::k];
    uint32_t ow[SideLayout<E>::KW];
    uint32_t nw[E::k];
    double x[E::n][E::k];
    uint32_t ord0, ord1;
};

// block record (scalar loads)
template <class E>
__device__ __forceinline__ void side_load_rec(const BlockArgs &g, int blk, SideBlock<E> &s)
{
    cint32 *r = (cint32 *)(g.brec) + 8 * static_cast<int64_t>(blk);
    s.blk = blk;
    s.e0 = r[0];
    s.e1 = r[1];
    s.r0 = r[2];
    s.r1 = r[3];
    s.base = r[4];
    s.nloc = r[5];
    s.o0 = r[6];
    s.o1 = r[7];
}

// schedule words are read once per block; STREAM loads them non-temporally
// (the batched kernel, whose many meshes stream through the caches: about
// 5 % faster there, while the single-mesh kernel is faster without)
template <bool STREAM, class T>
__device__ __forceinline__ T sched_load(const T *p)
{
    if constexpr (STREAM) return __builtin_nontemporal_load(p);
    else return *p;
}

template <class E, bool STREAM = false>
__device__ __forceinline__ void side_load_elem(const BlockArgs &g, int32_t idx, int32_t (&nid)[E::k],
                                               uint32_t (&ow)[SideLayout<E>::KW], uint32_t (&nw)[E::k])
{
    using L = SideLayout<E>;
#pragma unroll
    for (int a = 0; a < E::k; ++a) nid[a] = sched_load<STREAM>(&g.bconn[a * g.blen + idx]);
    const uint32_t *op = reinterpret_cast<const uint32_t *>(g.boff + static_cast<int64_t>(idx) * L::KKP);
#pragma unroll
    for (int w = 0; w < L::KW; ++w) ow[w] = sched_load<STREAM>(&op[w]);
    const uint32_t *np = g.bnode + static_cast<int64_t>(idx) * E::k;
#pragma unroll
    for (int a = 0; a < E::k; ++a) nw[a] = sched_load<STREAM>(&np[a]);
}

// this thread's first element of the block and its first ordered-entry record
template <class E, bool STREAM = false>
__device__ __forceinline__ void side_load_first(const BlockArgs &g, SideBlock<E> &s)
{
    const int32_t tid = threadIdx.x;
    if (s.e0 + tid < s.e1) side_load_elem<E, STREAM>(g, s.e0 + tid, s.nid, s.ow, s.nw);
    s.ord0 = 0;
    s.ord1 = 0;
    if (s.o0 + tid < s.o1) {
        s.ord0 = sched_load<STREAM>(&g.bord[2 * static_cast<int64_t>(s.o0 + tid)]);
        s.ord1 = sched_load<STREAM>(&g.bord[2 * static_cast<int64_t>(s.o0 + tid) + 1]);
    }
}

template <class E>
__device__ __forceinline__ void side_load_coords(const BlockArgs &g, SideBlock<E> &s)
{
    if (s.e0 + static_cast<int32_t>(threadIdx.x) < s.e1) gather_coords<E>(s.nid, g.coords, g.N, s.x);
}

// Which outputs carry a nodal coefficient: bit s (s < NM) for mass-class slot
// s, bit 2 for the stiffness; kCoefRuntime: decided from the pointers at run
// time.  A compile-time set keeps the unused coefficient paths out of the
// register allocation.
constexpr int kCoefRuntime = -1;

template <int CF>
__device__ __forceinline__ bool has_coef(int bit, const double *ptr)
{
    if constexpr (CF == kCoefRuntime) return ptr != nullptr;
    else return (CF >> bit) & 1;
}

// Q-point data of one element; returns the number of degenerate points.  The
// geometry pass keeps only w_q mu_q and K_q per point; nodal coefficients are
// interpolated afterwards so that they are not live during the geometry.
template <class E, int Q, int NM, bool HA, int CF>
__device__ __forceinline__ int side_qdata(const int32_t (&nid)[E::k], const double (&x)[E::n][E::k],
                                          const double *__restrict__ tab, const double *__restrict__ cm0,
                                          const double *__restrict__ cm1, const double *__restrict__ ca,
                                          double (&f)[NM > 0 ? NM : 1][Q],
                                          double (&kq)[HA ? Q : 1][E::nsym])
{
    double J0[E::n][E::d], H[E::n][E::nh > 0 ? E::nh : 1];
    jacobian_setup<E>(x, J0, H);
    double wmu[Q];
    int bad = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        cdouble *t = const_table(tab) + q * E::stride;
        double J[E::n][E::d];
        jacobian_q<E>(x, J0, H, t, J);
        double K[E::d][E::d], mu;
        geometry<E>(J, K, mu);
        bad += !(mu > 0.0 && mu < INFINITY);
        wmu[q] = t[0] * mu;
        if constexpr (HA) {
            int si = 0;
#pragma unroll
            for (int m = 0; m < E::d; ++m)
#pragma unroll
                for (int l = m; l < E::d; ++l) kq[q][si++] = K[m][l];
        }
        // one point at a time: interleaving the points' geometry raises
        // register pressure more than it hides latency
        __builtin_amdgcn_sched_barrier(0);
    }
    // coefficient at the points: c_h(xi_q) = sum_a c_a phi_a(xi_q)
    auto interp = [&](const double *__restrict__ c, double (&ch)[Q]) {
#pragma unroll
        for (int q = 0; q < Q; ++q) ch[q] = 0.0;
#pragma unroll
        for (int a = 0; a < E::k; ++a) {
            const double ca_ = c[nid[a]];
#pragma unroll
            for (int q = 0; q < Q; ++q) ch[q] = fma(ca_, const_table(tab)[q * E::stride + E::off_phi + a], ch[q]);
        }
    };
    if constexpr (HA) {
        if (has_coef<CF>(2, ca)) {
            double ah[Q];
            interp(ca, ah);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const double fa = wmu[q] * ah[q];
#pragma unroll
                for (int si = 0; si < E::nsym; ++si) kq[q][si] *= fa;
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int si = 0; si < E::nsym; ++si) kq[q][si] *= wmu[q];
        }
    }
    const double *cms[2] = {cm0, cm1};
#pragma unroll
    for (int s = 0; s < NM; ++s) {
        if (has_coef<CF>(s, cms[s])) {
            interp(cms[s], f[s]);
#pragma unroll
            for (int q = 0; q < Q; ++q) f[s][q] = wmu[q] * f[s][q];
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) f[s][q] = wmu[q];
        }
    }
    return bad;
}

__device__ __forceinline__ void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int K, int KW>
__device__ __forceinline__ int32_t slot_off(const uint32_t (&ow)[KW], int a, int b)
{
    const int slot = a * K + b;
    return static_cast<int32_t>((ow[slot >> 2] >> (8 * (slot & 3))) & 0xffu);
}

// values of local pair p (a <= b) of every selected matrix from the Q-point
// data and the pair-major reference tensors.  Sums are split into
// independent chains (mass: by point parity; stiffness: by slot of K) to
// shorten the dependent FMA sequences.
// TAB_LDS: tabp points to a copy of the pair table in LDS (high orders, whose
// table outgrows the scalar cache); otherwise it is read with scalar loads.
template <class E, int Q, int NM, bool HA, bool TAB_LDS = false>
__device__ __forceinline__ void pair_values(int p, const double (&f)[NM > 0 ? NM : 1][Q],
                                            const double (&kq)[HA ? Q : 1][E::nsym],
                                            const double *__restrict__ tabp,
                                            double (&v)[NM + (HA ? 1 : 0)])
{
    constexpr int PS = Q * (1 + E::nsym);
    constexpr int CA = E::nsym > 1 ? E::nsym : 3;  // stiffness chains
    using TabPtr = std::conditional_t<TAB_LDS, const double *, cdouble *>;
    TabPtr t;
    if constexpr (TAB_LDS) t = tabp + p * PS;
    else t = const_table(tabp) + p * PS;
#pragma unroll
    for (int s = 0; s < NM; ++s) {
        double acc[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q & 1] = fma(f[s][q], t[q], acc[q & 1]);
        v[s] = acc[0] + acc[1];
    }
    if constexpr (HA) {
        double acc[CA];
#pragma unroll
        for (int c = 0; c < CA; ++c) acc[c] = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int si = 0; si < E::nsym; ++si) {
                const int c = (q * E::nsym + si) % CA;
                acc[c] = fma(kq[q][si], t[Q + q * E::nsym + si], acc[c]);
            }
        double sum = acc[0];
#pragma unroll
        for (int c = 1; c < CA; ++c) sum += acc[c];
        v[NM] = sum;
    }
}

// form the element's values pair by pair and add them to the block in LDS.
// rb[a] is the entry of node a's row start in the block, or the lane's dump
// entry if the row is outside the block; nw[a] >> 16 is the side slot of the
// contribution (a, a) (0xffff: none).
template <class E, int Q, int NM, bool HA>
__device__ __forceinline__ void side_pairs(const double (&f)[NM > 0 ? NM : 1][Q],
                                           const double (&kq)[HA ? Q : 1][E::nsym],
                                           const double *__restrict__ tabp, const int32_t (&rb)[E::k],
                                           const uint32_t (&ow)[SideLayout<E>::KW],
                                           const uint32_t (&nw)[E::k], double *lds, int nloc, int rs)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    int p = 0;
#pragma unroll
    for (int a = 0; a < E::k; ++a)
#pragma unroll
        for (int b = a; b < E::k; ++b, ++p) {
            double v[NMAT];
            pair_values<E, Q, NM, HA>(p, f, kq, tabp, v);
            int32_t ea = rb[a] + slot_off<E::k>(ow, a, b);
            if (a == b) {
                const uint32_t sslot = nw[a] >> 16;
                ea = sslot != 0xffffu ? nloc + static_cast<int32_t>(sslot) : ea;
            }
#pragma unroll
            for (int mat = 0; mat < NMAT; ++mat) lds_add(&lds[mat * rs + ea], v[mat]);
            if (a != b) {
                const int32_t eb = rb[b] + slot_off<E::k>(ow, b, a);
#pragma unroll
                for (int mat = 0; mat < NMAT; ++mat) lds_add(&lds[mat * rs + eb], v[mat]);
            }
        }
}

// one element: row starts of its nodes in the block, Q-point data, pairs
template <class E, int Q, int NM, bool HA, int CF>
__device__ __forceinline__ int side_element(const BlockArgs &g, int nloc, const int32_t (&nid)[E::k],
                                            const double (&x)[E::n][E::k],
                                            const uint32_t (&ow)[SideLayout<E>::KW], const uint32_t (&nw)[E::k],
                                            double *lds, int32_t dump, int rs)
{
    const int32_t mine = dump + static_cast<int32_t>(threadIdx.x & 63);
    int32_t rb[E::k];
#pragma unroll
    for (int a = 0; a < E::k; ++a) {
        const uint32_t start = nw[a] & 0xffffu;
        rb[a] = start != 0xffffu ? static_cast<int32_t>(start) : mine;
    }
    double f[NM > 0 ? NM : 1][Q];
    double kq[HA ? Q : 1][E::nsym];
    const int bad = side_qdata<E, Q, NM, HA, CF>(nid, x, g.tab, g.cm0, g.cm1, g.ca, f, kq);
    // keep the pair sums out of the geometry phase (starting them early would
    // hold every pair's partial sums in registers)
    __builtin_amdgcn_sched_barrier(0);
    side_pairs<E, Q, NM, HA>(f, kq, g.tabp, rb, ow, nw, lds, nloc, rs);
    return bad;
}

// all elements of the block (the first chunk's data already in s); returns the
// number of degenerate quadrature points met.  With MULTI, elements beyond the
// first NT of the list are loaded here, with their own registers; without it
// the block must hold at most NT elements.
template <class E, int Q, int NM, bool HA, int CF, int NT, bool MULTI, bool STREAM = false>
__device__ __forceinline__ int side_compute(const BlockArgs &g, const SideBlock<E> &s, double *lds, int32_t dump,
                                            int rs)
{
    const int tid = threadIdx.x;
    int bad = 0;
    if (s.e0 + tid < s.e1) bad += side_element<E, Q, NM, HA, CF>(g, s.nloc, s.nid, s.x, s.ow, s.nw, lds, dump, rs);
    if constexpr (MULTI)
    for (int32_t c0 = s.e0 + NT; c0 < s.e1; c0 += NT) {
        const int32_t idx = c0 + tid;
        if (idx < s.e1) {
            int32_t nid[E::k];
            uint32_t ow[SideLayout<E>::KW], nw[E::k];
            double x[E::n][E::k];
            side_load_elem<E, STREAM>(g, idx, nid, ow, nw);
            gather_coords<E>(nid, g.coords, g.N, x);
            bad += side_element<E, Q, NM, HA, CF>(g, s.nloc, nid, x, ow, nw, lds, dump, rs);
        }
    }
    return bad;
}

// sum ordered diagonal w0 = (entry | count << 16) from its side slots starting
// at `first`, in element order, clearing the slots
template <int NMAT>
__device__ __forceinline__ void side_reduce_one(uint32_t w0, uint32_t first, int nloc, double *lds, int rs)
{
    const uint32_t idx = w0 & 0xffffu, cnt = w0 >> 16;
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat) {
        double *reg = lds + mat * rs;
        double *slots = reg + nloc + first;
        double acc = 0.0;
        for (uint32_t j = 0; j < cnt; ++j) {
            acc += slots[j];
            slots[j] = 0.0;
        }
        reg[idx] = acc;
    }
}

template <class E, int NMAT, int NT>
__device__ __forceinline__ void side_reduce(const BlockArgs &g, const SideBlock<E> &s, double *lds, int rs)
{
    const int32_t tid = threadIdx.x;
    if (s.o0 + tid < s.o1) side_reduce_one<NMAT>(s.ord0, s.ord1, s.nloc, lds, rs);
    for (int32_t r = s.o0 + tid + NT; r < s.o1; r += NT)
        side_reduce_one<NMAT>(g.bord[2 * static_cast<int64_t>(r)], g.bord[2 * static_cast<int64_t>(r) + 1],
                              s.nloc, lds, rs);
}

// store the block's values and clear them in LDS.  Thread t stores the
// values at global positions a0 + t + u NT, a0 = base rounded down to 16
// values, so that every wave stores whole 128-byte lines (only the block's
// first and last line are partial): the stores are non-temporal, and partial
// lines written by two different store instructions reach memory as two
// partial writes.
template <int NMAT, int NT>
__device__ __forceinline__ void side_write(const BlockArgs &g, int base, int nloc, double *lds, int rs)
{
    const int lead = base & 15;  // values of the first line that precede the block
#pragma unroll
    for (int mat = 0; mat < NMAT; ++mat) {
        double *__restrict__ out = g.v[mat] + base;
        double *reg = lds + mat * rs;  // index i below is value i - lead of the block
        // eight LDS reads in flight per thread before their stores; the
        // values are written once and not read again here, so the stores are
        // non-temporal (they do not displace the coordinates and element
        // words that halo elements re-read from L2: about 8 % faster)
        const int end = nloc + lead;
        int i = threadIdx.x;
        for (; i + 7 * NT < end; i += 8 * NT) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = i + u * NT >= lead ? reg[i + u * NT - lead] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i + u * NT >= lead) {
                    __builtin_nontemporal_store(t[u], &out[i + u * NT - lead]);
                    reg[i + u * NT - lead] = 0.0;
                }
        }
        for (; i < end; i += NT)
            if (i >= lead) {
                __builtin_nontemporal_store(reg[i - lead], &out[i - lead]);
                reg[i - lead] = 0.0;
            }
    }
}

// one block whose record, first elements and coordinates are loaded (or in
// flight) in s.  LDS value entries must be all zero on entry (and no thread
// may still be writing out a previous block) and are all zero on return.
// Used by the batched kernel: further element chunks stream their schedule
// words.
template <class E, int Q, int NM, bool HA, int CF, int NT>
__device__ __forceinline__ void side_block(const BlockArgs &g, const SideBlock<E> &s, double *lds, int32_t dump,
                                           int rs)
{
    constexpr int NMAT = NM + (HA ? 1 : 0);
    const int bad = side_compute<E, Q, NM, HA, CF, NT, true, true>(g, s, lds, dump, rs);
    if (bad) atomicAdd(g.degenerate, static_cast<unsigned long long>(bad));
    __syncthreads();
    side_reduce<E, NMAT, NT>(g, s, lds, rs);
    __syncthreads();
    side_write<NMAT, NT>(g, s.base, s.nloc, lds, rs);
    __syncthreads();
}

// dump entries after the value entries: one per lane and column offset
inline int side_dump_entries(int max_row) { return 64 + max_row; }

// doubles of one matrix region
inline int side_region(int cap, int max_row) { return cap + side_dump_entries(max_row); }

// bytes of dynamic LDS of the side-slot kernels for NMAT matrices, value
// capacity cap and longest row max_row
inline size_t side_lds_bytes(int nmat, int cap, int max_row)
{
    return static_cast<size_t>(nmat) * side_region(cap, max_row) * sizeof(double);
}

}  // namespace lfem
