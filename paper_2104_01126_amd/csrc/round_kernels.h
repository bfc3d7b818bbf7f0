// One round of the filtered Kruskal over the well-separated pair
// decomposition (paper Sec. 3.1.2-3.1.3, Alg. 1-3, and Sec. 3.2.2):
//
//   * node pairs whose weight lower bound is at most beta are expanded as in
//     FindPair: a well-separated pair yields its bichromatic closest pair
//     (BCCP, or BCCP* under mutual reachability); otherwise the node with the
//     larger bounding sphere is split;
//   * pairs whose points are already in one component are dropped (the
//     union-find filter);
//   * pairs whose lower bound exceeds beta wait in a frontier for a later
//     round, BCCP edges heavier than beta wait in a pool;
//   * the edges of weight at most beta are merged into the spanning forest
//     in key order (Kruskal's rule, done as Boruvka steps on the key ranks).
//
// Every bound used to schedule or prune is computed with the same operation
// order as the distances it bounds, so it never crosses a computed distance:
// rounding is monotone, hence fl(lo_B - hi_A) <= fl(|b - a|) per dimension and
// the sums keep the order.
#pragma once
#include "common.h"
#include "tree_kernels.h"

namespace geomst {

enum CounterSlot {
    C_QN = 0,  // next expansion queue
    C_Q,       // queue produced by the frontier split
    C_F,       // frontier out
    C_C,       // committed edges
    C_P,       // pool out
    C_BIG,     // pairs for the large-pair BCCP kernel
    C_OUT,     // spanning-tree edges found so far
    C_ALIVE,   // Boruvka: edges still undecided after this step
    C_ERR,     // device-side error flags
    C_FAR,     // far frontier out
    C_TINY,    // small separated pairs for the inline BCCP kernel
    C_NUM
};
// C64_EVALS counts |A||B| of every separated pair; C64_BIGWORK the part of it
// handed to the large-pair kernel, of which C64_BIGEVALS were evaluated (the
// rest was pruned by block bounds).
enum CounterSlot64 { C64_EVALS = 0, C64_VISITS, C64_BCCP, C64_BIGEVALS, C64_TASKS, C64_BIGWORK, C64_NUM };
enum MinSlot { M_F = 0, M_P, M_FAR, M_NUM };

struct Counters {
    u32 c[16];
    unsigned long long c64[C64_NUM];
    u64 m[4];  // bit patterns of non-negative doubles (all ones = none)
};

struct PairRec {
    u32 a, b;
    double lb2;  // lower bound of the pair's edge weights (squared)
};

struct EdgeList {
    double* w2;
    double* e2;
    u64* ids;  // (lo << 32) | hi, caller row indices
    u64* pos;  // (sorted position i << 32) | sorted position j of the two ends
};

struct RoundArgs {
    Counters* cnt;
    double beta2;
    double sep;      // separation constant s of the sphere test
    int mutual;      // HDBSCAN*: mutual unreachability also separates (0: geometric test only)
    u32 beta_card;   // GFK schedule: pairs with |A| + |B| <= this are due whatever their bound (0: off)
    double t_near;   // waiting pairs with bounds up to this go to the near list
    PairRec* ffar;   // far list (appended)
    u32 cap_far;
    const u32* uf;  // sorted position -> component root (fully compressed)
    PairRec* fout;
    u32 cap_f;
    PairRec* q;
    u32 cap_q;
    uint2* big;
    u32 cap_big;
    uint4* tiny;  // {first A, first B, count A << 16 | count B, 0}
    u32 cap_tiny;
    EdgeList c;
    u32 cap_c;
    EdgeList pout;
    u32 cap_p;
    const int* labels;  // compact copy of the node records' component labels
};

constexpr int kTinyEvals = 16;   // pairs with at most this many point pairs are solved inline

// ------------------------------------------------------------ bounds
template <int D>
__device__ __forceinline__ double box_lb2(const NodeRec<D>& A, const NodeRec<D>& B) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double g = fmax(fmax((double)B.lo[k] - (double)A.hi[k], (double)A.lo[k] - (double)B.hi[k]), 0.0);
        s = s + g * g;
    }
    return s;
}

template <int D>
__device__ __forceinline__ double box_diag2(const NodeRec<D>& A) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t = (double)A.hi[k] - (double)A.lo[k];
        s = s + t * t;
    }
    return s;
}

// Lower bound of the (squared) weight of any edge between the two nodes;
// ca/cb are the nodes' (min, max) squared core distances (HDBSCAN*).
template <int D>
__device__ __forceinline__ double pair_wlb2(const NodeRec<D>& A, const NodeRec<D>& B, int hdb, double2 ca,
                                            double2 cb) {
    double l = box_lb2<D>(A, B);
    if (hdb) l = fmax(l, fmax(ca.x, cb.x));
    return l;
}

// Whether nodes a and b lie in one component, from the compact copy of the
// records' component labels (4 bytes per node, equal to the records' labels
// after every refresh and negative, like theirs, before the first): for
// kernels that need no other field of the records.
__device__ __forceinline__ bool connected_lab(const int* labels, u32 a, u32 b) {
    const int ca = labels[a];
    return ca >= 0 && ca == labels[b];
}

// GFK schedule (Alg. 2): a pair of cardinality at most beta_card has its BCCP
// computed in this round whatever its bound (edges above the threshold wait
// in the pool, the BCCP cache).
template <int D>
__device__ __forceinline__ bool card_due(const TreeView& t, u32 beta_card, u32 a, u32 b) {
    if (!beta_card) return false;
    const NodeRec<D>* N = nodes_of<D>(t);
    return (u64)N[a].count + (u64)N[b].count <= (u64)beta_card;
}

// Well-separation test.  Geometric (Sec. 2.3, s = 2, in the form of
// Sec. 3.2.2): the gap between the bounding spheres is at least the larger
// sphere diameter.  For HDBSCAN* (mutual != 0) also mutual unreachability
// (Sec. 3.2.2): max(gap, cdmin A, cdmin B) >= max(diam A, diam B, cdmax A,
// cdmax B).  With mutual == 0 an HDBSCAN* solve uses the geometric test
// alone, as the HDBSCAN*-GanTao variant does (Sec. 3.2.1).
// Both are taken together with a strict guard on computed values (largest
// intra-node distance bound below the inter-node bound) which makes the
// BCCP edge of each pair contain the tree's edge exactly; a pair of two
// single points is always separated.
template <int D>
__device__ __forceinline__ bool well_separated(const NodeRec<D>& A, const NodeRec<D>& B, int mutual, double2 ca,
                                               double2 cb, double s, double dA, double dB, const TreeView& t, u32 ia,
                                               u32 ib) {
    if (A.count == 1 && B.count == 1) return true;
    double L = box_lb2<D>(A, B);
    // sphere radii: half the box diagonals (single precision suffices, the
    // sphere test only makes the strict box guard stricter)
    double ra = 0.5f * __builtin_sqrtf((float)dA), rb = 0.5f * __builtin_sqrtf((float)dB);
    double c2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double x = 0.5 * ((double)A.lo[k] + (double)A.hi[k]) - 0.5 * ((double)B.lo[k] + (double)B.hi[k]);
        c2 = c2 + x * x;
    }
    double need = ra + rb + s * fmax(ra, rb);
    bool geo = (fmax(dA, dB) < L) && (c2 >= need * need);
    if (geo || !mutual) return geo;
    // the mutual test compares core distances with each other: it takes the
    // exact ranges (a record's binary32 copy would make it stricter than
    // needed and lose most of its pairs)
    if constexpr (NodeBox<D>::cd_in) {
        ca = t.cdr[ia];
        cb = t.cdr[ib];
    }
    double gap = fmax(sqrt(c2) - ra - rb, 0.0);
    double lhs_s = fmax(fmax(dA, dB), fmax(ca.y, cb.y));
    double rhs_s = fmax(gap * gap, fmax(ca.x, cb.x));
    // The strict guard bounds the weight of a pair of distinct points inside
    // one node, max(diam^2, cdmax), below the pair's bound; a single-point
    // node has no such pair, so its own core distance does not enter.
    double la = A.count > 1 ? fmax(dA, ca.y) : -1.0, lb_ = B.count > 1 ? fmax(dB, cb.y) : -1.0;
    double lhs = fmax(la, lb_);
    double rhs = fmax(L, fmax(ca.x, cb.x));
    return (rhs_s >= lhs_s) && (lhs < rhs);
}

// ------------------------------------------------------------ edges
struct EdgeOut {
    EKey k;
    u32 i, j;  // sorted positions
};

// The weight and squared distance of point_edge alone (same operations).
// (HDBSCAN* reads the rows with the core distance appended, XC.)
template <int D>
__device__ __forceinline__ void point_w2(const TreeView& t, int hdb, u32 i, u32 j, double& w2, double& e2) {
    e2 = 0.0;
    if (hdb) {
        const double* a = t.XC + (size_t)i * (D + 1);
        const double* b = t.XC + (size_t)j * (D + 1);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double x = a[k] - b[k];
            e2 = e2 + x * x;
        }
        w2 = fmax(fmax(a[D], b[D]), e2);
        return;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double x = t.X[(size_t)i * D + k] - t.X[(size_t)j * D + k];
        e2 = e2 + x * x;
    }
    w2 = e2;
}

template <int D>
__device__ __forceinline__ EdgeOut point_edge(const TreeView& t, int hdb, u32 i, u32 j) {
    EdgeOut o;
    double e2, w2;
    point_w2<D>(t, hdb, i, j, w2, e2);
    u32 oi = t.orig[i], oj = t.orig[j];
    o.k.w2 = w2;
    o.k.e2 = e2;
    o.k.lo = oi < oj ? oi : oj;
    o.k.hi = oi < oj ? oj : oi;
    o.i = i;
    o.j = j;
    return o;
}

__device__ __forceinline__ void put_edge(EdgeList L, u32 s, const EdgeOut& e) {
    L.w2[s] = e.k.w2;
    L.e2[s] = e.k.e2;
    L.ids[s] = ((u64)e.k.lo << 32) | e.k.hi;
    L.pos[s] = ((u64)e.i << 32) | e.j;
}

__device__ __forceinline__ void put_edge_raw(EdgeList L, u32 s, double w2, double e2, u64 ids, u64 pos) {
    L.w2[s] = w2;
    L.e2[s] = e2;
    L.ids[s] = ids;
    L.pos[s] = pos;
}

__device__ __forceinline__ void flag_overflow(Counters* cnt) { atomicOr(&cnt->c[C_ERR], 1u); }
// level-queue overflow: its count may be cleared before the host looks, so
// it has a flag bit of its own
__device__ __forceinline__ void flag_overflow_q(Counters* cnt) { atomicOr(&cnt->c[C_ERR], 1u | 16u); }

// ------------------------------------------------------ block-level appends
// L output lists per block step.  Each thread passes how many entries it adds
// to each list; the counts travel packed B bits apiece in 64-bit words
// through one wave scan per word, and one atomic per non-empty list per block
// reserves the space; each thread gets its slot offsets back.  A block's
// total per list must stay below 2^B.  All threads of the block must call it.
template <int L, int B>
struct BlockAllocN {
    static constexpr int kPer = 64 / B;
    static constexpr int kWords = (L + kPer - 1) / kPer;
    u64 wsum[kWords][16];
    u32 base[L];
};

constexpr int kLists = 6;
using BlockAlloc = BlockAllocN<kLists, 16>;

__device__ __forceinline__ u64 wave_incl_scan_u64(u64 v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        u64 t = __shfl_up(v, o);
        if (lane_id() >= o) v += t;
    }
    return v;
}

template <int L, int B>
__device__ __forceinline__ void block_alloc(BlockAllocN<L, B>& S, const u32 (&cnt)[L], u32* const* counters,
                                            u32 (&off)[L]) {
    constexpr int P = BlockAllocN<L, B>::kPer, W = BlockAllocN<L, B>::kWords;
    constexpr u64 M = (1ull << B) - 1;
    const int w = threadIdx.x / kWave;
    u64 p[W], inc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) p[k] = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) p[l / P] |= (u64)cnt[l] << (B * (l % P));
#pragma unroll
    for (int k = 0; k < W; ++k) inc[k] = wave_incl_scan_u64(p[k]);
    if (lane_id() == kWave - 1) {
#pragma unroll
        for (int k = 0; k < W; ++k) S.wsum[k][w] = inc[k];
    }
    __syncthreads();
    if (w == 0) {
        // wave 0 turns the per-wave sums into exclusive prefixes (one lane
        // per wave) and reserves every list's block total with one atomic per
        // list, issued by lanes 0..L-1 together: the counters are distinct
        // addresses, so the atomics go out as one instruction and their
        // round trips overlap
        const int nw = (int)(blockDim.x / kWave);
        const int ln = lane_id();
        u64 tot[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const u64 v = ln < nw ? S.wsum[k][ln] : 0ull;
            const u64 incl = wave_incl_scan_u64(v);
            tot[k] = __shfl(incl, kWave - 1);
            if (ln < nw) S.wsum[k][ln] = incl - v;
        }
        u32 c = 0;
        u32* cp = nullptr;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (ln == l) {
                c = (u32)((tot[l / P] >> (B * (l % P))) & M);
                cp = counters[l];
            }
        }
        if (ln < L) S.base[ln] = (cp && c) ? atomicAdd(cp, c) : 0u;
    }
    __syncthreads();
    u64 e[W];
#pragma unroll
    for (int k = 0; k < W; ++k) e[k] = inc[k] - p[k] + S.wsum[k][w];
#pragma unroll
    for (int l = 0; l < L; ++l) off[l] = S.base[l] + (u32)((e[l / P] >> (B * (l % P))) & M);
    __syncthreads();
}

// ------------------------------------------------------ level-queue regions
// A level queue is cut into kRegions equal regions, one per XCD: workgroup
// b of a level launch runs on XCD b % 8 (the dispatcher deals workgroups to
// the XCDs in turn), reads a slice of the queue that is mostly its own
// region and appends the child pairs it makes to its own region.  A pair's
// descendants thus stay on one XCD, and the records of the subtree they
// touch stay in that XCD's L2.  The frontier split seeds the regions by tree
// position of a pair's first node (internal node i spans sorted position i,
// leaf n-1+i is position i), so a region starts out as one slab of the
// Morton curve.  Each region's counter has a 128-byte line of its own; the
// counters of one level form a slot of the kQRing-slot ring.
constexpr int kRegions = 8;
constexpr int kRegionStride = 32;  // u32 words between region counters
constexpr int kSlotWords = kRegions * kRegionStride;

__device__ __forceinline__ int node_region(u32 node, int n) {
    const u32 pos = node < (u32)(n - 1) ? node : node - (u32)(n - 1);
    return (int)(((u64)pos * kRegions) / (u64)n);
}

// Slot counts (clamped to the region capacity) as prefix sums pre[0..8].
__device__ __forceinline__ void region_prefix(const u32* slot, u32 cap, u32 (&pre)[kRegions + 1]) {
    pre[0] = 0;
#pragma unroll
    for (int x = 0; x < kRegions; ++x) pre[x + 1] = pre[x] + min(slot[x * kRegionStride], cap);
}

// Position in the queue buffer of entry v of the regions laid end to end.
__device__ __forceinline__ u32 region_index(const u32 (&pre)[kRegions + 1], u32 cap, u32 v) {
    u32 base = 0, start = 0;
#pragma unroll
    for (int x = 1; x < kRegions; ++x)
        if (v >= pre[x]) {
            base = (u32)x * cap;
            start = pre[x];
        }
    return base + (v - start);
}

// The wide small-level mode splits region x of a queue into kSub
// sub-segments of cap / kSub pairs, one per workgroup, with sub-segment w's
// count in word x * kRegionStride + w of the slot; `sub` (1 or kSub) names
// the layout of a queue, and its segments, in order, are (x, w) for x < 8,
// w < sub.
constexpr int kSub = kRegionStride;
constexpr int kSegs = kRegions * kSub;

// Prefix sums pre[0..8 sub] of the segment counts of a slot (each clamped to
// the segment capacity), written to LDS by wave 0 (the caller synchronises).
__device__ __forceinline__ void seg_prefix(const u32* slot, u32 cap, int sub, u32* pre) {
    if (threadIdx.x >= kWave) return;
    const int ln = lane_id();
    const int nseg = kRegions * sub, per = (nseg + kWave - 1) / kWave;
    const u32 scap = cap / (u32)sub;
    u32 c[kSegs / kWave];
    u64 sum = 0;
#pragma unroll
    for (int i = 0; i < kSegs / kWave; ++i) {
        const int sg = ln * per + i;
        c[i] = (i < per && sg < nseg) ? min(slot[(sg / sub) * kRegionStride + sg % sub], scap) : 0u;
        sum += c[i];
    }
    u64 run = wave_incl_scan_u64(sum) - sum;
    if (ln == 0) pre[0] = 0;
#pragma unroll
    for (int i = 0; i < kSegs / kWave; ++i) {
        const int sg = ln * per + i;
        run += c[i];
        if (i < per && sg < nseg) pre[sg + 1] = (u32)run;
    }
}

// Position in the queue buffer of entry v (< pre[nseg]) of the segments laid
// end to end: the segment s with pre[s] <= v < pre[s + 1], by bisection.
__device__ __forceinline__ u32 seg_index(const u32* pre, int sub, u32 cap, u32 v) {
    u32 lo = 0, hi = (u32)(kRegions * sub);
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (pre[mid] <= v) lo = mid;
        else hi = mid;
    }
    return (lo / (u32)sub) * cap + (lo % (u32)sub) * (cap / (u32)sub) + (v - pre[lo]);
}

// Block-wide minimum of a non-negative double, one atomic per block.
// sh holds one slot per wave.
__device__ __forceinline__ void block_atomic_min(double v, u64* dst, double* sh) {
    v = wave_min_f64(v);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) m = fmin(m, sh[i]);
        if (m < __longlong_as_double(0x7ff0000000000000ll)) atomic_min_pos_f64(dst, m);
    }
    __syncthreads();
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) sh[w] = v;
    __syncthreads();
    unsigned long long s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += sh[i];
    __syncthreads();
    return s;
}

constexpr int kBlock = 256;
constexpr int kSplitItems = 8;  // list items per thread in the split kernels (one append per 2048)
constexpr int kSplitTile = kSplitItems * kBlock;
constexpr int kGrid = 1024;      // blocks of the grid-stride round kernels
constexpr int kQRing = 4;        // level queue counters (ring)

// ------------------------------------------------------------ frontier
// Initial frontier: the two children of every internal node (Alg. 1, Wspd).
// In a batched solve (pinst non-null) the two children of a node that joins
// several instances belong to different instances: such a pair is never
// expanded (bound +inf, dropped by the far split).
template <int D>
__global__ void k_init_frontier(TreeView t, int hdb, const u32* pinst, PairRec* f) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.n - 1) return;
    const NodeRec<D>* N = nodes_of<D>(t);
    int2 c = node_kids(t.n, N[i].first, N[i].count, N[i].split);
    PairRec p;
    p.a = (u32)c.x;
    p.b = (u32)c.y;
    double2 z = make_double2(0.0, 0.0);
    const NodeRec<D> A = N[p.a], B = N[p.b];
    p.lb2 = pair_wlb2<D>(A, B, hdb, hdb ? node_cd<D>(t, A, p.a) : z, hdb ? node_cd<D>(t, B, p.b) : z);
    if (pinst && pinst[N[p.a].first] != pinst[N[p.b].first]) p.lb2 = __longlong_as_double(0x7ff0000000000000ll);
    f[i] = p;
}

// Start of a round: zero the per-round list counters, set the minima to
// "none", keep `far_keep` retained far pairs.  The error flags and the
// running totals are left alone.
__global__ void k_round_reset(Counters* cnt, u32 far_keep, u32* ring) {
    const int i = threadIdx.x;
    if (i < C_OUT) cnt->c[i] = 0;
    if (i == 0) {
        cnt->c[C_FAR] = far_keep;
        cnt->c[C_TINY] = 0;
    }
    if (i < M_NUM) cnt->m[i] = ~0ull;
    for (int w = i; w < kQRing * kSlotWords; w += blockDim.x) ring[w] = 0;  // level-queue counts
}

// Smallest positive lower bound over a pair list and, when `hist` is given,
// how many of the positive finite bounds fall in each binade (histogram over
// the binary64 exponent): the first beta is chosen from them.
constexpr int kExpBins = 2048;

__global__ void __launch_bounds__(kBlock) k_min_positive_lb(const PairRec* f, u32 nf, Counters* cnt, u32* hist) {
    __shared__ double sh[4];
    __shared__ u32 h[kExpBins];
    for (int b = threadIdx.x; b < kExpBins; b += kBlock) h[b] = 0;
    __syncthreads();
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    double v = inf;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x) {
        const double lb = f[i].lb2;
        if (lb > 0.0 && lb < inf) {  // +inf (cross-instance) never counts
            v = fmin(v, lb);
            if (hist) atomicAdd(&h[(u32)(dbits(lb) >> 52) & (kExpBins - 1)], 1u);
        }
    }
    __syncthreads();
    if (hist)
        for (int b = threadIdx.x; b < kExpBins; b += kBlock)
            if (h[b]) atomicAdd(&hist[b], h[b]);
    block_atomic_min(v, &cnt->m[M_F], sh);
}

// Near-frontier split: drop the pairs whose nodes already lie in one
// component (from the compact label copy: two 4-byte reads), queue the
// pairs whose lower bound is within beta (each in the region of its first
// node), keep the rest in the near list.
constexpr int kSplitLists = kRegions + 2;  // regions, near list, far list
using SplitAlloc = BlockAllocN<kSplitLists, 12>;

// appends item k to region `rg` of the queue: the region's next offset
__device__ __forceinline__ u32 take_region_slot(u32 (&off)[kSplitLists], int rg) {
    u32 slot = 0;
#pragma unroll
    for (int x = 0; x < kRegions; ++x)
        if (rg == x) slot = off[x]++;
    return slot;
}

__device__ __forceinline__ void put_queued(const RoundArgs& r, u32 slot, int rg, const PairRec& p) {
    if (slot < r.cap_q) r.q[(size_t)rg * r.cap_q + slot] = p;
    else flag_overflow(r.cnt);
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_split_frontier(TreeView t, RoundArgs r, const PairRec* fin, u32 nfin,
                                                           u32* qslot) {
    __shared__ SplitAlloc S;
    __shared__ double shm[4];
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    u32* ctr[kSplitLists];
#pragma unroll
    for (int x = 0; x < kRegions; ++x) ctr[x] = qslot + x * kRegionStride;
    ctr[kRegions] = &r.cnt->c[C_F];
    ctr[kRegions + 1] = nullptr;
    double minf = inf;
    for (u32 b0 = blockIdx.x * kSplitTile; b0 < nfin; b0 += gridDim.x * kSplitTile) {
        PairRec p[kSplitItems];
        u32 due = 0, wait = 0, rgs = 0;
        u32 cnt[kSplitLists] = {};
#pragma unroll
        for (int k = 0; k < kSplitItems; ++k) {
            const u32 i = b0 + k * kBlock + threadIdx.x;
            if (i < nfin) {
                p[k] = fin[i];
                const bool keep = !connected_lab(r.labels, p[k].a, p[k].b);
                const bool d = keep && (p[k].lb2 <= r.beta2 || card_due<D>(t, r.beta_card, p[k].a, p[k].b));
                due |= (u32)d << k;
                wait |= (u32)(keep && !d) << k;
                if (d) {
                    const int rg = node_region(p[k].a, t.n);
                    rgs |= (u32)rg << (3 * k);
#pragma unroll
                    for (int x = 0; x < kRegions; ++x) cnt[x] += (rg == x);
                } else if (keep) {
                    ++cnt[kRegions];
                    minf = fmin(minf, p[k].lb2);
                }
            }
        }
        u32 off[kSplitLists];
        block_alloc(S, cnt, ctr, off);
#pragma unroll
        for (int k = 0; k < kSplitItems; ++k) {
            if ((due >> k) & 1u) {
                const int rg = (int)((rgs >> (3 * k)) & 7u);
                put_queued(r, take_region_slot(off, rg), rg, p[k]);
            }
            if ((wait >> k) & 1u) {
                if (off[kRegions] < r.cap_f) r.fout[off[kRegions]] = p[k];
                else flag_overflow(r.cnt);
                ++off[kRegions];
            }
        }
    }
    block_atomic_min(minf, &r.cnt->m[M_F], shm);
}

// Far-frontier split at the start of a band: drop pairs whose points are now
// in one component, queue the due ones, move those within the new band edge
// to the near list and keep the rest far.
template <int D>
__global__ void __launch_bounds__(kBlock) k_split_far(TreeView t, RoundArgs r, const PairRec* fin, u32 nfin,
                                                      u32* qslot) {
    __shared__ SplitAlloc S;
    __shared__ double shm[4];
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    u32* ctr[kSplitLists];
#pragma unroll
    for (int x = 0; x < kRegions; ++x) ctr[x] = qslot + x * kRegionStride;
    ctr[kRegions] = &r.cnt->c[C_F];
    ctr[kRegions + 1] = &r.cnt->c[C_FAR];
    double minf = inf, minfar = inf;
    for (u32 b0 = blockIdx.x * kSplitTile; b0 < nfin; b0 += gridDim.x * kSplitTile) {
        PairRec p[kSplitItems];
        u32 cls = 0;  // 2 bits per item: 1 due, 2 near, 3 far, 0 dropped
        u32 rgs = 0;
        u32 cnt[kSplitLists] = {};
#pragma unroll
        for (int k = 0; k < kSplitItems; ++k) {
            const u32 i = b0 + k * kBlock + threadIdx.x;
            if (i < nfin) {
                p[k] = fin[i];
                const bool keep = p[k].lb2 < inf && !connected_lab(r.labels, p[k].a, p[k].b);
                const bool due = keep && (p[k].lb2 <= r.beta2 || card_due<D>(t, r.beta_card, p[k].a, p[k].b));
                const bool near = keep && !due && p[k].lb2 <= r.t_near;
                const bool far = keep && !due && !near;
                if (near) minf = fmin(minf, p[k].lb2);
                if (far) minfar = fmin(minfar, p[k].lb2);
                cls |= (due ? 1u : near ? 2u : far ? 3u : 0u) << (2 * k);
                if (due) {
                    const int rg = node_region(p[k].a, t.n);
                    rgs |= (u32)rg << (3 * k);
#pragma unroll
                    for (int x = 0; x < kRegions; ++x) cnt[x] += (rg == x);
                }
                cnt[kRegions] += near;
                cnt[kRegions + 1] += far;
            }
        }
        u32 off[kSplitLists];
        block_alloc(S, cnt, ctr, off);
#pragma unroll
        for (int k = 0; k < kSplitItems; ++k) {
            const u32 c = (cls >> (2 * k)) & 3u;
            if (c == 1u) {
                const int rg = (int)((rgs >> (3 * k)) & 7u);
                put_queued(r, take_region_slot(off, rg), rg, p[k]);
            } else if (c == 2u) {
                if (off[kRegions] < r.cap_f) r.fout[off[kRegions]] = p[k];
                else flag_overflow(r.cnt);
                ++off[kRegions];
            } else if (c == 3u) {
                if (off[kRegions + 1] < r.cap_far) r.ffar[off[kRegions + 1]] = p[k];
                else flag_overflow(r.cnt);
                ++off[kRegions + 1];
            }
        }
    }
    block_atomic_min(minf, &r.cnt->m[M_F], shm);
    block_atomic_min(minfar, &r.cnt->m[M_FAR], shm);
}

// ------------------------------------------------------------ expansion
// One breadth-first level of the FindPair recursion (Alg. 1).  Each lane
// takes one pair: a pair whose points are all in one component is dropped; a
// pair whose weight lower bound exceeds beta is parked in the frontier; a
// well-separated pair is queued for its BCCP edge (for k_tiny_bccp when it has
// at most kTinyEvals point pairs, else for the large-pair kernel); otherwise
// the node with the larger bounding sphere is split, and each child pair goes
// to the frontier (bound above beta) or to the next level.  Connectivity of a
// child pair is checked when it is expanded.
struct LevelAcc {
    double minf, minp, minfar;
    unsigned long long visits, evals, solved;
};

// One block step of a level: a thread with `have` takes pair qin[i]; child
// pairs due in this round go to qout through counter ctr[5].  All threads of
// the block must call it.
template <int D>
__device__ __forceinline__ void level_step(const TreeView& t, const RoundArgs& r, int hdb, bool have,
                                           const PairRec& pr, PairRec* qout, u32 cap_qout, u32* const* ctr,
                                           BlockAlloc& S, LevelAcc& acc) {
    const NodeRec<D>* N = nodes_of<D>(t);
    bool to_tiny = false, to_big = false, to_f = false;
    uint4 tp = make_uint4(0u, 0u, 0u, 0u);
    u32 a = 0, b = 0, oth = 0;
    int2 ch = make_int2(0, 0);
    double lb = 0.0;
    double lbc[2] = {0.0, 0.0};
    bool cf[2] = {false, false}, cq[2] = {false, false};
    if (have) {
        a = pr.a;
        b = pr.b;
        ++acc.visits;
        const NodeRec<D> A = N[a], B = N[b];
        const int ka = A.comp, kb = B.comp;
        if (!(ka >= 0 && ka == kb)) {
            double2 z = make_double2(0.0, 0.0);
            double2 ca = hdb ? node_cd<D>(t, A, a) : z, cb = hdb ? node_cd<D>(t, B, b) : z;
            lb = pair_wlb2<D>(A, B, hdb, ca, cb);
            const double dA = box_diag2<D>(A), dB = box_diag2<D>(B);
            if (lb > r.beta2 && !card_due<D>(t, r.beta_card, a, b)) {
                to_f = true;
            } else if (well_separated<D>(A, B, hdb && r.mutual, ca, cb, r.sep, dA, dB, t, a, b)) {
                u64 work = (u64)A.count * (u64)B.count;
                if (work <= (u64)kTinyEvals) {
                    // solved by k_tiny_bccp after the level loop, away from
                    // this step's barriers
                    to_tiny = true;
                    tp = make_uint4((u32)A.first, (u32)B.first, ((u32)A.count << 16) | (u32)B.count, 0u);
                } else {
                    to_big = true;
                }
            } else {
                // split the node with the larger bounding sphere (Alg. 1, FindPair)
                bool split_a = (B.count == 1) || (A.count > 1 && (dA > dB || (dA == dB && A.count >= B.count)));
                const NodeRec<D>& X = split_a ? A : B;
                const NodeRec<D>& O = split_a ? B : A;
                double2 co = split_a ? cb : ca;
                const int kother = split_a ? kb : ka;
                oth = split_a ? b : a;
                ch = node_kids(t.n, X.first, X.count, X.split);
                // the two children are usually adjacent records (and adjacent
                // component entries): drop connected child pairs, bound the
                // others, park the far ones
                const NodeRec<D> C0 = N[ch.x], C1 = N[ch.y];
                int kc[2] = {C0.comp, C1.comp};
                double2 c0 = hdb ? node_cd<D>(t, C0, (u32)ch.x) : z, c1 = hdb ? node_cd<D>(t, C1, (u32)ch.y) : z;
                lbc[0] = pair_wlb2<D>(C0, O, hdb, c0, co);
                lbc[1] = pair_wlb2<D>(C1, O, hdb, c1, co);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    if (kc[c] >= 0 && kc[c] == kother) continue;
                    if (lbc[c] > r.beta2 && !card_due<D>(t, r.beta_card, c == 0 ? (u32)ch.x : (u32)ch.y, oth))
                        cf[c] = true;
                    else
                        cq[c] = true;
                }
            }
        }
    }
    // waiting pairs: the pair itself (to_f) or its children (cf)
    PairRec wp[3];
    bool wnear[3] = {false, false, false}, wfar[3] = {false, false, false};
    u32 nn = 0, nf = 0, nq2 = 0;
    wp[0].a = a;
    wp[0].b = b;
    wp[0].lb2 = lb;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        wp[1 + c].a = (u32)(c == 0 ? ch.x : ch.y);
        wp[1 + c].b = oth;
        wp[1 + c].lb2 = lbc[c];
        nq2 += cq[c] ? 1 : 0;
    }
    bool wait[3] = {to_f, cf[0], cf[1]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!wait[k]) continue;
        if (wp[k].lb2 <= r.t_near) {
            wnear[k] = true;
            ++nn;
            acc.minf = fmin(acc.minf, wp[k].lb2);
        } else {
            wfar[k] = true;
            ++nf;
            acc.minfar = fmin(acc.minfar, wp[k].lb2);
        }
    }
    u32 cnt[kLists] = {(u32)to_tiny, 0u, (u32)to_big, nn, nf, nq2};
    u32 off[kLists];
    block_alloc(S, cnt, ctr, off);
    if (to_tiny) {
        if (off[0] < r.cap_tiny) r.tiny[off[0]] = tp;
        else flag_overflow(r.cnt);
    }
    if (to_big) {
        if (off[2] < r.cap_big) r.big[off[2]] = make_uint2(a, b);
        else flag_overflow(r.cnt);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (wnear[k]) {
            if (off[3] < r.cap_f) r.fout[off[3]] = wp[k];
            else flag_overflow(r.cnt);
            ++off[3];
        }
        if (wfar[k]) {
            if (off[4] < r.cap_far) r.ffar[off[4]] = wp[k];
            else flag_overflow(r.cnt);
            ++off[4];
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (cq[c]) {
            if (off[5] < cap_qout) qout[off[5]] = wp[1 + c];
            else flag_overflow_q(r.cnt);
            ++off[5];
        }
    }
}

// End of a level kernel: the block's three minima and three counts in one
// LDS round (one barrier), then wave 0 reduces over the waves and lanes 0..5
// issue the six atomics together.
template <int NT>
__device__ __forceinline__ void level_flush(const RoundArgs& r, LevelAcc& acc) {
    constexpr int NW = NT / kWave;
    __shared__ double shm[3][NW];
    __shared__ unsigned long long shs[3][NW];
    const double inf_ = __longlong_as_double(0x7ff0000000000000ll);
    double mv[3] = {acc.minf, acc.minp, acc.minfar};
    unsigned long long sv[3] = {acc.visits, acc.evals, acc.solved};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        mv[i] = wave_min_f64(mv[i]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sv[i] += __shfl_xor(sv[i], o);
    }
    const int w = threadIdx.x / kWave, ln = lane_id();
    if (ln == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            shm[i][w] = mv[i];
            shs[i][w] = sv[i];
        }
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mv[i] = wave_min_f64(ln < NW ? shm[i][ln] : inf_);
            sv[i] = ln < NW ? shs[i][ln] : 0ull;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) sv[i] += __shfl_xor(sv[i], o);
        }
        if (ln < 3) {
            const double v = ln == 0 ? mv[0] : (ln == 1 ? mv[1] : mv[2]);
            u64* dst = &r.cnt->m[ln == 0 ? M_F : (ln == 1 ? M_P : M_FAR)];
            if (v < inf_) atomic_min_pos_f64(dst, v);
        } else if (ln < 6 && sv[0]) {
            const unsigned long long v = ln == 3 ? sv[0] : (ln == 4 ? sv[1] : sv[2]);
            atomicAdd(&r.cnt->c64[ln == 3 ? C64_VISITS : (ln == 4 ? C64_EVALS : C64_BCCP)], v);
        }
    }
}

// Occupancy targets: the expansion is bound by the latency of dependent
// loads, so more resident waves help more than the few registers they cost.
template <int D>
struct LevelWaves {
    static constexpr int value = D <= 5 ? 4 : 3;
};

// One breadth-first level over the whole grid.  Blocks beyond the queue
// leave at once.  Blocks are large because every step appends to the shared
// lists with one atomic per list, and those few counters are the contended
// addresses of the expansion: fewer, larger steps mean fewer atomics.  One
// block per CU, as large as the registers allow: 1024 threads at four waves
// per SIMD where the level step fits 128 registers (d <= 5), else 768 at
// three (up to 168 registers).
template <int D>
struct LevelShape {
    static constexpr int block = D <= 5 ? 1024 : 768;
    static constexpr int grid = 256;
    static_assert(grid % kRegions == 0, "every XCD gets the same number of workgroups");
};

// The queue is read as its regions laid end to end; XCD x's workgroups take
// the x-th eighth of that sequence (its own region when the regions are
// balanced, a neighbour's surplus otherwise) and append children to region x
// of the output queue r.q (region capacity r.cap_q).
template <int D>
__global__ void __launch_bounds__(LevelShape<D>::block) __attribute__((amdgpu_waves_per_eu(LevelWaves<D>::value)))
k_level(TreeView t, RoundArgs r, int hdb, const PairRec* qin, u32 cap_in, int sub_in, const u32* slot_in,
        u32* slot_next, u32* slot_clear) {
    __shared__ BlockAlloc S;
    __shared__ u32 pre[kSegs + 1];  // segment prefix sums (in LDS: registers are the scarce resource here)
    if (blockIdx.x == 0 && threadIdx.x < kRegions) slot_clear[threadIdx.x * kRegionStride] = 0;
    // an overflowed previous level counts more pairs than it stored: read
    // only what the queue holds (the overflow flag makes the round restart)
    constexpr int NT = LevelShape<D>::block;
    if (sub_in == 1) {
        if (threadIdx.x == 0) {
            u32 p[kRegions + 1];
            region_prefix(slot_in, cap_in, p);
#pragma unroll
            for (int i = 0; i <= kRegions; ++i) pre[i] = p[i];
        }
    } else {
        seg_prefix(slot_in, cap_in, sub_in, pre);
    }
    __syncthreads();
    const u32 nq = pre[kRegions * sub_in];
    const int x = (int)(blockIdx.x % kRegions);
    const u32 j = blockIdx.x / kRegions, g = gridDim.x / kRegions;
    const u32 lo = (u32)((u64)nq * x / kRegions), hi = (u32)((u64)nq * (x + 1) / kRegions);
    if (lo + j * NT >= hi) return;
    u32* ctr[kLists] = {&r.cnt->c[C_TINY], nullptr, &r.cnt->c[C_BIG], &r.cnt->c[C_F], &r.cnt->c[C_FAR],
                        slot_next + x * kRegionStride};
    PairRec* qout = r.q + (size_t)x * r.cap_q;
    const double inf_ = __longlong_as_double(0x7ff0000000000000ll);
    LevelAcc acc = {inf_, inf_, inf_, 0, 0, 0};
    for (u32 v0 = lo + j * NT; v0 < hi; v0 += g * NT) {
        const u32 v = v0 + threadIdx.x;
        const bool have = v < hi;
        PairRec pr = {0u, 0u, 0.0};
        if (have) {
            u32 at;
            if (sub_in == 1) {
                u32 p[kRegions + 1];
#pragma unroll
                for (int i = 0; i <= kRegions; ++i) p[i] = pre[i];
                at = region_index(p, cap_in, v);
            } else {
                at = seg_index(pre, sub_in, cap_in, v);
            }
            pr = qin[at];
        }
        level_step<D>(t, r, hdb, have, pr, qout, r.cap_q, ctr, S, acc);
    }
    level_flush<NT>(r, acc);
}

// Many small levels without grid-wide launches: kRegions * sub_run
// workgroups, workgroup (x, w) = (blockIdx % 8, blockIdx / 8) expanding its
// own part of queue region x level by level (the level barrier is
// __syncthreads and the next queue's counter lives in LDS), so the thin
// levels of a round cost no kernel launches or host round trips.  With
// sub_run == 1 a workgroup owns region x; with sub_run == kSub it owns
// sub-segment w of region x.  A workgroup always takes its first level,
// then keeps going while its levels stay at most `small_max` pairs.
//
// Input: slot `slot_in` of the ring and buffer b_in, in layout sub_in (1 or
// kSub).  The first level reads the workgroup's share of region x: all of it
// (sub_run == 1, every sub-segment when sub_in == kSub), its own sub-segment
// (sub_in == sub_run == kSub), or the w-th kSub-th of the region's pairs
// (sub_in == 1, sub_run == kSub).  Levels are written to the workgroup's part
// of buffer b_out = b_in ^ 1 and, alternately, of a second buffer: b_in when
// the workgroup owns the whole region, else qt, so that no workgroup writes
// where another may still read its first level.  The remaining pairs end in
// the workgroup's part of b_out (copied there when the last level sits in the
// other buffer), in layout sub_run, with their counts in slot slot_in + 1 of
// the ring; slot slot_in + 2 is cleared for the grid-wide level that may
// follow, and slot_in is left alone (other workgroups of the region may still
// read it).  The remaining total is added to state[0], which is zero at
// launch.  Capacities are per region.
// 1024 threads where the level step fits 128 registers without spilling
// (d <= 4), else 768.
template <int D>
struct SmallBlock {
    static constexpr int value = D <= 4 ? 1024 : 768;
};

template <int D>
__global__ void __launch_bounds__(SmallBlock<D>::value) k_level_small(TreeView t, RoundArgs r, int hdb, PairRec* q0, u32 cap0,
                                                             PairRec* q1, u32 cap1, PairRec* qt, u32 capt, int b_in,
                                                             int sub_in, int sub_run, u32* ring, u32 slot_in,
                                                             u32 small_max, u32* state) {
    constexpr int NT = SmallBlock<D>::value;
    __shared__ BlockAlloc S;
    __shared__ u32 qn;
    const double inf_ = __longlong_as_double(0x7ff0000000000000ll);
    LevelAcc acc = {inf_, inf_, inf_, 0, 0, 0};
    const int x = (int)(blockIdx.x % kRegions), w = (int)(blockIdx.x / kRegions);
    const int b_out = b_in ^ 1;
    const u32 cap_in = b_in ? cap1 : cap0, cap_out = b_out ? cap1 : cap0;
    // the workgroup's parts of the output buffer and of the other buffer
    const u32 pcap = cap_out / (u32)sub_run;
    PairRec* const po = (b_out ? q1 : q0) + (size_t)x * cap_out + (size_t)w * pcap;
    const u32 ocap = (sub_run == 1 ? cap_in : capt) / (u32)sub_run;
    PairRec* const pt = sub_run == 1 ? (b_in ? q1 : q0) + (size_t)x * cap_in : qt + (size_t)x * capt + (size_t)w * ocap;
    // first-level input: npiece runs of pairs of buffer b_in (an overflowed
    // previous level counts more pairs than it stored)
    const u32* sl = ring + slot_in * kSlotWords + x * kRegionStride;
    const PairRec* qin = (b_in ? q1 : q0) + (size_t)x * cap_in;
    const int npiece = (sub_run == 1 && sub_in == kSub) ? kSub : 1;
    const u32 icap = cap_in / (u32)sub_in;
    u32 nq = 0;
    for (int k = 0; k < npiece; ++k) nq += min(sl[npiece > 1 ? k : (sub_in == kSub ? w : 0)], icap);
    bool first = true, in_po = false;
    while (nq > 0 && (first || nq <= small_max)) {
        if (threadIdx.x == 0) qn = 0;
        __syncthreads();
        u32* ctr[kLists] = {&r.cnt->c[C_TINY], nullptr, &r.cnt->c[C_BIG], &r.cnt->c[C_F], &r.cnt->c[C_FAR], &qn};
        // level 1 goes to po, then the levels alternate
        PairRec* const dst = (first || !in_po) ? po : pt;
        const u32 dcap = (first || !in_po) ? pcap : ocap;
        if (first) {
            for (int k = 0; k < npiece; ++k) {
                const PairRec* src;
                u32 c0, c1;
                if (npiece > 1) {  // every sub-segment of region x
                    src = qin + (size_t)k * icap;
                    c0 = 0;
                    c1 = min(sl[k], icap);
                } else if (sub_in == kSub) {  // own sub-segment
                    src = qin + (size_t)w * icap;
                    c0 = 0;
                    c1 = min(sl[w], icap);
                } else {  // the w-th share of the region (the whole region when sub_run == 1)
                    const u32 c = min(sl[0], icap);
                    src = qin;
                    c0 = (u32)((u64)c * (u32)w / (u32)sub_run);
                    c1 = (u32)((u64)c * (u32)(w + 1) / (u32)sub_run);
                }
                for (u32 b0 = c0; b0 < c1; b0 += NT) {
                    const u32 v = b0 + threadIdx.x;
                    const bool have = v < c1;
                    PairRec pr = {0u, 0u, 0.0};
                    if (have) pr = src[v];
                    level_step<D>(t, r, hdb, have, pr, dst, dcap, ctr, S, acc);
                }
            }
        } else {
            const PairRec* src = in_po ? po : pt;
            for (u32 b0 = 0; b0 < nq; b0 += NT) {
                const u32 v = b0 + threadIdx.x;
                const bool have = v < nq;
                PairRec pr = {0u, 0u, 0.0};
                if (have) pr = src[v];
                level_step<D>(t, r, hdb, have, pr, dst, dcap, ctr, S, acc);
            }
        }
        __syncthreads();
        const u32 nn = qn;
        first = false;
        in_po = dst == po;
        if (nn > dcap) {  // overflowed (flagged): stop, the round restarts
            nq = 0;
            break;
        }
        nq = nn;
        __syncthreads();
    }
    // leave the remaining pairs in the workgroup's part of b_out
    if (nq && !in_po) {
        if (nq > pcap) {
            if (threadIdx.x == 0) flag_overflow_q(r.cnt);
            nq = 0;
        }
        for (u32 v = threadIdx.x; v < nq; v += NT) po[v] = pt[v];
    }
    level_flush<NT>(r, acc);
    if (threadIdx.x == 0) {
        ring[((slot_in + 1) % kQRing) * kSlotWords + x * kRegionStride + w] = nq;
        ring[((slot_in + 2) % kQRing) * kSlotWords + x * kRegionStride + w] = 0u;
        if (nq) atomicAdd(&state[0], nq);
    }
}

// ------------------------------------------------------------ small pairs
// ------------------------------------------------------------ GetRho
// Threshold of the cardinality schedules (Alg. 3 GetRho; rho_hi of Alg. 2):
// the smallest weight lower bound over the well-separated pairs that descend
// from the waiting pairs, have |A| + |B| > beta_card and are not connected.
// One breadth-first level, one pair per lane: a pair is dropped when its
// nodes are connected, when |A| + |B| <= beta_card (every descendant is at
// most as large) or when its bound is not below the current rho (no
// descendant can lower it); a separated pair lowers rho; otherwise the node
// with the larger sphere is split and the child pairs that pass the same
// tests go to the next level (at most two per input, so `out` holds 2 nin).
template <int D>
__global__ void __launch_bounds__(kBlock) k_rho_level(TreeView t, int hdb, int mutual, double sep, const PairRec* in,
                                                      u32 nin, PairRec* out, u32* nout, u32 beta_card, u64* rho) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    const NodeRec<D>* N = nodes_of<D>(t);
    const double2 z = make_double2(0.0, 0.0);
    bool push0 = false, push1 = false;
    PairRec c0, c1;
    if (i < nin) {
        const PairRec p = in[i];
        const NodeRec<D> A = N[p.a], B = N[p.b];
        const double cur = bitsd(__hip_atomic_load(rho, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const bool conn = A.comp >= 0 && A.comp == B.comp;
        const double2 ca = hdb ? node_cd<D>(t, A, p.a) : z, cb = hdb ? node_cd<D>(t, B, p.b) : z;
        const double lb = pair_wlb2<D>(A, B, hdb, ca, cb);
        if (!conn && (u64)A.count + (u64)B.count > (u64)beta_card && lb < cur) {
            const double dA = box_diag2<D>(A), dB = box_diag2<D>(B);
            if (well_separated<D>(A, B, hdb && mutual, ca, cb, sep, dA, dB, t, p.a, p.b)) {
                atomicMin((unsigned long long*)rho, (unsigned long long)dbits(lb));
            } else {
                const bool split_a = (B.count == 1) || (A.count > 1 && (dA > dB || (dA == dB && A.count >= B.count)));
                const NodeRec<D>& X = split_a ? A : B;
                const NodeRec<D>& O = split_a ? B : A;
                const u32 oth = split_a ? p.b : p.a;
                const double2 co = split_a ? cb : ca;
                const int2 ch = node_kids(t.n, X.first, X.count, X.split);
                const NodeRec<D> C0 = N[ch.x], C1 = N[ch.y];
                const double2 k0 = hdb ? node_cd<D>(t, C0, (u32)ch.x) : z, k1 = hdb ? node_cd<D>(t, C1, (u32)ch.y) : z;
                c0.a = (u32)ch.x;
                c0.b = oth;
                c0.lb2 = pair_wlb2<D>(C0, O, hdb, k0, co);
                c1.a = (u32)ch.y;
                c1.b = oth;
                c1.lb2 = pair_wlb2<D>(C1, O, hdb, k1, co);
                push0 = !(C0.comp >= 0 && C0.comp == O.comp) && (u64)C0.count + (u64)O.count > (u64)beta_card &&
                        c0.lb2 < cur;
                push1 = !(C1.comp >= 0 && C1.comp == O.comp) && (u64)C1.count + (u64)O.count > (u64)beta_card &&
                        c1.lb2 < cur;
            }
        }
    }
    const u32 s0 = wave_append(nout, push0);
    if (push0) out[s0] = c0;
    const u32 s1 = wave_append(nout, push1);
    if (push1) out[s1] = c1;
}

__global__ void k_set_u64(u64* p, u64 v) { *p = v; }

// BCCP (or BCCP*) of the separated pairs with at most kTinyEvals point pairs,
// queued by the level steps: one pair per thread, kTinyItems pairs per
// thread per block step, by brute force over the point pairs.  The edge goes
// to the committed list when its weight is within beta, else to the pool.
constexpr int kTinyBlock = 256;
constexpr int kTinyItems = 2;
constexpr int kTinyTile = kTinyItems * kTinyBlock;
constexpr int kTinyGrid = 1024;

template <int D>
__global__ void __launch_bounds__(kTinyBlock) k_tiny_bccp(TreeView t, RoundArgs r, int hdb, const uint4* tiny,
                                                          u32 ntiny) {
    __shared__ BlockAlloc S;
    __shared__ double shm[kTinyBlock / kWave];
    __shared__ unsigned long long shs[kTinyBlock / kWave];
    u32* ctr[kLists] = {&r.cnt->c[C_C], &r.cnt->c[C_P], nullptr, nullptr, nullptr, nullptr};
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    double minp = inf;
    unsigned long long evals = 0, solved = 0;
    for (u32 b0 = blockIdx.x * kTinyTile; b0 < ntiny; b0 += gridDim.x * kTinyTile) {
        EdgeOut e[kTinyItems];
        u32 cls = 0, nc = 0, np = 0;
#pragma unroll
        for (int k = 0; k < kTinyItems; ++k) {
            const u32 i = b0 + k * kTinyBlock + threadIdx.x;
            if (i < ntiny) {
                const uint4 q = tiny[i];
                const u32 ca = q.z >> 16, cb = q.z & 0xffffu;
                // minimum of (w2, e2); the identifiers are read only to break
                // an exact tie of both, and once for the winner
                double bw = inf, be = inf;
                u32 bx = q.x, by = q.y;
                for (u32 x = q.x; x < q.x + ca; ++x)
                    for (u32 y = q.y; y < q.y + cb; ++y) {
                        double w2, e2;
                        point_w2<D>(t, hdb, x, y, w2, e2);
                        bool better = w2 < bw || (w2 == bw && e2 < be);
                        if (w2 == bw && e2 == be)
                            better = key_less(point_edge<D>(t, hdb, x, y).k, point_edge<D>(t, hdb, bx, by).k);
                        if (better) {
                            bw = w2;
                            be = e2;
                            bx = x;
                            by = y;
                        }
                    }
                e[k] = point_edge<D>(t, hdb, bx, by);
                evals += (unsigned long long)ca * cb;
                ++solved;
                const bool in = e[k].k.w2 <= r.beta2;
                cls |= (in ? 1u : 2u) << (2 * k);
                nc += in;
                np += !in;
                if (!in) minp = fmin(minp, e[k].k.w2);
            }
        }
        u32 cnt[kLists] = {nc, np, 0u, 0u, 0u, 0u};
        u32 off[kLists];
        block_alloc(S, cnt, ctr, off);
#pragma unroll
        for (int k = 0; k < kTinyItems; ++k) {
            const u32 c = (cls >> (2 * k)) & 3u;
            if (c == 1u) {
                if (off[0] < r.cap_c) put_edge(r.c, off[0], e[k]);
                else flag_overflow(r.cnt);
                ++off[0];
            } else if (c == 2u) {
                if (off[1] < r.cap_p) put_edge(r.pout, off[1], e[k]);
                else flag_overflow(r.cnt);
                ++off[1];
            }
        }
    }
    block_atomic_min(minp, &r.cnt->m[M_P], shm);
    const unsigned long long ev = block_sum_u64(evals, shs);
    const unsigned long long so = block_sum_u64(solved, shs);
    if (threadIdx.x == 0 && so) {
        atomicAdd(&r.cnt->c64[C64_EVALS], ev);
        atomicAdd(&r.cnt->c64[C64_BCCP], so);
    }
}

// ------------------------------------------------------------ large pairs
// A large separated pair is cut into tasks of up to kBigA points of the
// larger node (kBigAPL per lane) by up to bchunk points of the other (a
// multiple of 64, a launch parameter); one wave
// per task.  B points are staged in LDS 64 at a time (double-buffered: the
// next block is loaded into registers while the current one is used) and
// broadcast to all lanes.  The inner loop keeps only the running minimum
// weight per A point, plus the 64-point block where it was reached and
// whether a later block tied it; the exact key (w2, e2, ids) is then resolved
// by the whole wave rescanning only that block (or the task's whole B range
// after a tie) for each A point that holds the wave minimum.  Per-task
// partial keys are reduced per pair afterwards, one wave per pair.
//
// For BCCP* the weight max(cd(a), cd(b), d) is minimised over b as
// max(cd(a), min_b max(cd(b), d)), which is the same value (max with a
// constant is monotone) at one max per distance instead of two.
constexpr int kBigAPL = 4;
constexpr int kBigA = 64 * kBigAPL;
constexpr int kBigBDefault = 2048;
constexpr int kMidMax = 4096;  // pairs up to this many point pairs: one wave, flattened products
constexpr int kThinA = 4096;   // thin pairs (smaller side <= 64 points): A points per task

struct PartKey {
    double w2, e2;
    u64 ids, pos;
};

template <int D>
__device__ __forceinline__ void big_orient(const TreeView& t, uint2 pr, int2& ra, int2& rb) {
    const NodeRec<D>* N = nodes_of<D>(t);
    ra = make_int2(N[pr.x].first, N[pr.x].count);
    rb = make_int2(N[pr.y].first, N[pr.y].count);
    if (rb.y > ra.y) {
        int2 x = ra;
        ra = rb;
        rb = x;
    }
}

template <int D>
// Task count of every large pair; the pairs' distance evaluations and task
// totals are summed per block (one atomic per block and counter: the tasks
// themselves add nothing to shared counters).
__global__ void __launch_bounds__(kBlock) k_big_ntasks(TreeView t, const uint2* big, u32 nbig, u32* ntask,
                                                       int bchunk, Counters* cnt) {
    __shared__ unsigned long long sh[kBlock / kWave];
    u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    u64 c = 0, work = 0;
    if (i < nbig) {
        int2 ra, rb;
        big_orient<D>(t, big[i], ra, rb);
        work = (u64)ra.y * (u64)rb.y;
        c = work <= (u64)kMidMax ? 1ull
            : rb.y <= 64         ? (u64)((ra.y + kThinA - 1) / kThinA)
                                 : (u64)((ra.y + kBigA - 1) / kBigA) * (u64)((rb.y + bchunk - 1) / bchunk);
        ntask[i] = c < (1ull << 31) ? (u32)c : 1u;
    }
    const unsigned long long sc = block_sum_u64(c, sh);
    const unsigned long long sw = block_sum_u64(work, sh);
    if (threadIdx.x == 0) {
        atomicAdd(&cnt->c64[C64_TASKS], sc);  // the host rejects totals beyond 2^31
        atomicAdd(&cnt->c64[C64_EVALS], sw);
        atomicAdd(&cnt->c64[C64_BIGWORK], sw);
    }
}

// Box of every aligned 64-point block of sorted positions [64 i, 64 i + 64):
// bb[i * (2D + 1) + k] = min coordinate k, [.. + D + k] = max, [.. + 2D] =
// smallest squared core distance (0 for EMST).  Computed once per solve; a
// large-pair task bounds a B block by the boxes of the (at most two) aligned
// blocks that cover it, so a block it skips costs two box reads and no point
// loads.
template <int D>
__global__ void __launch_bounds__(kBlock) k_block_boxes(TreeView t, int hdb, double* bb) {
    const u32 b = blockIdx.x * blockDim.x + threadIdx.x;
    const u32 nb = (u32)((t.n + 63) / 64);
    if (b >= nb) return;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    double lo[D], hi[D], cm = inf;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = inf;
        hi[k] = -inf;
    }
    const u32 j0 = b * 64, j1 = min(j0 + 64, (u32)t.n);
    for (u32 j = j0; j < j1; ++j) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double x = t.X[(size_t)j * D + k];
            lo[k] = fmin(lo[k], x);
            hi[k] = fmax(hi[k], x);
        }
        if (hdb) cm = fmin(cm, t.cd2[j]);
    }
    double* o = bb + (size_t)b * (2 * D + 1);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        o[k] = lo[k];
        o[D + k] = hi[k];
    }
    o[2 * D] = hdb ? cm : 0.0;
}

// Pruning: a 64-point B block is skipped when the bound between the task's
// A points' box and the block's box exceeds the best weight seen so far, by
// this task or (through `ubest`, the bit patterns of each pair's best weight,
// all ones before the launch) by any task of the same pair.  The bound is the
// squared box gap summed in the distances' operation order (and for BCCP* the
// smallest core distances on either side), so it never exceeds a computed
// weight of the block: a skipped block holds no pair at or below the pair's
// final minimum.
template <int D, int HDB>
__global__ void __launch_bounds__(64) k_big_bccp(TreeView t, const uint2* big, u32 nbig, const u32* toff,
                                                  PartKey* part, Counters* cnt, int bchunk, u64* ubest,
                                                  u32* tdone, const double* bb) {
    __shared__ double sbuf[2][64 * D];
    __shared__ double scd[2][64];
    __shared__ u32 sorig[64];
    const int lane = lane_id();
    const u32 task = blockIdx.x;
    // pair owning this task: last i with toff[i] <= task
    u32 lo = 0, hi = nbig - 1;
    while (lo < hi) {
        u32 mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= task) lo = mid;
        else hi = mid - 1;
    }
    int2 ra, rb;
    big_orient<D>(t, big[lo], ra, rb);
    if ((u64)ra.y * (u64)rb.y <= (u64)kMidMax) {
        // medium pair: |B|^2 <= |A||B| <= kMidMax, so B (the smaller node)
        // fits one 64-row LDS tile.  Each lane takes A points in turn and
        // runs over the staged B rows comparing (w2, e2); the ids are read
        // (from the staged copy) only to break an exact tie of both.
        const u32 nb = (u32)rb.y, tot = (u32)ra.y * nb;
        if (lane < (int)nb) {
            const u32 j = (u32)rb.x + (u32)lane;
#pragma unroll
            for (int k = 0; k < D; ++k) sbuf[0][lane * D + k] = t.X[(size_t)j * D + k];
            scd[0][lane] = HDB ? t.cd2[j] : 0.0;
            sorig[lane] = t.orig[j];
        }
        __syncthreads();
        EdgeOut best;
        best.k = key_none();
        best.i = best.j = kNone;
        for (u32 ia = (u32)lane; ia < (u32)ra.y; ia += kWave) {
            const u32 i = (u32)ra.x + ia;
            double a[D];
#pragma unroll
            for (int k = 0; k < D; ++k) a[k] = t.X[(size_t)i * D + k];
            const double cda = HDB ? t.cd2[i] : 0.0;
            const u32 oa = t.orig[i];
            double bw = __longlong_as_double(0x7ff0000000000000ll), be = bw;
            u32 bj = 0;
            for (u32 jb = 0; jb < nb; ++jb) {
                double e2 = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double x = a[k] - sbuf[0][jb * D + k];
                    e2 = e2 + x * x;
                }
                const double w2 = HDB ? fmax(fmax(cda, scd[0][jb]), e2) : e2;
                bool better = w2 < bw || (w2 == bw && e2 < be);
                if (w2 == bw && e2 == be) {
                    const u32 ob = sorig[jb], oc = sorig[bj];
                    const u32 lo1 = min(oa, ob), hi1 = max(oa, ob), lo0 = min(oa, oc), hi0 = max(oa, oc);
                    better = lo1 < lo0 || (lo1 == lo0 && hi1 < hi0);
                }
                if (better) {
                    bw = w2;
                    be = e2;
                    bj = jb;
                }
            }
            EdgeOut c = point_edge<D>(t, HDB, i, (u32)rb.x + bj);
            if (key_less(c.k, best.k)) best = c;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            EdgeOut w;
            w.k.w2 = __shfl_xor(best.k.w2, o);
            w.k.e2 = __shfl_xor(best.k.e2, o);
            w.k.lo = __shfl_xor(best.k.lo, o);
            w.k.hi = __shfl_xor(best.k.hi, o);
            w.i = __shfl_xor(best.i, o);
            w.j = __shfl_xor(best.j, o);
            if (key_less(w.k, best.k)) best = w;
        }
        if (lane == 0) {
            PartKey pk;
            pk.w2 = best.k.w2;
            pk.e2 = best.k.e2;
            pk.ids = ((u64)best.k.lo << 32) | best.k.hi;
            pk.pos = ((u64)best.i << 32) | best.j;
            part[task] = pk;
            tdone[task] = tot;
        }
        return;
    }
    if (rb.y <= 64) {
        // Thin pair: B (at most 64 points) staged in LDS with its ids, the
        // task's A range (up to kThinA points) streamed in aligned 64-point
        // blocks, one A point per lane against every B row.  The block whose
        // box is nearest to B's box is evaluated first; every other block is
        // skipped when its bound (from the precomputed block boxes) exceeds
        // the best weight of this task or of the pair (shared through ubest).
        const double inf = __longlong_as_double(0x7ff0000000000000ll);
        const u32 nb = (u32)rb.y;
        const int a0 = ra.x + (int)(task - toff[lo]) * kThinA, a1 = min(a0 + kThinA, ra.x + ra.y);
        double blo[D], bhi[D], bcm = inf;
        if (lane < (int)nb) {
            const u32 j = (u32)rb.x + (u32)lane;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double x = t.X[(size_t)j * D + k];
                sbuf[0][lane * D + k] = x;
                blo[k] = x;
                bhi[k] = x;
            }
            const double c = HDB ? t.cd2[j] : 0.0;
            scd[0][lane] = c;
            bcm = c;
            sorig[lane] = t.orig[j];
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                blo[k] = inf;
                bhi[k] = -inf;
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            blo[k] = wave_uniform_f64(wave_min_f64(blo[k]));
            bhi[k] = wave_uniform_f64(-wave_min_f64(-bhi[k]));
        }
        if (HDB) bcm = wave_uniform_f64(wave_min_f64(bcm));
        __syncthreads();
        auto thin_bound = [&](u32 bi) -> double {
            const double* o = bb + (size_t)bi * (2 * D + 1);
            double g2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double g = fmax(fmax(o[k] - bhi[k], blo[k] - o[D + k]), 0.0);
                g2 = g2 + g * g;
            }
            if (HDB) g2 = fmax(g2, fmax(bcm, o[2 * D]));
            return g2;
        };
        EdgeOut best;
        best.k = key_none();
        best.i = best.j = kNone;
        u32 done = 0;
        // one 64-point block: lane l takes A point 64 bi + l (inside [a0, a1))
        auto eval_point = [&](int i, const double (&a)[D], double cda, u32 oa) -> double {
            double bw = inf, be = inf;
            u32 bj = 0;
            for (u32 jb = 0; jb < nb; ++jb) {
                double e2 = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double x = a[k] - sbuf[0][jb * D + k];
                    e2 = e2 + x * x;
                }
                const double w2 = HDB ? fmax(fmax(cda, scd[0][jb]), e2) : e2;
                bool better = w2 < bw || (w2 == bw && e2 < be);
                if (w2 == bw && e2 == be) {
                    const u32 ob = sorig[jb], oc = sorig[bj];
                    const u32 lo1 = min(oa, ob), hi1 = max(oa, ob), lo0 = min(oa, oc), hi0 = max(oa, oc);
                    better = lo1 < lo0 || (lo1 == lo0 && hi1 < hi0);
                }
                if (better) {
                    bw = w2;
                    be = e2;
                    bj = jb;
                }
            }
            // the point's best key, from the values just computed (the same
            // operations as point_edge)
            EdgeOut c;
            const u32 ob = sorig[bj];
            c.k.w2 = bw;
            c.k.e2 = be;
            c.k.lo = min(oa, ob);
            c.k.hi = max(oa, ob);
            c.i = (u32)i;
            c.j = (u32)rb.x + bj;
            if (key_less(c.k, best.k)) best = c;
            return bw;
        };
        // up to four blocks at once: every lane issues its four A-point loads
        // before any distance, so the load latencies overlap
        auto eval_blocks = [&](const u32 (&bis)[4], int nbk) -> double {
            double a[4][D], cda[4];
            u32 oa[4];
            bool in[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = (int)(bis[q] * 64u) + lane;
                in[q] = q < nbk && i >= a0 && i < a1;
                const int ic = in[q] ? i : a0;
#pragma unroll
                for (int k = 0; k < D; ++k) a[q][k] = t.X[(size_t)ic * D + k];
                cda[q] = HDB ? t.cd2[ic] : 0.0;
                oa[q] = t.orig[ic];
            }
            double wl = inf;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (in[q]) wl = fmin(wl, eval_point((int)(bis[q] * 64u) + lane, a[q], cda[q], oa[q]));
                if (q < nbk) done += (u32)(min(a1, (int)(bis[q] * 64u) + 64) - max(a0, (int)(bis[q] * 64u))) * nb;
            }
            return wave_uniform_f64(wave_min_f64(wl));
        };
        // A task covers at most kThinA / 64 + 1 = 65 aligned blocks: lane l
        // holds the bounds of blocks ib0 + l and ib0 + 64 + l in registers
        static_assert(kThinA <= 64 * 64, "two blocks per lane");
        const u32 ib0 = (u32)a0 >> 6, ib1 = (u32)(a1 - 1) >> 6;
        const u32 bl0 = ib0 + (u32)lane, bl1 = ib0 + 64u + (u32)lane;
        const double g0 = bl0 <= ib1 ? thin_bound(bl0) : inf, g1 = bl1 <= ib1 ? thin_bound(bl1) : inf;
        // nearest block first (smallest bound; ties to the lower block)
        double lbm = g0;
        u32 lbi = bl0;
        if (g1 < lbm) {
            lbm = g1;
            lbi = bl1;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double g = __shfl_xor(lbm, o);
            const u32 b2 = __shfl_xor(lbi, o);
            if (g < lbm || (g == lbm && b2 < lbi)) {
                lbm = g;
                lbi = b2;
            }
        }
        const u32 first_bi = (u32)__builtin_amdgcn_readfirstlane((int)lbi);
        const u32 fb[4] = {first_bi, first_bi, first_bi, first_bi};
        double mt = eval_blocks(fb, 1);
        u64 ub = ubest[lo];
        if (dbits(mt) < ub && lane == 0) atomicMin((unsigned long long*)&ubest[lo], (unsigned long long)dbits(mt));
        // then the blocks still within the best weight, in order; the masks
        // are re-taken against the best after every block
        u64 left0 = __ballot(bl0 <= ib1 && bl0 != first_bi), left1 = __ballot(bl1 <= ib1 && bl1 != first_bi);
        while (true) {
            const double lim = fmin(mt, __longlong_as_double((long long)ub));
            left0 &= __ballot(!(g0 > lim));
            left1 &= __ballot(!(g1 > lim));
            if (!left0 && !left1) break;
            u32 bis[4] = {0, 0, 0, 0};
            int nbk = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (left0) {
                    const int l = __ffsll((long long)left0) - 1;
                    left0 &= left0 - 1;
                    bis[q] = ib0 + (u32)l;
                    ++nbk;
                } else if (left1) {
                    const int l = __ffsll((long long)left1) - 1;
                    left1 &= left1 - 1;
                    bis[q] = ib0 + 64u + (u32)l;
                    ++nbk;
                }
            }
            const double w = eval_blocks(bis, nbk);
            if (w < mt) {
                mt = w;
                if (dbits(mt) < ub && lane == 0)
                    atomicMin((unsigned long long*)&ubest[lo], (unsigned long long)dbits(mt));
            }
            ub = ubest[lo];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            EdgeOut w;
            w.k.w2 = __shfl_xor(best.k.w2, o);
            w.k.e2 = __shfl_xor(best.k.e2, o);
            w.k.lo = __shfl_xor(best.k.lo, o);
            w.k.hi = __shfl_xor(best.k.hi, o);
            w.i = __shfl_xor(best.i, o);
            w.j = __shfl_xor(best.j, o);
            if (key_less(w.k, best.k)) best = w;
        }
        if (lane == 0) {
            PartKey pk;
            pk.w2 = best.k.w2;
            pk.e2 = best.k.e2;
            pk.ids = ((u64)best.k.lo << 32) | best.k.hi;
            pk.pos = ((u64)best.i << 32) | best.j;
            part[task] = pk;
            tdone[task] = done;
        }
        return;
    }
    u32 local = task - toff[lo];
    int nbt = (rb.y + bchunk - 1) / bchunk;
    int ta = (int)(local / (u32)nbt), tb = (int)(local % (u32)nbt);
    const int aend = ra.x + ra.y;
    const int abase = ra.x + ta * kBigA;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    double p[kBigAPL][D], ca[kBigAPL], m[kBigAPL];
    int blk[kBigAPL];
    bool tie[kBigAPL];
#pragma unroll
    for (int r = 0; r < kBigAPL; ++r) {
        int ai = abase + r * 64 + lane;
        int aic = ai < aend ? ai : ra.x;
#pragma unroll
        for (int k = 0; k < D; ++k) p[r][k] = t.X[(size_t)aic * D + k];
        ca[r] = HDB ? t.cd2[aic] : 0.0;
        m[r] = inf;
        tie[r] = false;
    }
    const int jb0 = rb.x + tb * bchunk;
    const int jb1 = min(jb0 + bchunk, rb.x + rb.y);
#pragma unroll
    for (int r = 0; r < kBigAPL; ++r) blk[r] = jb0;
    // box (and smallest core distance) of the task's A points; a task with
    // a single B block has nothing to prune and skips this
    const bool multi = jb1 - jb0 > 64;
    double alo[D], ahi[D], acm = inf;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        alo[k] = inf;
        ahi[k] = -inf;
    }
    if (multi) {
#pragma unroll
        for (int r = 0; r < kBigAPL; ++r)
            if (abase + r * 64 + lane < aend) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    alo[k] = fmin(alo[k], p[r][k]);
                    ahi[k] = fmax(ahi[k], p[r][k]);
                }
                if (HDB) acm = fmin(acm, ca[r]);
            }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            alo[k] = wave_uniform_f64(wave_min_f64(alo[k]));
            ahi[k] = wave_uniform_f64(-wave_min_f64(-ahi[k]));
        }
        if (HDB) acm = wave_uniform_f64(wave_min_f64(acm));
    }
    // bound between the A box and the B block [js, js + cnt): the smaller
    // of the bounds to the aligned blocks covering it (a bound to a union is
    // the smaller bound); every lane computes the same value from the same
    // box words
    auto box_bound = [&](u32 bi) -> double {
        const double* o = bb + (size_t)bi * (2 * D + 1);
        double g2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double g = fmax(fmax(o[k] - ahi[k], alo[k] - o[D + k]), 0.0);
            g2 = g2 + g * g;
        }
        if (HDB) g2 = fmax(g2, fmax(acm, o[2 * D]));
        return g2;
    };
    auto block_bound = [&](int js, int cnt) -> double {
        const u32 b0 = (u32)js >> 6, b1 = (u32)(js + cnt - 1) >> 6;
        const double x = box_bound(b0);
        return b1 != b0 ? fmin(x, box_bound(b1)) : x;
    };
    u64 ub = ubest[lo];
    double blb = multi ? block_bound(jb0, min(64, jb1 - jb0)) : 0.0;
    // stage the first block unless it is already known to be pruned
    const bool h0 = lane < jb1 - jb0 && !(blb > __longlong_as_double((long long)ub));
    if (h0) {
#pragma unroll
        for (int k = 0; k < D; ++k) sbuf[0][lane * D + k] = t.X[(size_t)(jb0 + lane) * D + k];
        if (HDB) scd[0][lane] = t.cd2[jb0 + lane];
    }
    // every load above has landed: keeps the compiler from placing waits for
    // them inside the inner loop, where they would also wait for the prefetch
    __builtin_amdgcn_s_waitcnt(0);
    double mt = inf;  // this task's best weight so far
    const u32 na_task = (u32)min(kBigA, aend - abase);
    u32 done = 0;     // distances evaluated
    __syncthreads();
    int buf = 0;
    for (int js = jb0; js < jb1; js += 64, buf ^= 1) {
        const int cntb = min(64, jb1 - js);
        // prefetch the next block (and the pair's best weight) into
        // registers, unless its bound already exceeds the best weight known
        // (the best only decreases, so it would be skipped anyway)
        const int jn = js + 64;
        const double nblb = (multi && jn < jb1) ? block_bound(jn, min(64, jb1 - jn)) : 0.0;
        const bool hn = jn < jb1 && lane < jb1 - jn && !(nblb > fmin(mt, __longlong_as_double((long long)ub)));
        double nx[D] = {}, ncd = inf;
        if (hn) {
#pragma unroll
            for (int k = 0; k < D; ++k) nx[k] = t.X[(size_t)(jn + lane) * D + k];
            if (HDB) ncd = t.cd2[jn + lane];
        }
        const u64 ubn = ubest[lo];
        const bool skip = blb > fmin(mt, __longlong_as_double((long long)ub));
        double bm[kBigAPL];
#pragma unroll
        for (int r = 0; r < kBigAPL; ++r) bm[r] = inf;
        const double* sb = sbuf[buf];
#pragma unroll 4
        for (int j = 0; j < (skip ? 0 : cntb); ++j) {
            double q[D];
#pragma unroll
            for (int k = 0; k < D; ++k) q[k] = sb[j * D + k];
            const double cb = HDB ? scd[buf][j] : 0.0;
            // dimension-major, so that the kBigAPL independent sums
            // interleave (each still adds its terms in dimension order)
            double d2[kBigAPL];
#pragma unroll
            for (int r = 0; r < kBigAPL; ++r) {
                double x = p[r][0] - q[0];
                d2[r] = x * x;
            }
#pragma unroll
            for (int k = 1; k < D; ++k)
#pragma unroll
                for (int r = 0; r < kBigAPL; ++r) {
                    double x = p[r][k] - q[k];
                    d2[r] = d2[r] + x * x;
                }
#pragma unroll
            for (int r = 0; r < kBigAPL; ++r) {
                if (HDB) d2[r] = fmax(cb, d2[r]);
                bm[r] = fmin(bm[r], d2[r]);
            }
        }
        if (!skip) {
            done += (u32)cntb * na_task;
            double mm = inf;
#pragma unroll
            for (int r = 0; r < kBigAPL; ++r) {
                double w = HDB ? fmax(ca[r], bm[r]) : bm[r];
                if (w < m[r]) {
                    m[r] = w;
                    blk[r] = js;
                    tie[r] = false;
                } else if (w == m[r]) {
                    tie[r] = true;
                }
                if (abase + r * 64 + lane < aend) mm = fmin(mm, m[r]);
            }
            mm = wave_uniform_f64(wave_min_f64(mm));
            if (mm < mt) {
                mt = mm;
                // shared only by tasks with several blocks (whose later blocks
                // can use it) and only when it beats the last bound read:
                // pairs cut into many one-block tasks would otherwise queue
                // an atomic per task on one address
                if (multi && dbits(mt) < ub && lane == 0)
                    atomicMin((unsigned long long*)&ubest[lo], (unsigned long long)dbits(mt));
            }
        }
        if (hn) {
#pragma unroll
            for (int k = 0; k < D; ++k) sbuf[buf ^ 1][lane * D + k] = nx[k];
            if (HDB) scd[buf ^ 1][lane] = ncd;
        }
        blb = nblb;
        ub = ubn;
        __syncthreads();
    }
    double mm = inf;
#pragma unroll
    for (int r = 0; r < kBigAPL; ++r)
        if (abase + r * 64 + lane < aend) mm = fmin(mm, m[r]);
    const double M = wave_min_f64(mm);
    // exact key: for each A point at the minimum, the wave rescans the block
    // where it was reached (the whole B range after a tie)
    EdgeOut best;
    best.k = key_none();
    best.i = best.j = kNone;
#pragma unroll
    for (int r = 0; r < kBigAPL; ++r) {
        const int ai = abase + r * 64 + lane;
        u64 mask = __ballot(ai < aend && m[r] == M);
        while (mask) {
            const int c = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            const int a = __shfl(ai, c);
            const int s0 = __shfl(tie[r] ? jb0 : blk[r], c);
            const int s1 = __shfl(tie[r] ? jb1 : min(blk[r] + 64, jb1), c);
            for (int j = s0 + lane; j < s1; j += 64) {
                EdgeOut e = point_edge<D>(t, HDB, (u32)a, (u32)j);
                if (key_less(e.k, best.k)) best = e;
            }
        }
    }
    // wave minimum of the exact keys (carrying the positions)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        EdgeOut w;
        w.k.w2 = __shfl_xor(best.k.w2, o);
        w.k.e2 = __shfl_xor(best.k.e2, o);
        w.k.lo = __shfl_xor(best.k.lo, o);
        w.k.hi = __shfl_xor(best.k.hi, o);
        w.i = __shfl_xor(best.i, o);
        w.j = __shfl_xor(best.j, o);
        if (key_less(w.k, best.k)) best = w;
    }
    if (lane == 0) {
        PartKey pk;
        pk.w2 = best.k.w2;
        pk.e2 = best.k.e2;
        pk.ids = ((u64)best.k.lo << 32) | best.k.hi;
        pk.pos = ((u64)best.i << 32) | best.j;
        part[task] = pk;
        tdone[task] = done;
    }
}

__device__ __forceinline__ bool part_less(const PartKey& x, const PartKey& b) {
    return (x.w2 != b.w2) ? (x.w2 < b.w2) : (x.e2 != b.e2) ? (x.e2 < b.e2) : (x.ids < b.ids);
}

// Per pair, the minimum of its task keys, written into the pair's first
// task slot; one wave per pair.
__global__ void __launch_bounds__(kBlock) k_big_reduce(u32 nbig, const u32* toff, const u32* ntask, PartKey* part,
                                                        const u32* tdone, unsigned long long* pdone) {
    const int lane = lane_id();
    const u32 i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (i >= nbig) return;
    const u32 o = toff[i], c = ntask[i];
    if (c == 1) {
        if (lane == 0) pdone[i] = tdone[o];
        return;
    }
    PartKey b;
    b.w2 = b.e2 = __longlong_as_double(0x7ff0000000000000ll);
    b.ids = ~0ull;
    b.pos = 0;
    unsigned long long dn = 0;
    for (u32 k = (u32)lane; k < c; k += kWave) {
        PartKey x = part[o + k];
        if (part_less(x, b)) b = x;
        dn += tdone[o + k];
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) dn += __shfl_xor(dn, s);
    if (lane == 0) pdone[i] = dn;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        PartKey x;
        x.w2 = __shfl_xor(b.w2, s);
        x.e2 = __shfl_xor(b.e2, s);
        x.ids = __shfl_xor(b.ids, s);
        x.pos = __shfl_xor(b.pos, s);
        if (part_less(x, b)) b = x;
    }
    if (lane == 0) part[o] = b;
}

// Commits or defers each large pair's BCCP edge (its key is in the pair's
// first task slot after k_big_reduce).
__global__ void __launch_bounds__(kBlock) k_big_combine(RoundArgs r, u32 nbig, const u32* toff,
                                                        const PartKey* part, const unsigned long long* pdone) {
    __shared__ BlockAlloc S;
    __shared__ double shm[4];
    __shared__ unsigned long long shs[kBlock / kWave];
    unsigned long long dn = 0;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    u32* ctr[kLists] = {&r.cnt->c[C_C], &r.cnt->c[C_P], nullptr, nullptr, nullptr, nullptr};
    double minp = inf;
    for (u32 b0 = blockIdx.x * kBlock; b0 < nbig; b0 += gridDim.x * kBlock) {
        u32 i = b0 + threadIdx.x;
        bool have = i < nbig;
        PartKey b;
        b.w2 = inf;
        b.e2 = inf;
        b.ids = ~0ull;
        b.pos = 0;
        if (have) {
            b = part[toff[i]];
            dn += pdone[i];
        }
        bool to_c = have && b.w2 <= r.beta2;
        bool to_p = have && !to_c;
        if (to_p) minp = fmin(minp, b.w2);
        u32 off[kLists];
        u32 cnt[kLists] = {(u32)to_c, (u32)to_p, 0, 0, 0, 0};
        block_alloc(S, cnt, ctr, off);
        if (to_c) {
            if (off[0] < r.cap_c) put_edge_raw(r.c, off[0], b.w2, b.e2, b.ids, b.pos);
            else flag_overflow(r.cnt);
        }
        if (to_p) {
            if (off[1] < r.cap_p) put_edge_raw(r.pout, off[1], b.w2, b.e2, b.ids, b.pos);
            else flag_overflow(r.cnt);
        }
    }
    block_atomic_min(minp, &r.cnt->m[M_P], shm);
    dn = block_sum_u64(dn, shs);
    if (threadIdx.x == 0 && dn) atomicAdd(&r.cnt->c64[C64_BIGEVALS], dn);  // distances the tasks evaluated
}

// ------------------------------------------------------------ pool split
// Deferred BCCP edges: drop the ones whose ends are now connected, commit
// those within the new beta, keep the rest.
__global__ void __launch_bounds__(kBlock) k_split_pool(RoundArgs r, EdgeList pin, u32 npin) {
    __shared__ BlockAlloc S;
    __shared__ double shm[4];
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    u32* ctr[kLists] = {&r.cnt->c[C_C], &r.cnt->c[C_P], nullptr, nullptr, nullptr, nullptr};
    double minp = inf;
    for (u32 b0 = blockIdx.x * kSplitTile; b0 < npin; b0 += gridDim.x * kSplitTile) {
        u64 pos[kSplitItems];
        u32 tc = 0, tp = 0, nc = 0, np = 0;
#pragma unroll
        for (int k = 0; k < kSplitItems; ++k) {
            const u32 i = b0 + k * kBlock + threadIdx.x;
            pos[k] = 0;
            if (i < npin) {
                pos[k] = pin.pos[i];
                if (r.uf[(u32)(pos[k] >> 32)] != r.uf[(u32)pos[k]]) {
                    const double w2 = pin.w2[i];
                    const bool c = w2 <= r.beta2;
                    tc |= (u32)c << k;
                    tp |= (u32)!c << k;
                    nc += c;
                    np += !c;
                    if (!c) minp = fmin(minp, w2);
                }
            }
        }
        u32 off[kLists];
        u32 cnt[kLists] = {nc, np, 0, 0, 0, 0};
        block_alloc(S, cnt, ctr, off);
#pragma unroll
        for (int k = 0; k < kSplitItems; ++k) {
            if (!(((tc | tp) >> k) & 1u)) continue;
            const u32 i = b0 + k * kBlock + threadIdx.x;
            const double w2 = pin.w2[i], e2 = pin.e2[i];
            const u64 ids = pin.ids[i];
            if ((tc >> k) & 1u) {
                if (off[0] < r.cap_c) put_edge_raw(r.c, off[0], w2, e2, ids, pos[k]);
                else flag_overflow(r.cnt);
                ++off[0];
            } else {
                if (off[1] < r.cap_p) put_edge_raw(r.pout, off[1], w2, e2, ids, pos[k]);
                else flag_overflow(r.cnt);
                ++off[1];
            }
        }
    }
    block_atomic_min(minp, &r.cnt->m[M_P], shm);
}

// ------------------------------------------------------------ Kruskal

// One key word of the edge order, gathered through the current permutation
// (identity when perm is null; perm may alias val): 0 = ids packed as
// (lo << B) | hi, 1 = d2 bits, 2 = w2 bits (non-negative doubles order like
// their bits).  Also records the word's min and max.
__global__ void __launch_bounds__(kBlock) k_gather_word(const EdgeList L, const u32* perm, u32 m, int kind, int B,
                                                        const u32* pinst, u64* key, u32* val, u64* minmax) {
    __shared__ u64 smin[4], smax[4];
    u64 mn = ~0ull, mx = 0;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        u32 e = perm ? perm[i] : i;
        u64 w;
        if (kind == 0) {
            u64 ids = L.ids[e];
            w = ((ids >> 32) << B) | (ids & 0xffffffffull);
        } else if (kind == 1) {
            w = dbits(L.e2[e]);
        } else if (kind == 2) {
            w = dbits(L.w2[e]);
        } else {
            w = pinst[(u32)(L.pos[e] >> 32)];  // instance of the edge (batched solves)
        }
        key[i] = w;
        val[i] = e;
        mn = w < mn ? w : mn;
        mx = w > mx ? w : mx;
    }
    mn = wave_min_u64(mn);
    mx = ~wave_min_u64(~mx);
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) {
        smin[wv] = mn;
        smax[wv] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) {
            mn = smin[i] < mn ? smin[i] : mn;
            mx = smax[i] > mx ? smax[i] : mx;
        }
        mn = smin[0] < mn ? smin[0] : mn;
        mx = smax[0] > mx ? smax[0] : mx;
        atomicMin((unsigned long long*)&minmax[0], (unsigned long long)mn);
        atomicMax((unsigned long long*)&minmax[1], (unsigned long long)mx);
    }
}

// Clears the per-word state of the edge sort: the key word's running min and
// max and two flag words (flags[1] is the long-run flag).
__global__ void k_sort_init(u64* minmax, u32* flags) {
    if (threadIdx.x == 0) {
        minmax[0] = ~0ull;
        minmax[1] = 0;
        flags[0] = 0;
        flags[1] = 0;
    }
}

// Whether two keys are equal in their bits from sh up (the bits a sort on a
// key's leading bits ordered).
__device__ __forceinline__ bool same_lead(u64 a, u64 b, int sh) { return ((a ^ b) >> sh) == 0; }

// The first w2 bit of a sort on the leading `lead` bits that vary between the
// recorded min and max (0 when fewer vary), for the sort's device-side shift.
__global__ void k_sort_lead(const u64* minmax, int lead, int* sh) {
    if (threadIdx.x == 0) {
        const u64 diff = minmax[0] ^ minmax[1];
        const int bits = diff ? 64 - __clzll((long long)diff) : 0;
        *sh = bits > lead ? bits - lead : 0;
    }
}

// After a sort by the bits of w2 from *dsh up (keys `key`, the whole w2 bits;
// permutation `val`): order every run of keys equal in those bits by (w2,
// d2, ids), which completes the order K (with no such run, `out` is `val`).  First the (d2, ids) of every
// element that belongs to a run are gathered into sorted order (te, ti), all
// elements in parallel; then every element of a run counts the run's members
// that precede it in (w2, d2, ids) and writes its edge to that rank in `out`
// (elements outside runs are copied).  The members of a run sit side by
// side, so the lanes of a run read the same words together.  A run longer
// than kRunMax is flagged (the caller then sorts by every word).
constexpr u32 kRunMax = 256;

__global__ void __launch_bounds__(kBlock) k_run_keys(const EdgeList L, const u64* key, const u32* val, u32 m,
                                                     u64* te, u64* ti, const int* dsh) {
    const int sh = *dsh;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const u64 k = key[i];
        if ((i > 0 && same_lead(key[i - 1], k, sh)) || (i + 1 < m && same_lead(key[i + 1], k, sh))) {
            const u32 v = val[i];
            te[i] = dbits(L.e2[v]);
            ti[i] = L.ids[v];
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_fix_runs(const u64* key, const u32* val, const u64* te, const u64* ti,
                                                     u32 m, u32* out, u32* longrun, const int* dsh) {
    const int sh = *dsh;
    bool too_long = false;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const u64 k = key[i];
        const bool left = i > 0 && same_lead(key[i - 1], k, sh), right = i + 1 < m && same_lead(key[i + 1], k, sh);
        if (!left && !right) {
            out[i] = val[i];
            continue;
        }
        u32 s = i, e = i + 1;
        while (s > 0 && i - s < kRunMax && same_lead(key[s - 1], k, sh)) --s;
        while (e < m && e - i < kRunMax && same_lead(key[e], k, sh)) ++e;
        if (e - s > kRunMax || (s > 0 && same_lead(key[s - 1], k, sh)) || (e < m && same_lead(key[e], k, sh))) {
            too_long = true;
            continue;
        }
        const u64 ve = te[i], vi = ti[i];
        u32 r = 0;
        for (u32 j = s; j < e; ++j) {
            const u64 uk = key[j], ue = te[j], uj = ti[j];
            r += (uk < k || (uk == k && (ue < ve || (ue == ve && (uj < vi || (uj == vi && j < i)))))) ? 1u : 0u;
        }
        out[s + r] = val[i];
    }
    if (__any(too_long) && lane_id() == 0) atomicOr(longrun, 1u);
}

// The whole order K for a short list in one workgroup: a bitonic sort of
// (w2 bits, d2 bits, ids, index) in LDS, padded to a power of two with keys
// above every edge's.  Writes the permutation (sorted rank -> edge).
constexpr int kSmallSort = 2048;
constexpr int kSmallSortBlock = 1024;

__global__ void __launch_bounds__(kSmallSortBlock) k_sort_small(const EdgeList L, u32 m, u32* perm) {
    __shared__ u64 kw[kSmallSort], ke[kSmallSort], ki[kSmallSort];
    __shared__ u32 kv[kSmallSort];
    u32 N = 2;
    while (N < m) N <<= 1;
    for (u32 i = threadIdx.x; i < N; i += blockDim.x) {
        const bool real = i < m;
        kw[i] = real ? dbits(L.w2[i]) : ~0ull;
        ke[i] = real ? dbits(L.e2[i]) : ~0ull;
        ki[i] = real ? L.ids[i] : ~0ull;
        kv[i] = i;
    }
    __syncthreads();
    for (u32 k = 2; k <= N; k <<= 1) {
        for (u32 j = k >> 1; j > 0; j >>= 1) {
            for (u32 t = threadIdx.x; t < N / 2; t += blockDim.x) {
                const u32 a = ((t & ~(j - 1)) << 1) | (t & (j - 1));  // bit j of a is clear
                const u32 b = a + j;
                const bool up = (a & k) == 0;
                const u64 wa = kw[a], wb = kw[b], ea = ke[a], eb = ke[b], ia = ki[a], ib = ki[b];
                const bool b_less =
                    wb < wa || (wb == wa && (eb < ea || (eb == ea && (ib < ia || (ib == ia && kv[b] < kv[a])))));
                if (b_less == up) {
                    kw[a] = wb;
                    kw[b] = wa;
                    ke[a] = eb;
                    ke[b] = ea;
                    ki[a] = ib;
                    ki[b] = ia;
                    const u32 v = kv[a];
                    kv[a] = kv[b];
                    kv[b] = v;
                }
            }
            __syncthreads();
        }
    }
    for (u32 i = threadIdx.x; i < m; i += blockDim.x) perm[i] = kv[i];
}

// Instance of every arena row (instances packed in order; binary search in
// their first rows).
__global__ void k_row_instance(const int2* irange, u32 count, u32 n, u32* row_inst) {
    u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u32 lo = 0, hi = count - 1;
    while (lo < hi) {
        u32 mid = (lo + hi + 1) >> 1;
        if ((u32)irange[mid].x <= i) lo = mid;
        else hi = mid - 1;
    }
    row_inst[i] = lo;
}

__global__ void k_iota(u32* a, u32 m) {
    u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) a[i] = i;
}

constexpr int kFindCap = 1 << 22;  // bound on union-find walks (never reached by a forest)

__device__ __forceinline__ u32 uf_find(u32* parent, u32 x, Counters* cnt) {
    // path halving; every write points a vertex at one of its ancestors
    for (int it = 0; it < kFindCap; ++it) {
        u32 p = parent[x];
        if (p == x) return x;
        u32 g = parent[p];
        if (g != p) parent[x] = g;
        x = g;
    }
    atomicOr(&cnt->c[C_ERR], 8u);
    return x;
}

// Boruvka step on the committed edges in key-rank order: every component
// picks its lightest incident edge (atomic minimum of the rank); all picked
// edges are tree edges by the cut property; components hook along them.
// best[c] holds (stamp << 32 | rank) of component c's lightest edge in the
// step with that stamp; stamps decrease step by step, so a new step's keys
// win over stale ones without clearing the array between steps.
// The alive list holds each undecided edge's rank and, alongside, a vertex
// of each end's component (apos): the end positions at first, the roots
// found by the last step once the edge has been kept, so a step reads no
// permutation and its finds start close to the roots.
__global__ void k_alive_init(const u32* perm, const EdgeList L, u32 m, u32* alive, u64* apos) {
    for (u32 s = blockIdx.x * blockDim.x + threadIdx.x; s < m; s += gridDim.x * blockDim.x) {
        alive[s] = s;
        apos[s] = L.pos[perm[s]];
    }
}

__global__ void k_bor_pick(const u32* alive, const u64* apos, const u32* nalive_p, u32 cap, u32* parent, u64* best,
                           u32 stamp, u32* ru, u32* rv, u32* nalive_next, Counters* cnt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *nalive_next = 0;  // the hook step appends after this kernel
    const u32 na = min(*nalive_p, cap);
    const int lane = lane_id();
    // the loop bound is uniform over the block, so every lane reaches the
    // shuffle below
    for (u32 s0 = blockIdx.x * blockDim.x; s0 < na; s0 += gridDim.x * blockDim.x) {
        const u32 s = s0 + threadIdx.x;
        u32 a = kNone, b = kNone;
        u64 key = ~0ull;
        if (s < na) {
            const u32 rank = alive[s];
            const u64 pos = apos[s];
            a = uf_find(parent, (u32)(pos >> 32), cnt);
            b = uf_find(parent, (u32)pos, cnt);
            if (a == b) {
                ru[s] = kNone;
                a = b = kNone;
            } else {
                ru[s] = a;
                rv[s] = b;
                key = ((u64)stamp << 32) | rank;
            }
        }
        // The alive list runs in rank order (within each hook block's
        // output), and runs of consecutive edges often share a component
        // (ties of core distances; a few large components late in the
        // tree).  An end whose component the previous lane's lighter edge
        // also touches needs no update: that edge, or a still lighter one
        // before it, reaches the component's minimum.  The lightest edge of
        // a component is never skipped, so the minima are unchanged.
        const u32 pa = __shfl_up(a, 1), pb = __shfl_up(b, 1);
        const u64 pk = __shfl_up(key, 1);
        if (a == kNone) continue;
        const bool prev = lane > 0 && pk < key;
        // read first: most candidates already lose to a smaller rank
        if (!(prev && (pa == a || pb == a)) && key < best[a])
            atomicMin((unsigned long long*)&best[a], (unsigned long long)key);
        if (!(prev && (pa == b || pb == b)) && key < best[b])
            atomicMin((unsigned long long*)&best[b], (unsigned long long)key);
    }
}

// Hook step: each component's lightest edge (its rank is in best) joins it
// to the other end's component.  Four consecutive edges per thread and
// 1024-thread blocks: one append per list per 4096 edges, and the kept edges
// of a block stay in their input order.
constexpr int kHookBlock = 1024;
constexpr int kHookItems = 4;
constexpr int kHookTile = kHookBlock * kHookItems;

__global__ void __launch_bounds__(kHookBlock) k_bor_hook(const u32* alive, const u32* nalive_p,
                                                         u32 cap, const u32* perm, const EdgeList L, u32* parent,
                                                         const u64* best, u32 stamp, const u32* ru, const u32* rv,
                                                         u32* alive_next, u64* apos_next, u32* nalive_next,
                                                         EdgeList out, u32 cap_out, Counters* cnt) {
    __shared__ BlockAlloc S;
    const u32 na = min(*nalive_p, cap);
    u32* ctr[kLists] = {&cnt->c[C_OUT], nalive_next, nullptr, nullptr, nullptr, nullptr};
    for (u32 b0 = blockIdx.x * kHookTile; b0 < na; b0 += gridDim.x * kHookTile) {
        u32 sel = 0, keep = 0, ns = 0, nk = 0;
        u32 rank[kHookItems];
        u64 roots[kHookItems];
#pragma unroll
        for (int k = 0; k < kHookItems; ++k) {
            const u32 s = b0 + threadIdx.x * kHookItems + k;
            rank[k] = 0;
            roots[k] = 0;
            const u32 a = s < na ? ru[s] : kNone;
            if (a == kNone) continue;
            const u32 b = rv[s];
            roots[k] = ((u64)a << 32) | b;
            rank[k] = alive[s];
            const u64 key = ((u64)stamp << 32) | rank[k];
            const bool pa = best[a] == key, pb = best[b] == key;
            if (pa || pb) {
                if (pa && pb) {
                    u32 hi = a > b ? a : b, lo = a > b ? b : a;
                    parent[hi] = lo;
                } else if (pa) {
                    parent[a] = b;
                } else {
                    parent[b] = a;
                }
                sel |= 1u << k;
                ++ns;
            } else {
                keep |= 1u << k;
                ++nk;
            }
        }
        u32 off[kLists];
        u32 cn[kLists] = {ns, nk, 0, 0, 0, 0};
        block_alloc(S, cn, ctr, off);
#pragma unroll
        for (int k = 0; k < kHookItems; ++k) {
            if ((sel >> k) & 1u) {
                const u32 e = perm[rank[k]];
                if (off[0] < cap_out) put_edge_raw(out, off[0], L.w2[e], L.e2[e], L.ids[e], L.pos[e]);
                else flag_overflow(cnt);
                ++off[0];
            }
            if ((keep >> k) & 1u) {
                if (off[1] < cap) {
                    // the ends' roots of this step: a later step's finds
                    // start there instead of at the end points
                    alive_next[off[1]] = rank[k];
                    apos_next[off[1]] = roots[k];
                }
                ++off[1];
            }
        }
    }
}

__global__ void k_set_u32(u32* p, u32 v) { *p = v; }

// Full path compression: afterwards parent[v] is v's component root.
__global__ void k_uf_compress(u32* parent, int n, Counters* cnt) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    u32 r = (u32)v;
    int it = 0;
    while (parent[r] != r && it < kFindCap) {
        r = parent[r];
        ++it;
    }
    if (it == kFindCap) atomicOr(&cnt->c[C_ERR], 8u);
    parent[v] = r;
}

// Component of each node: the root shared by all its points, else -1.
__global__ void k_boundaries(const u32* uf, int n, u32* bnd) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    bnd[p] = (p > 0 && uf[p] != uf[p - 1]) ? 1u : 0u;
}

// (ranges: every node's (first, count), a compact copy of the records'
// ranges, so that this pass reads 8 bytes per node instead of a record.)
// The labels are compared against a compact copy (4 bytes per node) and the
// record is written only when its label changed: most labels survive a
// round, and reading each record's line would cost 64 bytes per node.
template <int D>
__global__ void k_node_comp(NodeRec<D>* nodes, int* labels, const int2* ranges, const u32* uf, const u32* incl,
                            int nn) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
    int2 r = ranges[v];
    int last = r.x + r.y - 1;
    const int c = (incl[last] == incl[r.x]) ? (int)uf[r.x] : -1;
    if (labels[v] != c) {
        labels[v] = c;
        nodes[v].comp = c;
    }
}

template <int D>
__global__ void k_node_ranges(const NodeRec<D>* nodes, int nn, int2* ranges) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < nn) ranges[v] = make_int2(nodes[v].first, nodes[v].count);
}

// ------------------------------------------------------------ output
// Correctly rounded square root.  The library result y is checked against
// the exact condition lo^2 < x < hi^2, where lo and hi are the midpoints
// between y and its neighbouring binary64 values (a binary64 square root is
// never exactly halfway), using 128-bit integer arithmetic on the
// significands, and moved by one unit in the last place until it holds.
//
// Sign of (M * 2^e)^2 - x for an integer M < 2^56 and a normal x > 0.
__device__ __forceinline__ int cmp_sq(u64 M, int e, double x) {
    int ex;
    double fx = frexp(x, &ex);
    u64 X = (u64)ldexp(fx, 53);  // x = X * 2^(ex-53)
    unsigned __int128 S = (unsigned __int128)M * (unsigned __int128)M;  // value S * 2^(2e)
    int sh = (ex - 53) - 2 * e;  // compare S with X * 2^sh
    if (sh >= 0) {
        if (sh > 70) return -1;  // X * 2^sh >= 2^123 > S
        unsigned __int128 R = (unsigned __int128)X << sh;
        return S > R ? 1 : (S < R ? -1 : 0);
    }
    int s2 = -sh;
    if (s2 >= 120) return -1;  // S * 2^-s2 < 1 <= X
    unsigned __int128 S2 = S >> s2;
    unsigned __int128 lost = S - (S2 << s2);
    unsigned __int128 R = (unsigned __int128)X;
    if (S2 > R) return 1;
    if (S2 < R) return -1;
    return lost ? 1 : 0;
}

__device__ double sqrt_rn(double x) {
    if (!(x > 0.0)) return x == 0.0 ? 0.0 : x;
    // subnormal inputs: scale by 2^108 (exact), root scales by 2^54
    double scale = 1.0;
    if (x < 2.2250738585072014e-308) {
        x = ldexp(x, 108);
        scale = ldexp(1.0, -54);
    }
    double y = sqrt(x);
    for (int it = 0; it < 4; ++it) {
        int ey;
        double fy = frexp(y, &ey);
        u64 Y = (u64)ldexp(fy, 53);  // y = Y * 2^(ey-53), Y in [2^52, 2^53)
        // upper midpoint (2Y+1) * 2^(ey-54)
        if (cmp_sq(2 * Y + 1, ey - 54, x) < 0) {
            y = nextafter(y, __longlong_as_double(0x7ff0000000000000ll));
            continue;
        }
        // lower midpoint: (4Y-1) * 2^(ey-55) when y is a power of two, else (2Y-1) * 2^(ey-54)
        bool pow2 = Y == (1ull << 52);
        int c = pow2 ? cmp_sq(4 * Y - 1, ey - 55, x) : cmp_sq(2 * Y - 1, ey - 54, x);
        if (c > 0) {
            y = nextafter(y, 0.0);
            continue;
        }
        break;
    }
    return y * scale;
}

// Output edge k of the sorted order; batched solves subtract the instance's
// first row so that ids are local to the instance.
__global__ void k_write_edges(const EdgeList L, const u32* perm, u32 m, const u32* pinst, const int2* irange,
                              long long* edges, double* w, double* w2) {
    u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    u32 e = perm[k];
    u64 ids = L.ids[e];
    long long base = pinst ? (long long)irange[pinst[(u32)(L.pos[e] >> 32)]].x : 0ll;
    edges[2 * (size_t)k] = (long long)(ids >> 32) - base;
    edges[2 * (size_t)k + 1] = (long long)(ids & 0xffffffffull) - base;
    double x = L.w2[e];
    if (w) w[k] = sqrt_rn(x);
    if (w2) w2[k] = x;
}

__global__ void k_write_cd(const double* cd2s, const u32* orig, int n, double* cd, double* cd2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    u32 o = orig[p];
    double x = cd2s[p];
    if (cd) cd[o] = sqrt_rn(x);
    if (cd2) cd2[o] = x;
}

// Input check: non-finite coordinates or |x| > 2^500 (keeps every squared
// distance finite).
__global__ void k_check_input(const double* P, size_t m, Counters* cnt) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    for (; i < m; i += (size_t)gridDim.x * blockDim.x) {
        double x = P[i];
        bad |= !(fabs(x) <= 0x1p500);  // false for NaN
    }
    if (__any(bad) && lane_id() == 0) atomicOr(&cnt->c[C_ERR], 2u);
}

}  // namespace geomst
