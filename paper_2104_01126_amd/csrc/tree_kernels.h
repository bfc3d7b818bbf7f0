// Tree construction (the spatial tree the decomposition runs on; paper
// Sec. 2.3 "k-d tree" and Sec. 3.1.1) and core distances (Sec. 2.1 /
// Sec. 3.2.1: k-NN with k = minPts, the point itself included).
//
// The k-d tree is a Morton-order binary radix tree: points are sorted by the
// bit-interleaved code of their quantised coordinates, and every internal
// node splits its contiguous range at the highest differing code bit, i.e. at
// the spatial median of its cell along one dimension.  Leaves hold one point
// (leaf size c = 1, as in Sec. 3.1.1).  Node boxes are tight boxes of the
// node's actual points, so the quantisation only shapes the tree and never
// enters any distance.
#pragma once
#include <type_traits>
#include "common.h"

namespace geomst {

// Per-node record: box of the node's points, its contiguous range of sorted
// positions, the split position of the radix tree (children follow from it),
// and the component shared by all its points (or -1), which the decomposition
// reads together with the box (rewritten after Kruskal steps).  The sphere
// radius about the box centre is half the box diagonal and is derived from
// the box where needed.  Core-distance ranges (HDBSCAN*) live in their own
// array so that EMST never reads them.
//
// For d <= 3 the box is the tight binary64 box (the record is one 32- or
// 64-byte line).  For d >= 4 it is stored in binary32, each bound rounded
// outward from the tight box, so that it still contains every point exactly
// and the record fits one 64-byte line (80 bytes for d = 7) instead of two;
// every bound computed from it is then still a bound of the computed
// point-to-point values, only looser by the rounding.
//
// Where the padded record has 8 spare bytes (d = 4, 5, 7) it also carries
// the node's core-distance range (HDBSCAN*) in binary32, the minimum rounded
// down and the maximum up, so that the decomposition reads a node's box and
// core distances from one line; the exact binary64 ranges stay in their own
// array for every other use.
template <int D>
struct NodeBox {
    using type = typename std::conditional<(D >= 4), float, double>::type;
    static constexpr bool cd_in = D == 4 || D == 5 || D == 7;
    static constexpr int bytes = 2 * D * (int)sizeof(type) + 16 + (cd_in ? 8 : 0);
    static constexpr int align = bytes <= 32 ? 32 : bytes <= 64 ? 64 : 16;
};

template <bool C>
struct NodeCd {};
template <>
struct NodeCd<true> {
    float cdlo, cdhi;  // (min cd2, max cd2) of the node's points, rounded outward
};

template <int D>
struct alignas(NodeBox<D>::align) NodeRec : NodeCd<NodeBox<D>::cd_in> {
    typename NodeBox<D>::type lo[D];
    typename NodeBox<D>::type hi[D];
    int first, count;
    int split;  // radix-tree split position g of an internal node; -1 for a leaf
    int comp;   // component of all the node's points, or -1
};
static_assert(sizeof(NodeRec<3>) == 64 && sizeof(NodeRec<4>) == 64 && sizeof(NodeRec<5>) == 64 &&
                  sizeof(NodeRec<6>) == 64 && sizeof(NodeRec<7>) == 80,
              "one 64-byte line per record up to d = 6");

// Binary32 bounds rounded outward (towards -inf for a lower bound, +inf for
// an upper bound); the comparisons with the binary64 value are exact.
__device__ __forceinline__ float round_down_f32(double x) {
    float f = (float)x;
    return ((double)f > x) ? nextafterf(f, -__builtin_huge_valf()) : f;
}
__device__ __forceinline__ float round_up_f32(double x) {
    float f = (float)x;
    return ((double)f < x) ? nextafterf(f, __builtin_huge_valf()) : f;
}
__device__ __forceinline__ void store_lo(double& dst, double x) { dst = x; }
__device__ __forceinline__ void store_hi(double& dst, double x) { dst = x; }
__device__ __forceinline__ void store_lo(float& dst, double x) { dst = round_down_f32(x); }
__device__ __forceinline__ void store_hi(float& dst, double x) { dst = round_up_f32(x); }

struct TreeView {
    int n;              // points
    const double* X;    // sorted points, row-major [n][D]
    const u32* orig;    // sorted position -> caller row index
    const double* cd2;  // sorted position -> squared core distance, or null (EMST)
    const void* nodes;  // NodeRec<D>[2n-1]
    const double2* cdr; // [2n-1] (min cd2, max cd2) of the node's points (HDBSCAN*)
    const double* XC;   // HDBSCAN*: each sorted point followed by its cd2, row-major [n][D+1]
};
// Node ids: internal nodes 0..n-2 (0 is the root), the leaf of sorted
// position p is node n-1+p.

template <int D>
__device__ __forceinline__ const NodeRec<D>* nodes_of(const TreeView& t) {
    return (const NodeRec<D>*)t.nodes;
}

// Core-distance range (min cd2, max cd2) of node `id` whose record is X:
// from the record where it carries one (a range that contains the exact
// one), else from the exact array.
template <int D>
__device__ __forceinline__ double2 node_cd(const TreeView& t, const NodeRec<D>& X, u32 id) {
    if constexpr (NodeBox<D>::cd_in) return make_double2((double)X.cdlo, (double)X.cdhi);
    else return t.cdr[id];
}

// Stores a node's exact range and, where the record has room, its outward
// binary32 copy.
template <int D>
__device__ __forceinline__ void put_cd(NodeRec<D>& V, double2* cdr, int v, double2 cd) {
    cdr[v] = cd;
    if constexpr (NodeBox<D>::cd_in) {
        V.cdlo = round_down_f32(cd.x);
        V.cdhi = round_up_f32(cd.y);
    }
}

// Children of an internal node from its range [f, f+c) and split g: the left
// child covers [f, g], the right [g+1, f+c-1]; a one-point side is a leaf.
__device__ __forceinline__ int2 node_kids(int n, int f, int c, int g) {
    int left = (f == g) ? (n - 1 + g) : g;
    int right = (f + c - 1 == g + 1) ? (n - 1 + g + 1) : (g + 1);
    return make_int2(left, right);
}

// ------------------------------------------------------------ bounding box
template <int D>
__global__ void __launch_bounds__(256) k_bbox_partial(const double* P, int n, double* partial) {
    __shared__ double red[2 * D][256 / kWave];
    double lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = __longlong_as_double(0x7ff0000000000000ll);
        hi[k] = -lo[k];
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double x = P[(size_t)i * D + k];
            lo[k] = fmin(lo[k], x);
            hi[k] = fmax(hi[k], x);
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = wave_min_f64(lo[k]);
        hi[k] = -wave_min_f64(-hi[k]);
    }
    int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            red[k][w] = lo[k];
            red[D + k][w] = hi[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        int k = threadIdx.x;
        double v = red[k][0];
        for (int i = 1; i < 256 / kWave; ++i) v = (k < D) ? fmin(v, red[k][i]) : fmax(v, red[k][i]);
        partial[(size_t)blockIdx.x * 2 * D + k] = v;
    }
}

// Combines the per-block boxes: every lane folds a strided share of them
// (independent loads, not one dependent chain per coordinate), then the
// waves and the block reduce.
constexpr int kBboxFinal = 256;

template <int D>
__global__ void __launch_bounds__(kBboxFinal) k_bbox_final(const double* partial, int nb, double* bbox) {
    __shared__ double red[2 * D][kBboxFinal / kWave];
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    double lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = inf;
        hi[k] = -inf;
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            lo[k] = fmin(lo[k], partial[(size_t)b * 2 * D + k]);
            hi[k] = fmax(hi[k], partial[(size_t)b * 2 * D + D + k]);
        }
    }
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = wave_min_f64(lo[k]);
        hi[k] = -wave_min_f64(-hi[k]);
        if (lane_id() == 0) {
            red[k][w] = lo[k];
            red[D + k][w] = hi[k];
        }
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < 2 * D) {
        double v = red[k][0];
        for (int i = 1; i < kBboxFinal / kWave; ++i) v = (k < D) ? fmin(v, red[k][i]) : fmax(v, red[k][i]);
        bbox[k] = v;
    }
}

// ------------------------------------------------------------ Morton code
// Keys are built in levels.  Level 0 quantises every point in the global
// bounding box; each later level takes the groups of points whose keys are
// still equal and quantises them again inside the group's own bounding box,
// so the tree keeps splitting space (at the midpoint of the quantisation
// cell) however tightly points cluster.  The keys only shape the tree.
template <int D>
__device__ __forceinline__ int morton_bits() {
    return (63 / D) > 31 ? 31 : (63 / D);
}

template <int D>
__device__ __forceinline__ u64 morton_code(const double* x, const double* lo, const double* hi) {
    const int b = morton_bits<D>();
    const double top = (double)((1ull << b) - 1);
    u64 q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double r = hi[k] - lo[k];
        double t = r > 0.0 ? (x[k] - lo[k]) / r : 0.0;
        double f = floor(t * top);
        f = f < 0.0 ? 0.0 : (f > top ? top : f);
        q[k] = (u64)f;
    }
    u64 c = 0;
    for (int bit = b - 1; bit >= 0; --bit) {
#pragma unroll
        for (int k = 0; k < D; ++k) c = (c << 1) | ((q[k] >> bit) & 1ull);
    }
    return c;
}

template <int D>
__global__ void k_morton(const double* P, int n, const double* bbox, u64* key, u32* val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = morton_code<D>(P + (size_t)i * D, bbox, bbox + D);
    val[i] = (u32)i;
}

// Batched solves: the first key word is the point's instance, so every
// instance becomes one contiguous subtree and the refinement levels quantise
// each instance inside its own box.
__global__ void k_inst_key(const u32* row_inst, int n, u64* key, u32* val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = row_inst[i];
    val[i] = (u32)i;
}

// Group starts: flag[i] = 1 where the key words [0, L) of sorted positions i
// and i-1 differ (and at i = 0).  any_dup gets 1 if some group has >1 point.
__global__ void k_key_flags(const u64* keys, int n, int L, u32* flag, u32* any_dup) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool dup = false;
    if (i < n) {
        u32 f = 1;
        if (i > 0) {
            f = 0;
            for (int l = 0; l < L; ++l)
                if (keys[(size_t)l * n + i] != keys[(size_t)l * n + i - 1]) f = 1;
        }
        flag[i] = f;
        dup = (f == 0);
    }
    // a flag many waves raise: test before setting, so that once it is
    // visible the waves skip the contended atomic
    if (__any(dup) && lane_id() == 0 && *(volatile u32*)any_dup == 0u) atomicOr(any_dup, 1u);
}

// gid[i] = group of sorted position i (inclusive scan of flags minus one);
// start[g] = first position of group g.
__global__ void k_group_ids(const u32* incl, int n, u32* gid, u32* start) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u32 g = incl[i] - 1;
    gid[i] = g;
    if (i == 0 || incl[i] != incl[i - 1]) start[g] = (u32)i;
}

// One wave per group with more than one point: its bounding box, and
// whether it can still be split (non-zero extent).
template <int D>
__global__ void k_group_box(const double* P, const u32* val, int n, const u32* start, u32 ngroups, double* gbox,
                            u32* refinable) {
    u32 g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (g >= ngroups) return;
    u32 s = start[g];
    u32 e = (g + 1 < ngroups) ? start[g + 1] : (u32)n;
    if (e - s < 2) return;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    double lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = inf;
        hi[k] = -inf;
    }
    for (u32 i = s + lane_id(); i < e; i += kWave) {
        const double* x = P + (size_t)val[i] * D;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            lo[k] = fmin(lo[k], x[k]);
            hi[k] = fmax(hi[k], x[k]);
        }
    }
    bool ext = false;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = wave_min_f64(lo[k]);
        hi[k] = -wave_min_f64(-hi[k]);
        ext |= hi[k] > lo[k];
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            gbox[(size_t)g * 2 * D + k] = lo[k];
            gbox[(size_t)g * 2 * D + D + k] = hi[k];
        }
        if (ext && *(volatile u32*)refinable == 0u) atomicOr(refinable, 1u);  // test before setting
    }
}

// Next key word of every sorted position: its point quantised inside its
// group's box (0 for single-point groups).
template <int D>
__global__ void k_morton_level(const double* P, const u32* val, int n, const u32* gid, const u32* start,
                               u32 ngroups, const double* gbox, u64* key) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u32 g = gid[i];
    u32 s = start[g];
    u32 e = (g + 1 < ngroups) ? start[g + 1] : (u32)n;
    u64 c = 0;
    if (e - s > 1) c = morton_code<D>(P + (size_t)val[i] * D, gbox + (size_t)g * 2 * D, gbox + (size_t)g * 2 * D + D);
    key[i] = c;
}

// b[i] = a[perm[i]] widened to 64 bits (the sort key of a gathered word).
__global__ void k_gather_u32_u64(const u32* a, const u32* perm, int n, u64* b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[perm[i]];
}

// Apply a permutation of sorted positions to the point ids and key words.
__global__ void k_apply_perm(const u32* perm, int n, int L, const u32* val_in, u32* val_out, const u64* key_in,
                             u64* key_out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u32 p = perm[i];
    val_out[i] = val_in[p];
    for (int l = 0; l < L; ++l) key_out[(size_t)l * n + i] = key_in[(size_t)l * n + p];
}

template <int D>
__global__ void k_permute(const double* P, int n, const u32* val, double* X, u32* orig) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u32 src = val[i];
#pragma unroll
    for (int k = 0; k < D; ++k) X[(size_t)i * D + k] = P[(size_t)src * D + k];
    orig[i] = src;
}

// ------------------------------------------------------ binary radix tree
// Common-prefix length of the multi-word keys at sorted positions i and j
// (equal keys are told apart by their positions), -1 outside [0, n).
__device__ __forceinline__ int prefix_len(const u64* k, int n, int L, int i, int j) {
    if (j < 0 || j >= n) return -1;
    for (int l = 0; l < L; ++l) {
        u64 a = k[(size_t)l * n + i], b = k[(size_t)l * n + j];
        if (a != b) return 64 * l + __clzll((long long)(a ^ b));
    }
    return 64 * L + __clz((int)(i ^ j));
}

template <int D>
__global__ void k_karras(const u64* k, int n, int L, NodeRec<D>* nodes, int* parent) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int dir = (prefix_len(k, n, L, i, i + 1) - prefix_len(k, n, L, i, i - 1)) > 0 ? 1 : -1;
    int dmin = prefix_len(k, n, L, i, i - dir);
    int lmax = 2;
    while (prefix_len(k, n, L, i, i + lmax * dir) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(k, n, L, i, i + (l + t) * dir) > dmin) l += t;
    int j = i + l * dir;
    int dnode = prefix_len(k, n, L, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(k, n, L, i, i + (s + t) * dir) > dnode) s += t;
    } while (t > 1);
    int g = i + s * dir + (dir < 0 ? -1 : 0);
    int first = min(i, j), last = max(i, j);
    int left = (first == g) ? (n - 1 + g) : g;
    int right = (last == g + 1) ? (n - 1 + g + 1) : (g + 1);
    nodes[i].first = first;
    nodes[i].count = last - first + 1;
    nodes[i].split = g;
    parent[left] = i;
    parent[right] = i;
    if (i == 0) parent[0] = -1;
}

// ------------------------------------------------------------ node bounds
// Bottom-up: every internal node is finished by the second of its two
// children to arrive.  Phase 1: a block owns 1024 consecutive leaves and
// merges every node whose range lies inside them through LDS (arrival
// counters and boxes; workgroup-scope ordering only).  A thread whose climb
// reaches a node spanning several blocks records the child it came from, in
// the list of its super-block (kBoundsSpan leaves).  Phase 2: one workgroup
// per super-block finishes the spanning nodes inside it, starting from those
// children, and records the children of nodes that span super-blocks; then
// one workgroup finishes those.  Every arrival counter and record a
// workgroup touches is its own, so workgroup-scope ordering suffices
// throughout.
constexpr int kBoundsBlock = 1024;
constexpr int kBoundsTop = 1024;            // threads of a phase-2 workgroup
constexpr int kBoundsSpan = 64 * 1024;      // leaves per phase-2 super-block
constexpr int kBoundsSpanCap = 2 * kBoundsSpan;  // list slots per super-block

template <int D>
__device__ __forceinline__ void write_box(NodeRec<D>& V, const double* lo, const double* hi) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
        store_lo(V.lo[k], lo[k]);
        store_hi(V.hi[k], hi[k]);
    }
}

template <int D>
__global__ void __launch_bounds__(kBoundsBlock) k_bounds_local(int n, const double* X, const double* cd2,
                                                               const int* parent, NodeRec<D>* nodes, double2* cdr,
                                                               int geometry, u32* top, u32* ntop) {
    // top / ntop: per super-block lists of kBoundsSpanCap slots and counters
    __shared__ u32 lflag[kBoundsBlock];
    __shared__ double slo[kBoundsBlock][D], shi[kBoundsBlock][D];
    __shared__ double2 scd[kBoundsBlock];
    __shared__ int sfirst[kBoundsBlock], scount[kBoundsBlock], ssplit[kBoundsBlock], sparent[kBoundsBlock];
    const int base = blockIdx.x * kBoundsBlock;
    const int end = min(base + kBoundsBlock, n);  // leaves [base, end)
    lflag[threadIdx.x] = 0;
    // Internal node v covers sorted position v, so only nodes base..end-1
    // can lie inside the block: their ranges, splits and parents are loaded
    // once, side by side, and the climbs below read them from LDS.
    {
        const int v = base + threadIdx.x;
        if (v < end && v < n - 1) {
            sfirst[threadIdx.x] = nodes[v].first;
            scount[threadIdx.x] = nodes[v].count;
            ssplit[threadIdx.x] = nodes[v].split;
            sparent[threadIdx.x] = parent[v];
        }
    }
    __syncthreads();
    int p = base + threadIdx.x;
    if (p >= n) return;
    int leaf = n - 1 + p;
    if (geometry) {
        NodeRec<D>& L = nodes[leaf];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            store_lo(L.lo[k], X[(size_t)p * D + k]);
            store_hi(L.hi[k], X[(size_t)p * D + k]);
        }
        L.first = p;
        L.count = 1;
        L.split = -1;
        L.comp = -1;
    }
    if (cd2) put_cd<D>(nodes[leaf], cdr, leaf, make_double2(cd2[p], cd2[p]));
    int child = leaf;
    int v = parent[leaf];
    while (v >= 0) {
        NodeRec<D>& V = nodes[v];
        const bool local = v >= base && v < end;  // else v's range holds a position outside the block
        const int f = local ? sfirst[v - base] : 0, c = local ? scount[v - base] : 0;
        if (!local || !(f >= base && f + c <= end)) {
            // spanning node: hand the climb over to phase 2
            const u32 sb = (u32)base / kBoundsSpan;
            __threadfence();
            u32 s = atomicAdd(&ntop[sb], 1u);
            top[(size_t)sb * kBoundsSpanCap + s] = (u32)child;
            return;
        }
        __threadfence_block();
        if (atomicAdd(&lflag[v - base], 1u) == 0) return;
        __threadfence_block();
        int2 ch = node_kids(n, f, c, ssplit[v - base]);
        double lo[D], hi[D];
        double2 cd = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double a0, a1, b0, b1;
            if (ch.x >= n - 1) a0 = a1 = X[(size_t)(ch.x - (n - 1)) * D + k];
            else {
                a0 = slo[ch.x - base][k];
                a1 = shi[ch.x - base][k];
            }
            if (ch.y >= n - 1) b0 = b1 = X[(size_t)(ch.y - (n - 1)) * D + k];
            else {
                b0 = slo[ch.y - base][k];
                b1 = shi[ch.y - base][k];
            }
            lo[k] = fmin(a0, b0);
            hi[k] = fmax(a1, b1);
            slo[v - base][k] = lo[k];
            shi[v - base][k] = hi[k];
        }
        if (cd2) {
            double2 ca = (ch.x >= n - 1) ? make_double2(cd2[ch.x - (n - 1)], cd2[ch.x - (n - 1)]) : scd[ch.x - base];
            double2 cb = (ch.y >= n - 1) ? make_double2(cd2[ch.y - (n - 1)], cd2[ch.y - (n - 1)]) : scd[ch.y - base];
            cd = make_double2(fmin(ca.x, cb.x), fmax(ca.y, cb.y));
            scd[v - base] = cd;
            put_cd<D>(V, cdr, v, cd);
        }
        if (geometry) write_box<D>(V, lo, hi);
        child = v;
        v = sparent[v - base];
    }
}

// Phase 2: climb from the recorded children through the spanning nodes;
// gflags holds one arrival counter per internal node.  With out != null,
// workgroup g takes list g (top + g * kBoundsSpanCap, count ntop[g]) and
// stops at nodes spanning super-blocks, recording the child in out;
// otherwise one workgroup takes the single list and climbs to the root.
template <int D>
__global__ void __launch_bounds__(kBoundsTop) k_bounds_top(int n, const int* parent, NodeRec<D>* nodes, double2* cdr,
                                                           int geometry, int hdb, const u32* top, const u32* ntop,
                                                           u32* gflags, u32* out, u32* nout) {
    const u32 m = ntop[blockIdx.x];
    const u32* list = top + (size_t)blockIdx.x * kBoundsSpanCap;
    for (u32 i = threadIdx.x; i < m; i += blockDim.x) {
        int c = (int)list[i];
        int v = parent[c];
        while (v >= 0) {
            if (out) {
                const int f = nodes[v].first, cnt = nodes[v].count;
                if (f / kBoundsSpan != (f + cnt - 1) / kBoundsSpan) {
                    u32 s = atomicAdd(nout, 1u);
                    out[s] = (u32)c;
                    break;
                }
            }
            __threadfence_block();
            if (atomicAdd(&gflags[v], 1u) == 0) break;
            __threadfence_block();
            NodeRec<D>& V = nodes[v];
            int2 ch = node_kids(n, V.first, V.count, V.split);
            const volatile NodeRec<D>* A = nodes + ch.x;
            const volatile NodeRec<D>* B = nodes + ch.y;
            if (geometry) {
                double lo[D], hi[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    lo[k] = fmin((double)A->lo[k], (double)B->lo[k]);
                    hi[k] = fmax((double)A->hi[k], (double)B->hi[k]);
                }
                write_box<D>(V, lo, hi);
            }
            if (hdb) {
                const volatile double2* ca = cdr + ch.x;
                const volatile double2* cb = cdr + ch.y;
                put_cd<D>(V, cdr, v, make_double2(fmin(ca->x, cb->x), fmax(ca->y, cb->y)));
            }
            c = v;
            v = parent[v];
        }
    }
}

// Rows of X with each point's squared core distance appended (one line per
// point for the point-pair kernels instead of two).
template <int D>
__global__ void k_append_cd(const double* X, const double* cd2, double* XC, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
#pragma unroll
    for (int k = 0; k < D; ++k) XC[(size_t)p * (D + 1) + k] = X[(size_t)p * D + k];
    XC[(size_t)p * (D + 1) + D] = cd2[p];
}

// ------------------------------------------------------------ core distances
// One wave per 64 consecutive sorted points.  The wave walks the tree once,
// descending into a node while any lane's box distance beats its current
// k-th smallest squared distance; nodes of at most kLeafScan points are
// scanned by all lanes (each lane against every point of the node).  The
// per-lane k smallest values are kept sorted in registers.
constexpr int kKnnLeaf = 32;
constexpr int kKnnSeed = 32;  // sorted neighbours on each side of a wave's queries scanned first
// The walk's stack holds at most (tree depth + 1) nodes: each pop pushes at
// most two children.  A root-to-leaf path of the radix tree splits on a
// distinct bit of (key words, position) at every node, so the depth is at
// most 6 * 63 key bits + 26 position bits = 404 and 512 entries never
// overflow (the check below stays as a guard).  An entry is 8 bytes: the two
// children of an internal node, or (~node, first position) of a node small
// enough to scan, so that a pop needs no load of the node's own record
// before the loads of what comes next.  LDS per wave: the seed window's
// (64 + 2 * 32) rows of 8d bytes, whose bytes the walk then reuses for its
// 4 KB stack and one scanned node's 32 rows.
constexpr int kKnnStack = 512;

template <int D>
struct KnnLds {
    static constexpr int seed = (kWave + 2 * kKnnSeed) * D;    // doubles
    static constexpr int walk = kKnnLeaf * D + kKnnStack;      // doubles (one int2 each)
    static constexpr int doubles = seed > walk ? seed : walk;
};

// The stack entry of node v (its record R already loaded).
template <int D>
__device__ __forceinline__ int2 knn_entry(int n, int v, const NodeRec<D>& R) {
    return R.count <= kKnnLeaf ? make_int2(~v, R.first) : node_kids(n, R.first, R.count, R.split);
}

template <int KMAX>
__device__ __forceinline__ void topk_insert(double (&top)[KMAX], double v) {
    // new[s] = min(old[s], max(old[s-1], v)); new[0] = min(old[0], v)
#pragma unroll
    for (int s = KMAX - 1; s > 0; --s) top[s] = fmin(top[s], fmax(top[s - 1], v));
    top[0] = fmin(top[0], v);
}

template <int D>
__device__ __forceinline__ double sqdist(const double (&a)[D], const double* b) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t = a[k] - b[k];
        s = s + t * t;
    }
    return s;
}

// Squared distance from a point to a box, computed so that it never exceeds
// the computed squared distance to any point of the box.
template <int D, class B>
__device__ __forceinline__ double point_box_lb2(const double (&q)[D], const B* lo, const B* hi) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double g = fmax(fmax((double)lo[k] - q[k], q[k] - (double)hi[k]), 0.0);
        s = s + g * g;
    }
    return s;
}

// Five waves per SIMD where the registers allow (d <= 5, k <= 16).
template <int D, int KMAX>
struct KnnWaves {
    static constexpr int value = (D <= 5 && KMAX <= 16) ? 5 : 1;
};

// Batched solves pass the instance of each sorted position and each
// instance's (first position, size) and k: a lane only accepts points of its
// own instance (the sorted positions of an instance are contiguous).
template <int D, int KMAX>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KnnWaves<D, KMAX>::value))) k_knn(TreeView t, int kk_all, const u32* pinst, const int2* irange,
                                           const int* ik, double* cd2_out, u32* err) {
    static_assert(kKnnLeaf <= kWave, "a leaf is staged one row per lane");
    __shared__ double lds[KnnLds<D>::doubles];
    double* rows = lds;  // the seed window's rows, then one scanned node's
    int2* stack = reinterpret_cast<int2*>(lds + kKnnLeaf * D);  // used after the seed scan
    const int n = t.n;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    int p = blockIdx.x * kWave + lane_id();
    bool live = p < n;
    int pq = live ? p : n - 1;
    int lo_r = 0, hi_r = n, kk = kk_all;
    if (pinst) {
        u32 ins = pinst[pq];
        int2 rg = irange[ins];
        lo_r = rg.x;
        hi_r = rg.x + rg.y;
        kk = ik[ins];
    }
    // the positions inside every lane's instance (all of [0, n) outside a
    // batch), in scalar registers
    int lo_all = lo_r, hi_all = hi_r;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo_all = max(lo_all, __shfl_xor(lo_all, o));
        hi_all = min(hi_all, __shfl_xor(hi_all, o));
    }
    lo_all = __builtin_amdgcn_readfirstlane(lo_all);
    hi_all = __builtin_amdgcn_readfirstlane(hi_all);
    double q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) q[k] = t.X[(size_t)pq * D + k];
    // slots [0, KMAX-kk) hold -inf so that the kk-th smallest value seen is
    // always in the last slot
    double top[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s) top[s] = (s < KMAX - kk) ? -inf : inf;
    double kth = inf;
    // Seed the k smallest with the sorted neighbourhood of the wave's 64
    // queries (Morton order keeps it close), so that the walk from the root
    // prunes with a small k-th distance from its first levels; the walk then
    // skips the positions scanned here.
    const int w0 = blockIdx.x * kWave;
    const int pre_lo = max(max(w0 - kKnnSeed, 0), lo_r);
    const int pre_hi = min(min(w0 + kWave + kKnnSeed, n), hi_r);
    // the wave loads the candidate rows into LDS together (coalesced), then
    // every lane reads them from there: one memory round trip per batch of
    // rows instead of one per row
    // rows (the window is the same for the whole wave; in a batched solve a
    // lane skips the rows of other instances)
    const int win_lo = max(w0 - kKnnSeed, 0), win_hi = min(w0 + kWave + kKnnSeed, n);
    for (int r = lane_id(); r < win_hi - win_lo; r += kWave)
#pragma unroll
        for (int k = 0; k < D; ++k) rows[r * D + k] = t.X[(size_t)(win_lo + r) * D + k];
    __syncthreads();
    for (int j = win_lo; j < win_hi; ++j) {
        if (j < pre_lo || j >= pre_hi) continue;
        double dd = sqdist<D>(q, rows + (j - win_lo) * D);
        if (dd < kth) {
            topk_insert<KMAX>(top, dd);
            kth = top[KMAX - 1];
        }
    }
    const NodeRec<D>* N = nodes_of<D>(t);
    __syncthreads();  // the seed rows are read before the stack reuses them
    if (lane_id() == 0) stack[0] = knn_entry<D>(n, 0, N[0]);  // root (the single leaf when n == 1)
    int sp = 1;
    __syncthreads();
    while (sp > 0) {
        --sp;
        const int ex = __builtin_amdgcn_readfirstlane(stack[sp].x);
        const int ey = __builtin_amdgcn_readfirstlane(stack[sp].y);
        __syncthreads();
        if (ex < 0) {
            // A node of at most kKnnLeaf points: its rows are loaded together
            // with its record and staged before the bound is tested (a row
            // past the node is loaded when it exists and never read).
            const int v = ~ex, f = ey;
            const int row = f + lane_id();
            if (lane_id() < kKnnLeaf && row < n)
#pragma unroll
                for (int k = 0; k < D; ++k) rows[lane_id() * D + k] = t.X[(size_t)row * D + k];
            const double lb = point_box_lb2<D>(q, N[v].lo, N[v].hi);
            const int c = __builtin_amdgcn_readfirstlane(N[v].count);
            const bool want = live && lb < kth && f < hi_r && f + c > lo_r;
            if (!__any(want)) continue;
            __syncthreads();
            // A node outside the seed window and inside every lane's
            // instance needs no per-row test beyond the distance itself.
            const bool plain = (f >= win_hi || f + c <= win_lo) && f >= lo_all && f + c <= hi_all;
            if (plain) {
                int i = 0;
                for (; i + 4 <= c; i += 4) {
                    double dd[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) dd[u] = sqdist<D>(q, rows + (i + u) * D);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (dd[u] < kth) {
                            topk_insert<KMAX>(top, dd[u]);
                            kth = top[KMAX - 1];
                        }
                }
                for (; i < c; ++i) {
                    const double dd = sqdist<D>(q, rows + i * D);
                    if (dd < kth) {
                        topk_insert<KMAX>(top, dd);
                        kth = top[KMAX - 1];
                    }
                }
            } else {
                for (int i = 0; i < c; ++i) {
                    const int j = f + i;
                    const double dd = sqdist<D>(q, rows + i * D);
                    if (dd < kth && (j < pre_lo || j >= pre_hi) && j >= lo_r && j < hi_r) {  // not seeded, own instance
                        topk_insert<KMAX>(top, dd);
                        kth = top[KMAX - 1];
                    }
                }
            }
            __syncthreads();  // the rows are read before the next node is staged
        } else {
            // An internal node: the children's records are loaded at once.
            // A child goes on the stack only if some lane may still want it
            // (its range meets the lane's instance and its bound is below the
            // lane's k-th distance): the k-th distances only shrink, so a
            // child no lane wants now is never wanted later.  A child's box
            // lies inside its parent's and the bound is monotone in the box,
            // so a parent that no lane wants any more pushes nothing.  The
            // child nearer to the queries of most lanes is visited first.
            const NodeRec<D>& A = N[ex];
            const NodeRec<D>& B = N[ey];
            const double la = point_box_lb2<D>(q, A.lo, A.hi);
            const double lb = point_box_lb2<D>(q, B.lo, B.hi);
            const int af = A.first, ac = A.count, bf = B.first, bc = B.count;
            const bool wa = __any(live && la < kth && af < hi_r && af + ac > lo_r);
            const bool wb = __any(live && lb < kth && bf < hi_r && bf + bc > lo_r);
            if (!wa && !wb) continue;
            if (sp + 2 > kKnnStack) {
                if (lane_id() == 0) atomicOr(err, 4u);
                continue;
            }
            const bool bfirst = __popcll(__ballot(la <= lb)) >= 32;  // b pushed first, popped second
            const int2 ea = knn_entry<D>(n, ex, A), eb = knn_entry<D>(n, ey, B);
            const int2 first = bfirst ? eb : ea, second = bfirst ? ea : eb;
            const bool wfirst = bfirst ? wb : wa, wsecond = bfirst ? wa : wb;
            if (lane_id() == 0) {
                if (wfirst) stack[sp] = first;
                if (wsecond) stack[sp + (wfirst ? 1 : 0)] = second;
            }
            sp += (wfirst ? 1 : 0) + (wsecond ? 1 : 0);
            __syncthreads();
        }
    }
    if (live) cd2_out[p] = top[KMAX - 1];
}

}  // namespace geomst
