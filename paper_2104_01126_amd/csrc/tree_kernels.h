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
#include "common.h"

namespace geomst {

struct TreeView {
    int n;              // points
    const double* X;    // sorted points, row-major [n][D]
    const u32* orig;    // sorted position -> caller row index
    const double* cd2;  // sorted position -> squared core distance, or null (EMST)
    const double* box;  // [2n-1][2D]: lo[0..D) then hi[0..D)
    const double* rad;  // [2n-1] radius of the sphere about the box centre
    const int2* rng;    // [2n-1] (first sorted position, count)
    const int2* kids;   // [n-1] (left, right) node ids of internal nodes
    const double2* cdb; // [2n-1] (min cd2, max cd2) over the node (HDBSCAN*)
    const int* comp;    // [2n-1] component shared by all the node's points, or -1
};
// Node ids: internal nodes 0..n-2 (0 is the root), the leaf of sorted
// position p is node n-1+p.

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

template <int D>
__global__ void k_bbox_final(const double* partial, int nb, double* bbox) {
    int k = threadIdx.x;
    if (k >= 2 * D) return;
    double v = partial[k];
    for (int b = 1; b < nb; ++b) {
        double x = partial[(size_t)b * 2 * D + k];
        v = (k < D) ? fmin(v, x) : fmax(v, x);
    }
    bbox[k] = v;
}

// ------------------------------------------------------------ Morton code
template <int D>
__device__ __forceinline__ int morton_bits() {
    return (63 / D) > 31 ? 31 : (63 / D);
}

template <int D>
__global__ void k_morton(const double* P, int n, const double* bbox, u64* key, u32* val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = morton_bits<D>();
    const double top = (double)((1ull << b) - 1);
    u64 q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double lo = bbox[k], hi = bbox[D + k];
        double r = hi - lo;
        double t = r > 0.0 ? (P[(size_t)i * D + k] - lo) / r : 0.0;
        double f = floor(t * top);
        f = f < 0.0 ? 0.0 : (f > top ? top : f);
        q[k] = (u64)f;
    }
    u64 c = 0;
    for (int bit = b - 1; bit >= 0; --bit) {
#pragma unroll
        for (int k = 0; k < D; ++k) c = (c << 1) | ((q[k] >> bit) & 1ull);
    }
    key[i] = c;
    val[i] = (u32)i;
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
// Common-prefix length of the codes at sorted positions i and j (equal codes
// are told apart by their positions), -1 outside [0, n).
__device__ __forceinline__ int prefix_len(const u64* k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    u64 a = k[i], b = k[j];
    if (a == b) return 64 + __clz((int)(i ^ j));
    return __clzll((long long)(a ^ b));
}

__global__ void k_karras(const u64* k, int n, int2* rng, int2* kids, int* parent) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int dir = (prefix_len(k, n, i, i + 1) - prefix_len(k, n, i, i - 1)) > 0 ? 1 : -1;
    int dmin = prefix_len(k, n, i, i - dir);
    int lmax = 2;
    while (prefix_len(k, n, i, i + lmax * dir) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(k, n, i, i + (l + t) * dir) > dmin) l += t;
    int j = i + l * dir;
    int dnode = prefix_len(k, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(k, n, i, i + (s + t) * dir) > dnode) s += t;
    } while (t > 1);
    int g = i + s * dir + (dir < 0 ? -1 : 0);
    int first = min(i, j), last = max(i, j);
    int left = (first == g) ? (n - 1 + g) : g;
    int right = (last == g + 1) ? (n - 1 + g + 1) : (g + 1);
    rng[i] = make_int2(first, last - first + 1);
    kids[i] = make_int2(left, right);
    parent[left] = i;
    parent[right] = i;
    if (i == 0) parent[0] = -1;
}

// ------------------------------------------------------------ node bounds
// Leaves take their point's box; every internal node is finished by the
// second of its two children to arrive (bottom-up climb with arrival counters).
template <int D>
__device__ __forceinline__ void merge_node(int v, const int2* kids, double* box, double* rad, double2* cdb,
                                           bool geometry, bool cdbounds) {
    int2 c = kids[v];
    if (geometry) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double lo = fmin(box[(size_t)c.x * 2 * D + k], box[(size_t)c.y * 2 * D + k]);
            double hi = fmax(box[(size_t)c.x * 2 * D + D + k], box[(size_t)c.y * 2 * D + D + k]);
            box[(size_t)v * 2 * D + k] = lo;
            box[(size_t)v * 2 * D + D + k] = hi;
            double t = hi - lo;
            s = s + t * t;
        }
        rad[v] = 0.5 * sqrt(s);
    }
    if (cdbounds) {
        double2 a = cdb[c.x], b = cdb[c.y];
        cdb[v] = make_double2(fmin(a.x, b.x), fmax(a.y, b.y));
    }
}

template <int D>
__global__ void k_bounds(int n, const double* X, const double* cd2, const int2* kids, const int* parent,
                         double* box, double* rad, double2* cdb, int2* rng, u32* flags, int geometry,
                         int cdbounds) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int leaf = n - 1 + p;
    if (geometry) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double x = X[(size_t)p * D + k];
            box[(size_t)leaf * 2 * D + k] = x;
            box[(size_t)leaf * 2 * D + D + k] = x;
        }
        rad[leaf] = 0.0;
        rng[leaf] = make_int2(p, 1);
    }
    if (cdbounds) cdb[leaf] = make_double2(cd2[p], cd2[p]);
    int v = parent[leaf];
    while (v >= 0) {
        __threadfence();
        u32 old = atomicAdd(&flags[v], 1u);
        if (old == 0) return;  // the sibling's thread finishes this node
        __threadfence();
        merge_node<D>(v, kids, box, rad, cdb, geometry, cdbounds);
        v = parent[v];
    }
}

// ------------------------------------------------------------ core distances
// One wave per 64 consecutive sorted points.  The wave walks the tree once,
// descending into a node while any lane's box distance beats its current
// k-th smallest squared distance; nodes of at most kLeafScan points are
// scanned by all lanes (each lane against every point of the node).  The
// per-lane k smallest values are kept sorted in registers.
constexpr int kKnnLeaf = 32;
constexpr int kKnnStack = 192;

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
template <int D>
__device__ __forceinline__ double point_box_lb2(const double (&q)[D], const double* bx) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double g = fmax(fmax(bx[k] - q[k], q[k] - bx[D + k]), 0.0);
        s = s + g * g;
    }
    return s;
}

template <int D, int KMAX>
__global__ void __launch_bounds__(64) k_knn(TreeView t, int kk, double* cd2_out, u32* err) {
    __shared__ int stack[kKnnStack];
    const int n = t.n;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    int p = blockIdx.x * kWave + lane_id();
    bool live = p < n;
    int pq = live ? p : n - 1;
    double q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) q[k] = t.X[(size_t)pq * D + k];
    // slots [0, KMAX-kk) hold -inf so that the kk-th smallest value seen is
    // always in the last slot
    double top[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s) top[s] = (s < KMAX - kk) ? -inf : inf;
    double kth = inf;
    if (lane_id() == 0) stack[0] = 0;  // root (the single leaf when n == 1)
    int sp = 1;
    __syncthreads();
    while (sp > 0) {
        --sp;
        int v = stack[sp];
        __syncthreads();
        double lb = point_box_lb2<D>(q, t.box + (size_t)v * 2 * D);
        bool want = live && lb < kth;
        if (!__any(want)) continue;
        int2 r = t.rng[v];
        if (r.y <= kKnnLeaf) {
            for (int j = r.x; j < r.x + r.y; ++j) {
                double dd = sqdist<D>(q, t.X + (size_t)j * D);
                if (dd < kth) {
                    topk_insert<KMAX>(top, dd);
                    kth = top[KMAX - 1];
                }
            }
        } else {
            if (sp + 2 > kKnnStack) {
                if (lane_id() == 0) atomicOr(err, 4u);
                continue;
            }
            int2 c = t.kids[v];
            // visit first the child nearer to lane 0's query
            double la = point_box_lb2<D>(q, t.box + (size_t)c.x * 2 * D);
            double lr = point_box_lb2<D>(q, t.box + (size_t)c.y * 2 * D);
            bool leftfirst = __shfl(la <= lr ? 1 : 0, 0) != 0;
            if (lane_id() == 0) {
                stack[sp] = leftfirst ? c.y : c.x;
                stack[sp + 1] = leftfirst ? c.x : c.y;
            }
            sp += 2;
            __syncthreads();
        }
    }
    if (live) cd2_out[p] = top[KMAX - 1];
}

}  // namespace geomst
