// Ordered dendrogram and reachability plot of a weighted spanning tree
// (Sec. 2.1 "dendrogram", "reachability plot"; Sec. 4, the top-down
// heavy/light construction; Sec. 4.1, the ordered dendrogram of a start
// vertex s).
//
// Input: the n-1 tree edges in their total order (edge k is the k-th
// lightest), so internal node n + k of the dendrogram is edge k.  Output:
// the two children of every internal node (left = the cluster that holds the
// endpoint nearer to s), its point count, and the plot (Prim's visiting order
// from s on the tree, with the weight of the edge that reached each point).
//
// Steps (all data parallel):
//  1. Root the tree at s: Euler tour over the arcs sorted by source vertex,
//     list ranking by pointer jumping; an arc that comes before its twin in
//     the tour points away from s.  This gives, for every edge, its endpoint
//     nearer to s and, for every point, the edge towards s (the edge Prim
//     reaches it by: the visited set is a subtree holding s).
//  2. Children by heavy/light halving.  Edges [a, b) of one subproblem act on
//     the clusters formed by all edges below a; it splits into the light half
//     [a, mid), on the same clusters, and the heavy half [mid, b), on the
//     clusters after the light half has merged them.  A cluster is named by
//     its dendrogram root (a leaf id, or n + its heaviest edge), so the heavy
//     half's endpoints are renamed to the root of their light component: this
//     is where the light subproblems' dendrograms attach below the heavy
//     one.  Halving all blocks of one size at once gives one level; after the
//     level of blocks of two, each edge's two endpoint names are its children.
//     Within a level every cluster name occurs in one block only (a later
//     block's clusters already contain an earlier block's edges, so they
//     carry a larger root), so one union-find over node ids serves all blocks
//     of the level at once.
//  3. In-order positions: the left child's point count is added along every
//     path to the root (pointer jumping over the dendrogram); the leaves'
//     positions are the plot order (Sec. 4.1: the in-order traversal of the
//     ordered dendrogram is the reachability plot).
#pragma once
#include "common.h"

namespace geomst {

constexpr u32 kDgErrIds = 1u;   // an endpoint out of range, a self-loop, or a bad start
constexpr u32 kDgErrTree = 2u;  // the edges do not connect every point to the start
constexpr u32 kDgErrPos = 4u;   // internal: a position outside [0, n)

__device__ __forceinline__ u32 dg_load(const u32* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dg_store(u32* p, u32 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Edge k -> arcs 2k (u -> v) and 2k+1 (v -> u), keyed by their source.
__global__ void k_dg_load(const long long* edges, u32 m, u32 n, u32* eu, u32* ev, u64* akey, u32* aval, u32* err) {
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const long long a = edges[2 * (size_t)k], b = edges[2 * (size_t)k + 1];
    const bool bad = a < 0 || b < 0 || a >= (long long)n || b >= (long long)n || a == b;
    const u32 u = bad ? 0u : (u32)a, v = bad ? 1u : (u32)b;  // n >= 2 here
    if (bad) atomicOr(err, kDgErrIds);
    eu[k] = u;
    ev[k] = v;
    akey[2 * k] = u;
    aval[2 * k] = 2 * k;
    akey[2 * k + 1] = v;
    aval[2 * k + 1] = 2 * k + 1;
}

// Sorted arcs: position of every arc, and the first position of each source.
__global__ void k_dg_adj(const u64* skey, const u32* sarc, u32 na, u32* pos, u32* first) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na) return;
    pos[sarc[i]] = i;
    if (i == 0 || skey[i - 1] != skey[i]) first[(u32)skey[i]] = i;
}

// Euler tour successor: after arc (x -> y) comes the arc that follows
// (y -> x) around y (cyclically).  The tour starts with s's first arc, so the
// arc leading back into it ends the list.  Also starts the list ranking:
// nx = successor, dd = 1 (0 at the end).
__global__ void k_dg_succ(const u64* skey, const u32* sarc, const u32* pos, const u32* first, u32 na, u32 s,
                          u32* nx, u32* dd, u32* err) {
    const u32 a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    const u32 f = first[s];
    if (f == kNone) {  // the start has no edge
        if (a == 0) atomicOr(err, kDgErrTree);
        nx[a] = kNone;
        dd[a] = 0;
        return;
    }
    const u32 a0 = sarc[f];
    const u32 t = a ^ 1u;
    const u32 y = (u32)skey[pos[t]];  // source of the twin = head of a
    u32 p = pos[t] + 1;
    if (p == na || (u32)skey[p] != y) p = first[y];
    const u32 nxt = sarc[p];
    nx[a] = nxt == a0 ? kNone : nxt;
    dd[a] = nxt == a0 ? 0u : 1u;
}

// One pointer-jumping round of list ranking: dd = arcs after a in the tour.
__global__ void k_dg_jump(const u32* nx_in, const u32* dd_in, u32* nx_out, u32* dd_out, u32 na) {
    const u32 a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    const u32 j = nx_in[a];
    if (j == kNone) {
        nx_out[a] = kNone;
        dd_out[a] = dd_in[a];
    } else {
        nx_out[a] = nx_in[j];
        dd_out[a] = dd_in[a] + dd_in[j];
    }
}

// Orientation from the ranks: arc (x -> y) before its twin points away from
// s, so x is the endpoint nearer to s and edge k is y's edge towards s.
__global__ void k_dg_orient(const u32* eu, const u32* ev, const u32* nx, const u32* dd, u32 m, unsigned char* near_u,
                            u32* pedge, u32* err) {
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    if (nx[2 * k] != kNone || nx[2 * k + 1] != kNone) {  // an arc off the tour: not one tree
        atomicOr(err, kDgErrTree);
        return;
    }
    const bool down = dd[2 * k] > dd[2 * k + 1];
    near_u[k] = down ? 1 : 0;
    pedge[down ? ev[k] : eu[k]] = k;
}

// Heavy/light levels.  lab[side * m + k] is the name (dendrogram node id) of
// the cluster of edge k's endpoint on `side` (0 = u, 1 = v) in the clusters
// of k's current block; sz the cluster's point count.  In the level of
// blocks of size 2^j, edge k is light when bit j-1 of k is 0.
__device__ __forceinline__ bool dg_light(u32 k, int j) { return ((k >> (j - 1)) & 1u) == 0u; }

// Level set-up: every name used by the level starts as its own root with no
// light edge, no size and no size contribution yet.
__global__ void k_dg_level_reset(const u32* lab, u32 m, u32* P, u32* MX, u32* SZ, u32* OWN) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * m) return;
    const u32 x = lab[i];
    P[x] = x;
    MX[x] = 0;
    SZ[x] = 0;
    OWN[x] = 0;
}

// Path halving; every parent has a smaller id than its child, so walks end.
__device__ __forceinline__ u32 dg_find(u32* P, u32 x) {
    while (true) {
        const u32 p = dg_load(&P[x]);
        if (p == x) return x;
        const u32 g = dg_load(&P[p]);
        if (g != p) dg_store(&P[x], g);
        x = g;
    }
}

// Union of the light edges' endpoint clusters (the larger root hooks under
// the smaller, by compare-and-swap on the root's own entry).
__global__ void k_dg_level_union(const u32* lab, u32 m, int j, u32* P) {
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m || !dg_light(k, j)) return;
    u32 a = lab[k], b = lab[m + k];
    while (true) {
        a = dg_find(P, a);
        b = dg_find(P, b);
        if (a == b) return;
        if (a < b) {
            const u32 t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&P[a], a, b) == a) return;
    }
}

// Per light component: its heaviest edge (the new cluster's root) and its
// point count (each member cluster's count added once, by the first lane to
// claim its name).  In the first levels a block's light half forms a few
// huge components, and one atomic per edge on their roots would serialise:
// lanes whose root equals the first remaining lane's root combine their
// values in the wave first (two such rounds), the others update directly.
__device__ __forceinline__ u32 wave_max_u32(u32 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (u32)__shfl_xor((int)v, o));
    return v;
}
__device__ __forceinline__ u32 wave_sum_u32(u32 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (u32)__shfl_xor((int)v, o);
    return v;
}

__global__ void k_dg_level_info(const u32* lab, const u32* sz, u32 m, int j, u32* P, u32* MX, u32* SZ, u32* OWN) {
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = k < m && dg_light(k, j);
    u32 r = 0, add = 0;
    if (act) {
        const u32 a = lab[k], b = lab[m + k];
        r = dg_find(P, a);
        if (atomicCAS(&OWN[a], 0u, 1u) == 0u) add += sz[k];
        if (atomicCAS(&OWN[b], 0u, 1u) == 0u) add += sz[m + k];
    }
    bool mine = act;  // this lane's values are still to be applied
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        const u64 left = __ballot(mine);
        if (!left) break;
        const int leader = __ffsll((long long)left) - 1;
        const u32 rl = (u32)__shfl((int)r, leader);
        const bool same = mine && r == rl;
        const u32 mx = wave_max_u32(same ? k + 1 : 0u);
        const u32 sm = wave_sum_u32(same ? add : 0u);
        if (lane_id() == leader) {
            atomicMax(&MX[rl], mx);
            if (sm) atomicAdd(&SZ[rl], sm);
        }
        if (same) mine = false;
    }
    if (mine) {
        atomicMax(&MX[r], k + 1);
        if (add) atomicAdd(&SZ[r], add);
    }
}

// Heavy edges of blocks that have a light half: rename each endpoint cluster
// to the root of its light component (unchanged if no light edge touched it).
__global__ void k_dg_level_rename(u32* lab, u32* sz, u32 m, u32 n, int j, u32* P, const u32* MX, const u32* SZ) {
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m || dg_light(k, j)) return;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const u32 i = side * m + k;
        const u32 r = dg_find(P, lab[i]);
        const u32 mx = MX[r];
        if (mx != 0) {
            lab[i] = n + (mx - 1);
            sz[i] = SZ[r];
        }
    }
}

// Children of each internal node, oriented by the start; parent links and
// in-order offsets (a right child follows its left sibling's points).
__global__ void k_dg_children(const u32* lab, const u32* sz, const unsigned char* near_u, u32 m, u32 n, long long* children,
                              long long* size, u32* par, u32* off) {
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const bool ul = near_u[k] != 0;
    const u32 L = ul ? lab[k] : lab[m + k], R = ul ? lab[m + k] : lab[k];
    const u32 sl = ul ? sz[k] : sz[m + k], sr = ul ? sz[m + k] : sz[k];
    if (children) {
        children[2 * (size_t)k] = L;
        children[2 * (size_t)k + 1] = R;
    }
    if (size) size[k] = (long long)sl + sr;
    par[L] = n + k;
    off[L] = 0;
    par[R] = n + k;
    off[R] = sl;
    if (k == m - 1) {  // the heaviest edge is the root
        par[n + k] = kNone;
        off[n + k] = 0;
    }
}

// A single point: the plot is that point at height +inf.
__global__ void k_dg_single(long long* order, double* reach) {
    order[0] = 0;
    reach[0] = __longlong_as_double(0x7ff0000000000000ll);
}

__global__ void k_dg_fill_u32(u32* p, u32 count, u32 v) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Leaves' in-order positions are the plot; each point's height is the weight
// of its edge towards s (the edge Prim reaches it by), +inf for s.
__global__ void k_dg_plot(const u32* pos, const u32* pedge, const double* w, u32 n, u32 s, long long* order,
                          double* reach, u32* err) {
    const u32 x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const u32 p = pos[x];
    if (p >= n || (x == s) != (p == 0)) {
        atomicOr(err, kDgErrPos);
        return;
    }
    order[p] = x;
    reach[p] = x == s ? __longlong_as_double(0x7ff0000000000000ll) : w[pedge[x]];
}

}  // namespace geomst
