// Approximate OPTICS (paper Appendix, "Parallel Approximate OPTICS", after
// Gan and Tao): the MST of an approximate base graph built on a
// well-separated pair decomposition with separation s = sqrt(8 / rho).
//
// For every well-separated pair (A, B) the base graph holds, by the four
// cases of the Appendix (a node X is "large" when |X| >= minPts):
//   neither large   every point of A with every point of B;
//   only A large    the representative of A with every point of B;
//   only B large    every point of A with the representative of B;
//   both large      the two representatives;
// with weight max{cd(u), cd(v), d(u, v) / (1 + rho)}.  As in the paper's
// implementation each pair contributes the lightest of its edges (under the
// total order K = (w^2, d^2, min id, max id)), and the MST of these candidates
// is the result.  The paper draws the representative points at random; here
// a node's representative is its first point in tree order, so the result is
// deterministic.
//
// The decomposition is the FindPair recursion of Alg. 1 from the children of
// every internal node, one breadth-first level per launch, with the sphere
// test of Sec. 2.3: A and B are separated when balls of the common radius
// r = max(rA, rB) about the box midpoints (rX half the box diagonal) are at
// least s r apart, i.e. |cA - cB| >= (s + 2) r, evaluated on squares.  There
// is no beta threshold and no connectivity pruning in the decomposition:
// every pair yields its candidate; a filtered Kruskal over the candidates
// follows (below).
#pragma once
#include "round_kernels.h"

namespace geomst {

struct ApproxArgs {
    Counters* cnt;
    double K;         // (s + 2)^2
    double q;         // (1 + rho)^2
    int min_pts;
    PairRec* qout;    // next level (room for two children per input pair)
    EdgeList c;       // candidates (room for one per input pair beyond the count)
};

template <int D>
__device__ __forceinline__ double approx_diag2(const NodeRec<D>& A) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t = (double)A.hi[k] - (double)A.lo[k];
        s = s + t * t;
    }
    return s;
}

// Sec. 2.3 separation on the boxes' bounding balls (squares, no rounding of
// a square root enters the decision).
template <int D>
__device__ __forceinline__ bool approx_separated(const NodeRec<D>& A, const NodeRec<D>& B, double K, double dA,
                                                 double dB) {
    double dc2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t = 0.5 * ((double)A.lo[k] + (double)A.hi[k]) - 0.5 * ((double)B.lo[k] + (double)B.hi[k]);
        dc2 = dc2 + t * t;
    }
    const double r2 = 0.25 * fmax(dA, dB);
    return dc2 >= K * r2;
}

// Base-graph edge between sorted positions i and j.
template <int D>
__device__ __forceinline__ EKey approx_key(const TreeView& t, double q, u32 i, u32 j) {
    double e2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double x = t.X[(size_t)i * D + k] - t.X[(size_t)j * D + k];
        e2 = e2 + x * x;
    }
    EKey key;
    key.w2 = fmax(fmax(t.cd2[i], t.cd2[j]), e2 / q);
    key.e2 = e2;
    const u32 oi = t.orig[i], oj = t.orig[j];
    key.lo = oi < oj ? oi : oj;
    key.hi = oi < oj ? oj : oi;
    return key;
}

using ApproxAlloc = BlockAllocN<2, 16>;
constexpr int kApproxBlock = 256;

// One level of the decomposition: lane v takes pair qin[v].  A separated
// pair writes its candidate edge (the case's lightest); any other pair is
// replaced by the two pairs (child, other) of the node with the larger box
// diagonal (ties: more points, then A; a one-point node is never split).
template <int D>
__global__ void __launch_bounds__(kApproxBlock) k_approx_level(TreeView t, ApproxArgs r, const PairRec* qin, u32 nq) {
    __shared__ ApproxAlloc S;
    __shared__ unsigned long long shs[kApproxBlock / kWave];
    const NodeRec<D>* N = nodes_of<D>(t);
    u32* ctr[2] = {&r.cnt->c[C_QN], &r.cnt->c[C_C]};
    unsigned long long visits = 0, evals = 0, sep = 0;
    const u32 stride = gridDim.x * kApproxBlock;
    for (u32 v0 = blockIdx.x * kApproxBlock; v0 < nq; v0 += stride) {
        const u32 v = v0 + threadIdx.x;
        bool cand = false, split = false;
        EdgeOut e;
        PairRec c0, c1;
        if (v < nq) {
            const PairRec p = qin[v];
            const NodeRec<D> A = N[p.a], B = N[p.b];
            const double dA = approx_diag2<D>(A), dB = approx_diag2<D>(B);
            ++visits;
            if (approx_separated<D>(A, B, r.K, dA, dB)) {
                const bool bigA = A.count >= r.min_pts, bigB = B.count >= r.min_pts;
                const u32 a0 = (u32)A.first, a1 = bigA ? a0 + 1 : a0 + (u32)A.count;
                const u32 b0 = (u32)B.first, b1 = bigB ? b0 + 1 : b0 + (u32)B.count;
                EKey best = approx_key<D>(t, r.q, a0, b0);
                u32 bi = a0, bj = b0;
                for (u32 i = a0; i < a1; ++i)
                    for (u32 j = b0; j < b1; ++j) {
                        const EKey k = approx_key<D>(t, r.q, i, j);
                        if (key_less(k, best)) {
                            best = k;
                            bi = i;
                            bj = j;
                        }
                    }
                evals += (unsigned long long)(a1 - a0) * (b1 - b0);
                ++sep;
                e.k = best;
                e.i = bi;
                e.j = bj;
                cand = true;
            } else {
                const bool split_a =
                    (B.count == 1) || (A.count > 1 && (dA > dB || (dA == dB && A.count >= B.count)));
                const NodeRec<D>& X = split_a ? A : B;
                const u32 oth = split_a ? p.b : p.a;
                const int2 ch = node_kids(t.n, X.first, X.count, X.split);
                c0.a = (u32)ch.x;
                c0.b = oth;
                c0.lb2 = 0.0;
                c1.a = (u32)ch.y;
                c1.b = oth;
                c1.lb2 = 0.0;
                split = true;
            }
        }
        const u32 cnt[2] = {split ? 2u : 0u, cand ? 1u : 0u};
        u32 off[2];
        block_alloc(S, cnt, ctr, off);
        // room for every append was made before the launch
        if (split) {
            r.qout[off[0]] = c0;
            r.qout[off[0] + 1] = c1;
        }
        if (cand) put_edge(r.c, off[1], e);
    }
    visits = block_sum_u64(visits, shs);
    evals = block_sum_u64(evals, shs);
    sep = block_sum_u64(sep, shs);
    if (threadIdx.x == 0 && visits) {
        atomicAdd(&r.cnt->c64[C64_VISITS], visits);
        atomicAdd(&r.cnt->c64[C64_EVALS], evals);
        atomicAdd(&r.cnt->c64[C64_BCCP], sep);
    }
}

// Filtered Kruskal over the candidates (as the exact path filters pairs by
// rounds of growing weight): a threshold t splits the remaining candidates
// into the light ones (w2 bit pattern below t), which go to Kruskal, and the
// heavy ones, which are kept only while their ends lie in different
// components.  Every light key precedes every heavy key in K, so taking the
// light ones first and dropping heavy edges inside a component (cycle
// property) gives the same tree as one Kruskal pass over all candidates.

// Every step-th squared weight of the list (the sample the threshold is
// taken from).
__global__ void k_sample_w2(const double* w2, u64 m, u64 step, u32 ns, double* out) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) out[i] = w2[(u64)i * step < m ? (u64)i * step : m - 1];
}

constexpr int kPartBlock = 256;
using PartAlloc = BlockAllocN<2, 16>;

// Light candidates to `light` (counter c[C_QN]; room for cap_light of them:
// the caller sees a larger count and takes another route); heavy ones whose
// ends are still in different components to `heavy` (counter c[C_C]; room for
// every input).
__global__ void __launch_bounds__(kPartBlock) k_partition_cand(EdgeList in, u32 m, u64 tbits, EdgeList light,
                                                               u32 cap_light, EdgeList heavy, u32* parent,
                                                               Counters* cnt) {
    __shared__ PartAlloc S;
    u32* ctr[2] = {&cnt->c[C_QN], &cnt->c[C_C]};
    const u32 stride = gridDim.x * kPartBlock;
    for (u32 v0 = blockIdx.x * kPartBlock; v0 < m; v0 += stride) {
        const u32 v = v0 + threadIdx.x;
        bool lt = false, hv = false;
        double w2 = 0.0, e2 = 0.0;
        u64 ids = 0, pos = 0;
        if (v < m) {
            w2 = in.w2[v];
            e2 = in.e2[v];
            ids = in.ids[v];
            pos = in.pos[v];
            if ((u64)__double_as_longlong(w2) < tbits) {
                lt = true;
            } else {
                const u32 a = uf_find(parent, (u32)(pos >> 32), cnt), b = uf_find(parent, (u32)pos, cnt);
                hv = a != b;
            }
        }
        const u32 c2[2] = {lt ? 1u : 0u, hv ? 1u : 0u};
        u32 off[2];
        block_alloc(S, c2, ctr, off);
        if (lt && off[0] < cap_light) put_edge_raw(light, off[0], w2, e2, ids, pos);  // else: counted, not kept
        if (hv) put_edge_raw(heavy, off[1], w2, e2, ids, pos);
    }
}

// Weight buckets of the candidates: bucket b holds the candidates whose w2
// bit pattern is at least t[b-1] and below t[b] (t ascending; the last
// bucket is open above).  Counted first, then scattered into one list laid
// out bucket after bucket, so the filtered Kruskal moves every candidate
// once.
constexpr int kMaxBuckets = 8;
struct Buckets {
    u64 t[kMaxBuckets - 1];
    int nt;  // thresholds in use; nt + 1 buckets
};

__device__ __forceinline__ int bucket_of(const Buckets& bk, double w2) {
    const u64 x = (u64)__double_as_longlong(w2);
    int b = 0;
#pragma unroll
    for (int i = 0; i < kMaxBuckets - 1; ++i) b += (i < bk.nt && x >= bk.t[i]) ? 1 : 0;
    return b;
}

__global__ void __launch_bounds__(kPartBlock) k_bucket_count(const double* w2, u32 m, Buckets bk, u32* counts) {
    __shared__ u32 h[kMaxBuckets];
    if (threadIdx.x < kMaxBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    for (u32 v = blockIdx.x * kPartBlock + threadIdx.x; v < m; v += gridDim.x * kPartBlock)
        atomicAdd(&h[bucket_of(bk, w2[v])], 1u);
    __syncthreads();
    if (threadIdx.x <= (unsigned)bk.nt && h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

using BucketAlloc = BlockAllocN<kMaxBuckets, 16>;

// Scatter: bucket b's candidates go to out[base[b] + k], k from cursor[b].
__global__ void __launch_bounds__(kPartBlock) k_bucket_scatter(EdgeList in, u32 m, Buckets bk, EdgeList out,
                                                               Buckets base, u32* cursor) {
    __shared__ BucketAlloc S;
    u32* ctr[kMaxBuckets];
#pragma unroll
    for (int i = 0; i < kMaxBuckets; ++i) ctr[i] = i <= bk.nt ? cursor + i : nullptr;
    const u32 stride = gridDim.x * kPartBlock;
    for (u32 v0 = blockIdx.x * kPartBlock; v0 < m; v0 += stride) {
        const u32 v = v0 + threadIdx.x;
        int b = -1;
        double w2 = 0.0, e2 = 0.0;
        u64 ids = 0, pos = 0;
        if (v < m) {
            w2 = in.w2[v];
            e2 = in.e2[v];
            ids = in.ids[v];
            pos = in.pos[v];
            b = bucket_of(bk, w2);
        }
        u32 c[kMaxBuckets];
#pragma unroll
        for (int i = 0; i < kMaxBuckets; ++i) c[i] = b == i ? 1u : 0u;
        u32 off[kMaxBuckets];
        block_alloc(S, c, ctr, off);
        if (b >= 0) {
            u32 o = 0;
            u64 bs = 0;
#pragma unroll
            for (int i = 0; i < kMaxBuckets; ++i)
                if (b == i) {
                    o = off[i];
                    bs = i == 0 ? 0ull : base.t[i - 1];
                }
            put_edge_raw(out, (u32)(bs + o), w2, e2, ids, pos);
        }
    }
}

}  // namespace geomst
