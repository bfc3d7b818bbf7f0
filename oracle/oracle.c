/*
 * CPU checker for the Euclidean MST, the HDBSCAN* mutual-reachability MST and
 * the approximate OPTICS MST.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is compared against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg load it; the library never
 * does, and the two share no source, header or table.
 *
 * What is computed (paper Sec. 2.1, "Problem Definitions"):
 *   EMST      the minimum spanning tree of the complete graph on the n points
 *             with Euclidean edge weights.
 *   HDBSCAN*  the core distance cd(p) = distance from p to its minPts-nearest
 *             neighbour counting p itself, the mutual reachability distance
 *             d_m(p,q) = max{cd(p), cd(q), d(p,q)}, and the MST of the
 *             complete graph weighted by d_m.
 *   OPTICS-GanTaoApprox (paper Appendix)  the MST of the approximate base
 *             graph built on a well-separated pair decomposition; its
 *             readings (tree, separation, representatives, edge cases) are
 *             stated at oracle_optics_approx below.
 *
 * Arithmetic and order (readings of a paper that fixes no precision):
 *   d2(p,q) = sum over k = 0..d-1, in that order, of (p_k - q_k)^2 in IEEE
 *             binary64, round to nearest, no fused multiply-add (this file
 *             must be compiled with -ffp-contract=off).  d2 is symmetric bit
 *             for bit because x - y = -(y - x) exactly.
 *   cd2(p)    the minPts-th smallest value of d2(p, j) over all j, including
 *             j = p itself (value 0).
 *   w2(p,q)   d2 for EMST; max(cd2(p), cd2(q), d2(p,q)) for HDBSCAN*.
 *   key       K(p,q) = (w2, d2, min(p,q), max(p,q)) compared
 *             lexicographically.  K is a total order on edges, so the MST is
 *             unique; for EMST it is (weight, min id, max id).
 * The MST is found by textbook dense Prim (O(n^2) time, O(n) memory).  Ties
 * inside Prim are resolved by K, so any start vertex gives the same tree.
 * Reported weights are sqrt(w2) with C's correctly rounded sqrt.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -3

/* ---------------------------------------------------------------- helpers */

/* Squared Euclidean distance, summed in dimension order (definition above). */
static double d2_of(const double *P, int32_t d, int64_t i, int64_t j)
{
    const double *a = P + i * (int64_t)d;
    const double *b = P + j * (int64_t)d;
    double s = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        s = s + t * t;
    }
    return s;
}

typedef struct {
    double w2, e2;
    int64_t lo, hi;
} key_t_;

static key_t_ make_key(const double *P, int32_t d, const double *cd2, int64_t i, int64_t j)
{
    key_t_ k;
    double e2 = d2_of(P, d, i, j);
    double w2 = e2;
    if (cd2) {
        double c = cd2[i] > cd2[j] ? cd2[i] : cd2[j];
        w2 = c > e2 ? c : e2;
    }
    k.w2 = w2;
    k.e2 = e2;
    k.lo = i < j ? i : j;
    k.hi = i < j ? j : i;
    return k;
}

/* strict lexicographic "a < b" on K */
static int key_less(key_t_ a, key_t_ b)
{
    if (a.w2 != b.w2) return a.w2 < b.w2;
    if (a.e2 != b.e2) return a.e2 < b.e2;
    if (a.lo != b.lo) return a.lo < b.lo;
    return a.hi < b.hi;
}

static int key_cmp_qsort(const void *pa, const void *pb)
{
    key_t_ a = *(const key_t_ *)pa, b = *(const key_t_ *)pb;
    if (key_less(a, b)) return -1;
    if (key_less(b, a)) return 1;
    return 0;
}

static int check_points(const double *P, int64_t n, int32_t d)
{
    if (!P && n > 0) return OR_EINVAL;
    if (n < 1 || d < 1) return OR_EINVAL;
    for (int64_t i = 0; i < n * (int64_t)d; ++i)
        if (!isfinite(P[i])) return OR_EINVAL;
    return OR_OK;
}

/* ------------------------------------------------------------ core distance */

/* cd2 of one point: the k-th smallest of d2(i, j) over all j (j = i included).
 * Kept as a sorted list of the k smallest values seen so far. */
static double core_d2_one(const double *P, int64_t n, int32_t d, int32_t k, int64_t i, double *buf)
{
    int32_t len = 0;
    for (int64_t j = 0; j < n; ++j) {
        double v = d2_of(P, d, i, j);
        if (len == k && !(v < buf[k - 1])) continue;
        int32_t pos = (len < k) ? len : k - 1;
        while (pos > 0 && buf[pos - 1] > v) {
            buf[pos] = buf[pos - 1];
            --pos;
        }
        buf[pos] = v;
        if (len < k) ++len;
    }
    return buf[k - 1];
}

/* cd2 for the m query rows idx[0..m) (all rows when idx is NULL, m = n). */
int oracle_core_dist2(const double *P, int64_t n, int32_t d, int32_t min_pts,
                      const int64_t *idx, int64_t m, double *cd2_out)
{
    int rc = check_points(P, n, d);
    if (rc) return rc;
    if (min_pts < 1 || min_pts > n || !cd2_out) return OR_EINVAL;
    if (!idx) m = n;
    int bad = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)min_pts);
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t q = 0; q < m; ++q) {
                int64_t i = idx ? idx[q] : q;
                cd2_out[q] = core_d2_one(P, n, d, min_pts, i, buf);
            }
            free(buf);
        }
    }
    return bad ? OR_ENOMEM : OR_OK;
}

/* ----------------------------------------------------------------- Prim */

/* Dense Prim under K.  cd2 == NULL gives EMST, otherwise the mutual
 * reachability MST.  Outputs sorted by K: edges[k] = (min id, max id),
 * w2[k], e2[k] (e2 may be NULL). */
static int prim_dense(const double *P, int64_t n, int32_t d, const double *cd2,
                      int64_t *edges, double *w2o, double *e2o)
{
    if (n == 1) return OR_OK;
    key_t_ *best = (key_t_ *)malloc(sizeof(key_t_) * (size_t)n);
    unsigned char *in_tree = (unsigned char *)calloc((size_t)n, 1);
    key_t_ *tree = (key_t_ *)malloc(sizeof(key_t_) * (size_t)(n - 1));
    int nth = omp_get_max_threads();
    int64_t *arg = (int64_t *)malloc(sizeof(int64_t) * (size_t)nth);
    if (!best || !in_tree || !tree || !arg) {
        free(best); free(in_tree); free(tree); free(arg);
        return OR_ENOMEM;
    }
    /* start the tree at vertex 0 */
    in_tree[0] = 1;
#pragma omp parallel for schedule(static)
    for (int64_t v = 1; v < n; ++v) best[v] = make_key(P, d, cd2, 0, v);

    int64_t v_new = -1;
    for (int64_t it = 0; it < n - 1; ++it) {
        /* argmin over vertices outside the tree (per thread, then combined) */
#pragma omp parallel
        {
            int t = omp_get_thread_num();
            int64_t a = -1;
#pragma omp for schedule(static)
            for (int64_t v = 0; v < n; ++v) {
                if (in_tree[v]) continue;
                if (a < 0 || key_less(best[v], best[a])) a = v;
            }
            arg[t] = a;
        }
        int64_t a = -1;
        for (int t = 0; t < nth; ++t)
            if (arg[t] >= 0 && (a < 0 || key_less(best[arg[t]], best[a]))) a = arg[t];
        v_new = a;
        tree[it] = best[v_new];
        in_tree[v_new] = 1;
        /* relax the edges of the new vertex */
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < n; ++v) {
            if (in_tree[v]) continue;
            key_t_ k = make_key(P, d, cd2, v_new, v);
            if (key_less(k, best[v])) best[v] = k;
        }
    }
    qsort(tree, (size_t)(n - 1), sizeof(key_t_), key_cmp_qsort);
    for (int64_t k = 0; k < n - 1; ++k) {
        edges[2 * k] = tree[k].lo;
        edges[2 * k + 1] = tree[k].hi;
        if (w2o) w2o[k] = tree[k].w2;
        if (e2o) e2o[k] = tree[k].e2;
    }
    free(best); free(in_tree); free(tree); free(arg);
    return OR_OK;
}

/* EMST: n-1 edges sorted by K, their squared weights and weights. */
int oracle_emst(const double *P, int64_t n, int32_t d, int64_t *edges, double *w2, double *w)
{
    int rc = check_points(P, n, d);
    if (rc) return rc;
    if (n > 1 && (!edges || !w2)) return OR_EINVAL;
    rc = prim_dense(P, n, d, NULL, edges, w2, NULL);
    if (rc) return rc;
    if (w)
        for (int64_t k = 0; k < n - 1; ++k) w[k] = sqrt(w2[k]);
    return OR_OK;
}

/* HDBSCAN*: core distances (squared and plain) and the mutual reachability
 * MST sorted by K, with w2 and e2 (= d2) of each edge. */
int oracle_hdbscan(const double *P, int64_t n, int32_t d, int32_t min_pts,
                   double *cd2, double *cd, int64_t *edges, double *w2, double *e2, double *w)
{
    int rc = check_points(P, n, d);
    if (rc) return rc;
    if (min_pts < 1 || min_pts > n || !cd2) return OR_EINVAL;
    if (n > 1 && (!edges || !w2)) return OR_EINVAL;
    rc = oracle_core_dist2(P, n, d, min_pts, NULL, n, cd2);
    if (rc) return rc;
    if (cd)
        for (int64_t i = 0; i < n; ++i) cd[i] = sqrt(cd2[i]);
    rc = prim_dense(P, n, d, cd2, edges, w2, e2);
    if (rc) return rc;
    if (w)
        for (int64_t k = 0; k < n - 1; ++k) w[k] = sqrt(w2[k]);
    return OR_OK;
}

/* ------------------------------------------------ one-at-a-time queries */

/* K of given edges (for checking sampled outputs at sizes Prim cannot reach):
 * w2[k], e2[k] of the pair (a[k], b[k]). cd2 == NULL means EMST. */
int oracle_edge_keys(const double *P, int64_t n, int32_t d, const double *cd2,
                     const int64_t *a, const int64_t *b, int64_t m, double *w2, double *e2)
{
    if (!P || n < 1 || d < 1 || !a || !b || !w2) return OR_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        key_t_ kk = make_key(P, d, cd2, a[k], b[k]);
        w2[k] = kk.w2;
        if (e2) e2[k] = kk.e2;
    }
    return OR_OK;
}

/* The K-lightest edge leaving the vertex set S (in_s[v] != 0), by exhaustive
 * scan of S x (complement).  By the cut property every MST edge is the
 * lightest edge across the cut that removing it creates; the tests use this
 * at full workload sizes on cuts whose small side is small. */
int oracle_lightest_cut_edge(const double *P, int64_t n, int32_t d, const double *cd2,
                             const unsigned char *in_s, int64_t *lo, int64_t *hi,
                             double *w2, double *e2)
{
    if (!P || n < 2 || !in_s) return OR_EINVAL;
    int64_t ns = 0;
    for (int64_t v = 0; v < n; ++v) ns += in_s[v] ? 1 : 0;
    if (ns == 0 || ns == n) return OR_EINVAL;
    int64_t *s = (int64_t *)malloc(sizeof(int64_t) * (size_t)ns);
    if (!s) return OR_ENOMEM;
    for (int64_t v = 0, c = 0; v < n; ++v)
        if (in_s[v]) s[c++] = v;
    int nth = omp_get_max_threads();
    key_t_ *part = (key_t_ *)malloc(sizeof(key_t_) * (size_t)nth);
    unsigned char *has = (unsigned char *)calloc((size_t)nth, 1);
    if (!part || !has) {
        free(s); free(part); free(has);
        return OR_ENOMEM;
    }
#pragma omp parallel
    {
        int t = omp_get_thread_num();
        key_t_ b = {0.0, 0.0, -1, -1};
        int hb = 0;
#pragma omp for schedule(static)
        for (int64_t v = 0; v < n; ++v) {
            if (in_s[v]) continue;
            for (int64_t q = 0; q < ns; ++q) {
                key_t_ k = make_key(P, d, cd2, s[q], v);
                if (!hb || key_less(k, b)) { b = k; hb = 1; }
            }
        }
        part[t] = b;
        has[t] = (unsigned char)hb;
    }
    key_t_ best = {0.0, 0.0, -1, -1};
    int hb = 0;
    for (int t = 0; t < nth; ++t)
        if (has[t] && (!hb || key_less(part[t], best))) { best = part[t]; hb = 1; }
    *lo = best.lo;
    *hi = best.hi;
    if (w2) *w2 = best.w2;
    if (e2) *e2 = best.e2;
    free(s); free(part); free(has);
    return OR_OK;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------ dendrogram and plot */

/*
 * Ordered dendrogram and reachability plot of a weighted spanning tree
 * (paper Sec. 2.1, "dendrogram" and "reachability plot"; Sec. 4.1, ordered
 * dendrogram of a start vertex s).
 *
 * Input: the n-1 tree edges in the order that is their total order (the MST
 * calls return them sorted by K, so edge k is the k-th lightest), weights[k]
 * the height of edge k, and the start vertex s.
 *
 * Dendrogram (the sequential bottom-up definition of Sec. 4): every point
 * starts as its own cluster (leaf node i, 0 <= i < n); edges are taken in
 * order, and edge k merges the clusters of its two endpoints into internal
 * node n + k, whose height is weights[k] and whose size is the number of
 * points below it.  Ordered: of the two clusters merged by edge (u, v), the
 * one holding the endpoint nearer to s in the tree (fewer tree edges from s,
 * the "vertex distance") is the left child.
 *
 * Reachability plot: the order in which Prim's algorithm run on the tree
 * from s visits the points, always taking the lightest edge (lowest index)
 * leaving the visited set, and for each visited point the weight of the edge
 * that reached it (s gets +infinity).
 *
 * children[k] = {left, right} node ids of internal node n + k; size[k] its
 * point count; order[i] the i-th point of the plot; reach[i] its height.
 * Returns OR_EINVAL if the edges are not a spanning tree of 0..n-1.
 */
static int64_t uf_find(int64_t *par, int64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

/* binary min-heap of edge indices */
static void heap_push(int64_t *h, int64_t *len, int64_t v)
{
    int64_t i = (*len)++;
    h[i] = v;
    while (i > 0 && h[(i - 1) / 2] > h[i]) {
        int64_t p = (i - 1) / 2, t = h[p];
        h[p] = h[i];
        h[i] = t;
        i = p;
    }
}

static int64_t heap_pop(int64_t *h, int64_t *len)
{
    int64_t top = h[0];
    h[0] = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *len && h[l] < h[m]) m = l;
        if (r < *len && h[r] < h[m]) m = r;
        if (m == i) break;
        int64_t t = h[m];
        h[m] = h[i];
        h[i] = t;
        i = m;
    }
    return top;
}

int oracle_dendrogram(const int64_t *edges, const double *weights, int64_t n, int64_t s,
                      int64_t *children, int64_t *size, int64_t *order, double *reach)
{
    if (n < 1 || s < 0 || s >= n || !order || !reach) return OR_EINVAL;
    if (n > 1 && (!edges || !weights || !children || !size)) return OR_EINVAL;
    int64_t m = n - 1;
    for (int64_t k = 0; k < 2 * m; ++k)
        if (edges[k] < 0 || edges[k] >= n) return OR_EINVAL;
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *top = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *heap = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    unsigned char *seen = (unsigned char *)calloc((size_t)n, 1);
    int rc = OR_OK;
    if (!deg || !adj || !fill || !dist || !queue || !par || !top || !cnt || !heap || !seen) {
        rc = OR_ENOMEM;
        goto done;
    }
    /* adjacency lists: edge indices incident to each vertex */
    for (int64_t k = 0; k < m; ++k) {
        deg[edges[2 * k] + 1]++;
        deg[edges[2 * k + 1] + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) deg[v + 1] += deg[v];
    for (int64_t v = 0; v <= n; ++v) fill[v] = deg[v];
    for (int64_t k = 0; k < m; ++k) {
        adj[fill[edges[2 * k]]++] = k;
        adj[fill[edges[2 * k + 1]]++] = k;
    }
    /* vertex distances from s by breadth-first search over the tree */
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    int64_t qh = 0, qt = 0;
    dist[s] = 0;
    queue[qt++] = s;
    while (qh < qt) {
        int64_t x = queue[qh++];
        for (int64_t j = deg[x]; j < deg[x + 1]; ++j) {
            int64_t k = adj[j];
            int64_t y = edges[2 * k] == x ? edges[2 * k + 1] : edges[2 * k];
            if (dist[y] < 0) {
                dist[y] = dist[x] + 1;
                queue[qt++] = y;
            }
        }
    }
    if (qt != n) { /* not connected, hence (with n-1 edges) not a tree */
        rc = OR_EINVAL;
        goto done;
    }
    /* bottom-up merges in edge order (Kruskal's order) */
    for (int64_t v = 0; v < n; ++v) {
        par[v] = v;
        top[v] = v;
        cnt[v] = 1;
    }
    for (int64_t k = 0; k < m; ++k) {
        int64_t u = edges[2 * k], v = edges[2 * k + 1];
        int64_t ru = uf_find(par, u), rv = uf_find(par, v);
        if (ru == rv) { /* a cycle */
            rc = OR_EINVAL;
            goto done;
        }
        int u_left = dist[u] < dist[v];
        children[2 * k] = u_left ? top[ru] : top[rv];
        children[2 * k + 1] = u_left ? top[rv] : top[ru];
        size[k] = cnt[ru] + cnt[rv];
        par[rv] = ru;
        cnt[ru] += cnt[rv];
        top[ru] = n + k;
    }
    /* Prim on the tree from s: lowest-index edge leaving the visited set */
    int64_t hl = 0, no = 0;
    seen[s] = 1;
    order[no] = s;
    reach[no++] = INFINITY;
    for (int64_t j = deg[s]; j < deg[s + 1]; ++j) heap_push(heap, &hl, adj[j]);
    while (hl > 0) {
        int64_t k = heap_pop(heap, &hl);
        int64_t u = edges[2 * k], v = edges[2 * k + 1];
        int64_t y = seen[u] ? v : u;
        if (seen[y]) continue;
        seen[y] = 1;
        order[no] = y;
        reach[no++] = weights[k];
        for (int64_t j = deg[y]; j < deg[y + 1]; ++j)
            if (adj[j] != k) heap_push(heap, &hl, adj[j]);
    }
done:
    free(deg); free(adj); free(fill); free(dist); free(queue); free(par); free(top); free(cnt);
    free(heap); free(seen);
    return rc;
}

/* ------------------------------------------------ approximate OPTICS */

/*
 * OPTICS-GanTaoApprox: the MST of Gan and Tao's approximate base graph, built
 * on a well-separated pair decomposition (paper Appendix, "Parallel
 * Approximate OPTICS").  Parameters minPts and rho >= 0; separation
 * s = sqrt(8 / rho).
 *
 * The result depends on the spatial tree the decomposition runs on, so the
 * tree is part of the definition here (paper Sec. 3.1.1: a spatial-median
 * k-d tree with one point per leaf).  Readings, in the order they are used:
 *
 *  T1 (tree)  The spatial-median k-d tree of quantisation cells: every
 *     point's coordinates are quantised inside the bounding box of all points
 *     to b = min(31, floor(63 / d)) bits per dimension,
 *         q_k = clamp(floor(((x_k - lo_k) / (hi_k - lo_k)) * (2^b - 1)), 0, 2^b - 1)
 *     (q_k = 0 when hi_k = lo_k), and the bits are interleaved (bit b-1 of
 *     every dimension first, dimension 0 first within a bit).  Points whose
 *     codes are all equal form a group; a group of several points whose box
 *     has some extent is quantised again inside its own box, giving a
 *     further code word (single-point groups get 0), at most 6 words in all.
 *     Points are ordered by their code words, then by input row.  A node is
 *     a range of that order: it splits at the highest bit where the codes of
 *     its first and last point differ (the next cell bisection that separates
 *     its points), or, when all its codes are equal, at the highest bit where
 *     its first and last positions differ.  Each such split halves the node's
 *     cell along one dimension: the cell's spatial median.
 *  T2 (boxes) A node's box is the tight box of its points; for d >= 4 each
 *     bound is then rounded outward to binary32 (the box still holds every
 *     point).
 *  W1 (separation, Sec. 2.3) Nodes A and B are well separated when two balls
 *     of the common radius r = max(rA, rB), centred at the box midpoints,
 *     with rX half the box diagonal, are at least s r apart:
 *         dist(cA, cB) - 2 r >= s r,  evaluated as  dc2 >= (s + 2)^2 * r2,
 *     with dc2 = sum_k (cA_k - cB_k)^2, c_k = 0.5 * (lo_k + hi_k),
 *     r2 = 0.25 * max(diag2(A), diag2(B)), diag2 = sum_k (hi_k - lo_k)^2,
 *     and (s + 2)^2 formed as (s + 2) * (s + 2).
 *  W2 (FindPair, Alg. 1) The decomposition starts from the two children of
 *     every internal node.  A pair that is not well separated is replaced by
 *     the two pairs (child, other) of the node with the larger diag2 (ties:
 *     the node with more points, then A; a one-point node is never split).
 *  R  (representatives) The paper draws the pair of representative points
 *     at random; here the representative of a node is its first point in the
 *     tree order, so the result is deterministic.
 *  E  (base-graph edges of a pair, the four cases of the Appendix) with
 *     c(X) = |X| >= minPts:
 *         neither A nor B large: every point of A with every point of B;
 *         A large, B not:        rep(A) with every point of B;
 *         B large, A not:        every point of A with rep(B);
 *         both large:            rep(A) with rep(B).
 *     The edge weight is max{cd(u), cd(v), d(u, v) / (1 + rho)}, computed as
 *         w2 = max(cd2(u), cd2(v), d2(u, v) / q),  q = (1 + rho) * (1 + rho).
 *  M  (MST) As in the paper's implementation, each pair contributes the
 *     K-lightest of its edges, K = (w2, d2, min id, max id); the output is
 *     Kruskal's MST of these candidates under K (one candidate per pair
 *     joins the two nodes, so the candidates span every point).
 *
 * Outputs: cd2[n]; the n-1 tree edges (min id, max id) sorted by K with w2
 * and d2; stats[0] = well-separated pairs, stats[1] = point pairs whose
 * weight was evaluated, stats[2] = pairs examined by the decomposition.
 */
#define AO_MAXW 6

typedef struct {
    int64_t first, count; /* range of tree positions */
    int64_t left, right;  /* child node indices, -1 for a leaf */
    double lo[7], hi[7];
} ao_node_t;

typedef struct {
    const double *P;
    int32_t d, L;
    int64_t n;
    uint64_t *w; /* code words, word-major: w[l * n + row] */
} ao_sort_ctx_t;

static ao_sort_ctx_t g_ao; /* qsort comparator context (one call at a time) */

static int ao_bits(int32_t d) { return (63 / d) > 31 ? 31 : (63 / d); }

static uint64_t ao_code(const double *x, const double *lo, const double *hi, int32_t d)
{
    int b = ao_bits(d);
    double top = (double)((1ull << b) - 1);
    uint64_t q[7];
    for (int32_t k = 0; k < d; ++k) {
        double r = hi[k] - lo[k];
        double t = r > 0.0 ? (x[k] - lo[k]) / r : 0.0;
        double f = floor(t * top);
        f = f < 0.0 ? 0.0 : (f > top ? top : f);
        q[k] = (uint64_t)f;
    }
    uint64_t c = 0;
    for (int bit = b - 1; bit >= 0; --bit)
        for (int32_t k = 0; k < d; ++k) c = (c << 1) | ((q[k] >> bit) & 1ull);
    return c;
}

static int ao_row_cmp(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    for (int32_t l = 0; l < g_ao.L; ++l) {
        uint64_t x = g_ao.w[(int64_t)l * g_ao.n + a], y = g_ao.w[(int64_t)l * g_ao.n + b];
        if (x != y) return x < y ? -1 : 1;
    }
    return (a > b) - (a < b);
}

static int ao_clz64(uint64_t x) { return x ? __builtin_clzll(x) : 64; }
static int ao_clz32(uint32_t x) { return x ? __builtin_clz(x) : 32; }

/* common-prefix length of the codes at tree positions i and j (positions
 * tell equal codes apart) */
static int ao_plen(const uint64_t *w, int64_t n, int32_t L, const int64_t *row, int64_t i, int64_t j)
{
    for (int32_t l = 0; l < L; ++l) {
        uint64_t a = w[(int64_t)l * n + row[i]], b = w[(int64_t)l * n + row[j]];
        if (a != b) return 64 * l + ao_clz64(a ^ b);
    }
    return 64 * L + ao_clz32((uint32_t)(i ^ j));
}

static float ao_down(double x)
{
    float f = (float)x;
    return ((double)f > x) ? nextafterf(f, -INFINITY) : f;
}
static float ao_up(double x)
{
    float f = (float)x;
    return ((double)f < x) ? nextafterf(f, INFINITY) : f;
}

/* T1 + T2: the tree order row[0..n) and the nodes (node 0 is the root). */
static int ao_tree(const double *P, int64_t n, int32_t d, int64_t *row, ao_node_t **nodes_out)
{
    uint64_t *w = (uint64_t *)calloc((size_t)AO_MAXW * (size_t)n, 8);
    int64_t *gs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    double *gb = (double *)malloc(sizeof(double) * 14 * (size_t)n);
    ao_node_t *nd = (ao_node_t *)malloc(sizeof(ao_node_t) * (size_t)(2 * n));
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n + 2));
    if (!w || !gs || !gb || !nd || !stk) {
        free(w); free(gs); free(gb); free(nd); free(stk);
        return OR_ENOMEM;
    }
    double lo[7], hi[7];
    for (int32_t k = 0; k < d; ++k) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < d; ++k) {
            double x = P[i * d + k];
            lo[k] = x < lo[k] ? x : lo[k];
            hi[k] = x > hi[k] ? x : hi[k];
        }
    for (int64_t i = 0; i < n; ++i) {
        w[i] = ao_code(P + i * d, lo, hi, d);
        row[i] = i;
    }
    int32_t L = 1;
    g_ao.P = P;
    g_ao.d = d;
    g_ao.n = n;
    g_ao.w = w;
    g_ao.L = L;
    qsort(row, (size_t)n, sizeof(int64_t), ao_row_cmp);
    while (L < AO_MAXW && n > 1) {
        /* groups of equal code words */
        int64_t ng = 0;
        int dup = 0;
        for (int64_t i = 0; i < n; ++i) {
            int same = i > 0;
            for (int32_t l = 0; l < L && same; ++l)
                if (w[(int64_t)l * n + row[i]] != w[(int64_t)l * n + row[i - 1]]) same = 0;
            if (!same) gs[ng++] = i;
            else dup = 1;
        }
        gs[ng] = n;
        if (!dup) break;
        int refinable = 0;
        for (int64_t g = 0; g < ng; ++g) {
            double *b = gb + 14 * g;
            for (int32_t k = 0; k < d; ++k) {
                b[k] = INFINITY;
                b[7 + k] = -INFINITY;
            }
            if (gs[g + 1] - gs[g] < 2) continue;
            for (int64_t i = gs[g]; i < gs[g + 1]; ++i)
                for (int32_t k = 0; k < d; ++k) {
                    double x = P[row[i] * d + k];
                    b[k] = x < b[k] ? x : b[k];
                    b[7 + k] = x > b[7 + k] ? x : b[7 + k];
                }
            for (int32_t k = 0; k < d; ++k)
                if (b[7 + k] > b[k]) refinable = 1;
        }
        if (!refinable) break;
        for (int64_t g = 0; g < ng; ++g)
            for (int64_t i = gs[g]; i < gs[g + 1]; ++i)
                w[(int64_t)L * n + row[i]] =
                    (gs[g + 1] - gs[g] > 1) ? ao_code(P + row[i] * d, gb + 14 * g, gb + 14 * g + 7, d) : 0;
        ++L;
        g_ao.L = L;
        qsort(row, (size_t)n, sizeof(int64_t), ao_row_cmp);
    }
    /* radix tree over positions, top-down */
    int64_t nn = 0, sp = 0;
    nd[nn].first = 0;
    nd[nn].count = n;
    stk[sp++] = nn++;
    while (sp) {
        int64_t x = stk[--sp];
        int64_t f = nd[x].first, c = nd[x].count;
        for (int32_t k = 0; k < d; ++k) {
            double a = INFINITY, b = -INFINITY;
            for (int64_t i = f; i < f + c; ++i) {
                double v = P[row[i] * d + k];
                a = v < a ? v : a;
                b = v > b ? v : b;
            }
            if (d >= 4) {
                a = (double)ao_down(a);
                b = (double)ao_up(b);
            }
            nd[x].lo[k] = a;
            nd[x].hi[k] = b;
        }
        nd[x].left = nd[x].right = -1;
        if (c == 1) continue;
        int64_t l = f + c - 1;
        int dl = ao_plen(w, n, L, row, f, l);
        /* last position whose prefix with f is longer than dl */
        int64_t a = f, b = l - 1;
        while (a < b) {
            int64_t m = a + (b - a + 1) / 2;
            if (ao_plen(w, n, L, row, f, m) > dl) a = m;
            else b = m - 1;
        }
        int64_t g = a;
        nd[nn].first = f;
        nd[nn].count = g - f + 1;
        nd[x].left = nn;
        stk[sp++] = nn++;
        nd[nn].first = g + 1;
        nd[nn].count = l - g;
        nd[x].right = nn;
        stk[sp++] = nn++;
    }
    free(w); free(gs); free(gb); free(stk);
    *nodes_out = nd;
    return OR_OK;
}

static double ao_diag2(const ao_node_t *A, int32_t d)
{
    double s = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = A->hi[k] - A->lo[k];
        s = s + t * t;
    }
    return s;
}

/* W1 */
static int ao_separated(const ao_node_t *A, const ao_node_t *B, int32_t d, double K, double dA, double dB)
{
    double dc2 = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = 0.5 * (A->lo[k] + A->hi[k]) - 0.5 * (B->lo[k] + B->hi[k]);
        dc2 = dc2 + t * t;
    }
    double r2 = 0.25 * (dA > dB ? dA : dB);
    return dc2 >= K * r2;
}

typedef struct {
    key_t_ k;
} ao_cand_t;

static int ao_cand_cmp(const void *pa, const void *pb)
{
    const key_t_ *a = (const key_t_ *)pa, *b = (const key_t_ *)pb;
    if (key_less(*a, *b)) return -1;
    if (key_less(*b, *a)) return 1;
    return 0;
}

static key_t_ ao_key(const double *P, int32_t d, const double *cd2, double q, int64_t u, int64_t v)
{
    key_t_ k;
    double e2 = d2_of(P, d, u, v);
    double c = cd2[u] > cd2[v] ? cd2[u] : cd2[v];
    double a = e2 / q;
    k.w2 = c > a ? c : a;
    k.e2 = e2;
    k.lo = u < v ? u : v;
    k.hi = u < v ? v : u;
    return k;
}

/* Walk the decomposition.  With pairs_out, every well-separated pair is
 * written as (first A, count A, first B, count B) in tree positions (up to
 * cap of them); with cand, each pair's candidate edge (E) is stored. */
static int ao_walk(const double *P, int64_t n, int32_t d, const int64_t *row, const ao_node_t *nd, double rho,
                   int32_t min_pts, const double *cd2, key_t_ **cand_out, int64_t *pairs_out, int64_t cap,
                   int64_t *stats)
{
    double s = sqrt(8.0 / rho);
    double K = (s + 2.0) * (s + 2.0);
    double q = (1.0 + rho) * (1.0 + rho);
    int64_t ccap = 1024, m = 0, evals = 0, visits = 0;
    key_t_ *cand = cand_out ? (key_t_ *)malloc(sizeof(key_t_) * (size_t)ccap) : NULL;
    int64_t scap = 1024, sp = 0;
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)scap);
    if ((cand_out && !cand) || !stk) {
        free(cand);
        free(stk);
        return OR_ENOMEM;
    }
    /* W2: the children of every internal node */
    for (int64_t x = 0; x < 2 * n - 1; ++x) {
        if (nd[x].left < 0) continue;
        if (sp == scap) {
            scap *= 2;
            int64_t *t = (int64_t *)realloc(stk, sizeof(int64_t) * 2 * (size_t)scap);
            if (!t) { free(cand); free(stk); return OR_ENOMEM; }
            stk = t;
        }
        stk[2 * sp] = nd[x].left;
        stk[2 * sp + 1] = nd[x].right;
        ++sp;
    }
    while (sp) {
        --sp;
        const ao_node_t *A = nd + stk[2 * sp], *B = nd + stk[2 * sp + 1];
        int64_t ia = stk[2 * sp], ib = stk[2 * sp + 1];
        ++visits;
        double dA = ao_diag2(A, d), dB = ao_diag2(B, d);
        if (ao_separated(A, B, d, K, dA, dB)) {
            if (pairs_out && m < cap) {
                pairs_out[4 * m] = A->first;
                pairs_out[4 * m + 1] = A->count;
                pairs_out[4 * m + 2] = B->first;
                pairs_out[4 * m + 3] = B->count;
            }
            if (cand_out) {
                /* E: the case's edge set, and its K-lightest edge */
                int bigA = A->count >= min_pts, bigB = B->count >= min_pts;
                int64_t a0 = A->first, a1 = bigA ? A->first + 1 : A->first + A->count;
                int64_t b0 = B->first, b1 = bigB ? B->first + 1 : B->first + B->count;
                key_t_ best = ao_key(P, d, cd2, q, row[a0], row[b0]);
                for (int64_t i = a0; i < a1; ++i)
                    for (int64_t j = b0; j < b1; ++j) {
                        key_t_ k = ao_key(P, d, cd2, q, row[i], row[j]);
                        if (key_less(k, best)) best = k;
                    }
                evals += (a1 - a0) * (b1 - b0);
                if (m == ccap) {
                    ccap *= 2;
                    key_t_ *t = (key_t_ *)realloc(cand, sizeof(key_t_) * (size_t)ccap);
                    if (!t) { free(cand); free(stk); return OR_ENOMEM; }
                    cand = t;
                }
                cand[m] = best;
            }
            ++m;
            continue;
        }
        int split_a = (B->count == 1) || (A->count > 1 && (dA > dB || (dA == dB && A->count >= B->count)));
        const ao_node_t *X = split_a ? A : B;
        int64_t oth = split_a ? ib : ia;
        if (sp + 2 > scap) {
            scap *= 2;
            int64_t *t = (int64_t *)realloc(stk, sizeof(int64_t) * 2 * (size_t)scap);
            if (!t) { free(cand); free(stk); return OR_ENOMEM; }
            stk = t;
        }
        stk[2 * sp] = X->left;
        stk[2 * sp + 1] = oth;
        ++sp;
        stk[2 * sp] = X->right;
        stk[2 * sp + 1] = oth;
        ++sp;
    }
    free(stk);
    if (stats) {
        stats[0] = m;
        stats[1] = evals;
        stats[2] = visits;
    }
    if (cand_out) *cand_out = cand;
    return OR_OK;
}

static int ao_check(const double *P, int64_t n, int32_t d, double rho)
{
    if (check_points(P, n, d)) return OR_EINVAL;
    if (d > 7 || !(rho > 0.0) || !isfinite(rho)) return OR_EINVAL;
    return OR_OK;
}

int oracle_optics_approx(const double *P, int64_t n, int32_t d, int32_t min_pts, double rho, double *cd2,
                         int64_t *edges, double *w2, double *e2, int64_t *stats)
{
    if (ao_check(P, n, d, rho) || min_pts < 1 || min_pts > n || !cd2) return OR_EINVAL;
    int rc = oracle_core_dist2(P, n, d, min_pts, NULL, n, cd2);
    if (rc) return rc;
    if (stats) stats[0] = stats[1] = stats[2] = 0;
    if (n == 1) return OR_OK;
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!row || !par) {
        free(row);
        free(par);
        return OR_ENOMEM;
    }
    ao_node_t *nd = NULL;
    rc = ao_tree(P, n, d, row, &nd);
    key_t_ *cand = NULL;
    int64_t st[3] = {0, 0, 0};
    if (!rc) rc = ao_walk(P, n, d, row, nd, rho, min_pts, cd2, &cand, NULL, 0, st);
    free(nd);
    free(row);
    if (rc) {
        free(par);
        return rc;
    }
    /* M: Kruskal on the candidates in K order */
    qsort(cand, (size_t)st[0], sizeof(key_t_), ao_cand_cmp);
    for (int64_t i = 0; i < n; ++i) par[i] = i;
    int64_t t = 0;
    for (int64_t i = 0; i < st[0] && t < n - 1; ++i) {
        int64_t a = uf_find(par, cand[i].lo), b = uf_find(par, cand[i].hi);
        if (a == b) continue;
        par[a] = b;
        edges[2 * t] = cand[i].lo;
        edges[2 * t + 1] = cand[i].hi;
        w2[t] = cand[i].w2;
        if (e2) e2[t] = cand[i].e2;
        ++t;
    }
    free(cand);
    free(par);
    if (stats) {
        stats[0] = st[0];
        stats[1] = st[1];
        stats[2] = st[2];
    }
    return t == n - 1 ? OR_OK : OR_EINVAL;
}

/* The decomposition alone (W1, W2 on the tree of T1, T2): the tree order
 * (row_of_pos[i] = input row at tree position i) and up to cap pairs as
 * (first A, count A, first B, count B); returns the number of pairs in
 * *npairs. */
int oracle_optics_wspd(const double *P, int64_t n, int32_t d, double rho, int64_t *row_of_pos, int64_t *pairs,
                       int64_t cap, int64_t *npairs)
{
    if (ao_check(P, n, d, rho) || !row_of_pos || !npairs) return OR_EINVAL;
    *npairs = 0;
    if (n == 1) {
        row_of_pos[0] = 0;
        return OR_OK;
    }
    ao_node_t *nd = NULL;
    int rc = ao_tree(P, n, d, row_of_pos, &nd);
    int64_t st[3] = {0, 0, 0};
    if (!rc) rc = ao_walk(P, n, d, row_of_pos, nd, rho, 1, NULL, NULL, pairs, cap, st);
    free(nd);
    *npairs = st[0];
    return rc;
}
