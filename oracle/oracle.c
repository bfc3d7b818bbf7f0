/*
 * CPU checker for the Euclidean MST and the HDBSCAN* mutual-reachability MST.
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
