// geomst C ABI and host orchestration (one solve = tree build, optional core
// distances, filtered-Kruskal rounds, output).  Every step of the solve runs
// in the kernels of this library; the host only sizes launches, reads
// counters back and decides when the rounds end.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>
#include <algorithm>

#include "../../include/geomst.h"
#include "internal.h"
#include "common.h"
#include "tree_kernels.h"
#include "round_kernels.h"

namespace geomst {
namespace {

thread_local std::string g_err;
thread_local geomst_stats_t g_stats;
double g_beta_growth = 2.0;

struct Fail {
    int code;
};

#define HIPCHK(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            g_err = std::string(#x) + ": " + hipGetErrorString(e_);                           \
            throw Fail{e_ == hipErrorOutOfMemory ? GEOMST_ENOMEM : GEOMST_EDEVICE};           \
        }                                                                                     \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

inline unsigned blocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Grow-only device buffer.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need, size_t keep = 0, hipStream_t s = 0) {
        if (need <= bytes) return;
        size_t nb = std::max(need, bytes + bytes / 2);
        nb = (nb + 255) & ~(size_t)255;
        void* q = nullptr;
        if (p) HIPCHK(hipDeviceSynchronize());  // queued kernels may still use p
        HIPCHK(hipMalloc(&q, nb));
        if (keep && p) {
            HIPCHK(hipMemcpyAsync(q, p, std::min(keep, bytes), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        if (p) HIPCHK(hipFree(p));
        p = q;
        bytes = nb;
    }
    template <class T>
    T* as() const {
        return (T*)p;
    }
};

struct EdgeBufs {
    DBuf w2, e2, ids, pos;
    size_t cap = 0;
    void ensure(size_t need, size_t keep, hipStream_t s) {
        if (need <= cap) return;
        size_t nc = std::max(need, cap + cap / 2);
        w2.ensure(nc * 8, keep * 8, s);
        e2.ensure(nc * 8, keep * 8, s);
        ids.ensure(nc * 8, keep * 8, s);
        pos.ensure(nc * 8, keep * 8, s);
        cap = nc;
    }
    EdgeList list() const { return EdgeList{w2.as<double>(), e2.as<double>(), ids.as<u64>(), pos.as<u64>()}; }
};

struct Device {
    std::mutex mu;
    bool init = false;
    hipStream_t own = nullptr;
    Counters* hcnt = nullptr;  // pinned mirror
    DBuf cnt;
    // input staging (host API)
    DBuf pin, eout, wout, cdout;
    // tree
    DBuf part, bbox, key, val, key2, val2, stemp, X, orig, cd2, box, rad, rng, kids, npar, cdb, flags, comp;
    // union-find / component refresh
    DBuf uf, best, bnd, incl;
    // rounds
    DBuf F[2], Q[2], big, ntask, toff, parts;
    size_t capF[2] = {0, 0}, capQ[2] = {0, 0}, capBig = 0;
    EdgeBufs C, P[2], OUT;
    // Kruskal
    DBuf kid, ke2, kw2, perm[2], alive[2], ru, rv, nalive;
    struct Prof* prof = nullptr;
};

Device g_dev[16];
bool g_kernel_timing = false;

// Optional device timing of kernel families: event pairs recorded on the
// solve's stream around each launch group, resolved after the final sync.
struct Prof {
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, size_t>> pend;  // (family, first event index)
    size_t used = 0;
    bool on = false;
    void begin(bool enable) {
        on = enable;
        used = 0;
        pend.clear();
    }
    size_t rec(hipStream_t s) {
        if (used == pool.size()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            pool.push_back(e);
        }
        HIPCHK(hipEventRecord(pool[used], s));
        return used++;
    }
    void finish(geomst_stats_t& st) {
        for (auto& p : pend) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pool[p.second], pool[p.second + 1]));
            st.kernel_ms[p.first] += ms;
            st.kernel_launches[p.first] += 1;
        }
        pend.clear();
        used = 0;
    }
};
Prof g_prof[16];

struct TimedScope {
    Prof& P;
    hipStream_t s;
    int fam;
    size_t a = 0;
    TimedScope(Prof& p, hipStream_t st, int f) : P(p), s(st), fam(f) {
        if (P.on) a = P.rec(s);
    }
    ~TimedScope() {
        // never throws: a failed record only loses this sample
        if (P.on && P.used < P.pool.size() + 1) {
            if (P.used == P.pool.size()) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                P.pool.push_back(e);
            }
            if (hipEventRecord(P.pool[P.used], s) != hipSuccess) return;
            ++P.used;
            P.pend.push_back({fam, a});
        }
    }
};
#define TIMED(fam) TimedScope timed_scope_(*D.prof, s, fam)

void counters_reset_round(Device& D, hipStream_t s) {
    // zero the per-round counters and set the minima to "none" (all ones)
    HIPCHK(hipMemsetAsync(D.cnt.p, 0, sizeof(u32) * C_OUT, s));
    HIPCHK(hipMemsetAsync((char*)D.cnt.p + offsetof(Counters, m), 0xff, sizeof(u64) * 4, s));
}

void read_counters(Device& D, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(D.hcnt, D.cnt.p, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

void write_counters(Device& D, const Counters& c, hipStream_t s) {
    *D.hcnt = c;
    HIPCHK(hipMemcpyAsync(D.cnt.p, D.hcnt, sizeof(Counters), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

double bits_to_double(u64 b) {
    double x;
    memcpy(&x, &b, 8);
    return x;
}

const double kInf = __builtin_inf();

int id_bits(int n) {
    u32 m = (u32)(n - 1);
    int b = 0;
    while (m) {
        ++b;
        m >>= 1;
    }
    return b < 1 ? 1 : b;
}

// Sort m edges of L by K; returns the permutation (sorted rank -> edge).
u32* sort_edges(Device& D, const EdgeList& L, u32 m, int n, bool hdb, hipStream_t s) {
    D.kid.ensure((size_t)m * 8);
    D.kw2.ensure((size_t)m * 8);
    if (hdb) D.ke2.ensure((size_t)m * 8);
    D.perm[0].ensure((size_t)m * 4);
    D.perm[1].ensure((size_t)m * 4);
    D.stemp.ensure(radix_temp_bytes(m));
    int B = id_bits(n);
    TIMED(GEOMST_K_SORT);
    g_stats.sort_elems += (int64_t)m * ((2 * B + 7) / 8 + (hdb ? 8 : 0) + 8);
    k_sortkeys<<<blocks(m, 256), 256, 0, s>>>(L, m, B, D.kid.as<u64>(), hdb ? D.ke2.as<u64>() : nullptr,
                                              D.kw2.as<u64>(), D.perm[0].as<u32>());
    LAUNCHCHK();
    u32* a = D.perm[0].as<u32>();
    u32* b = D.perm[1].as<u32>();
    auto pass = [&](const u64* w, int bits) {
        if (radix_sort_index(w, a, b, m, bits, D.stemp.p, s)) std::swap(a, b);
        LAUNCHCHK();
    };
    pass(D.kid.as<u64>(), 2 * B);
    if (hdb) pass(D.ke2.as<u64>(), 64);
    pass(D.kw2.as<u64>(), 64);
    return a;
}

template <int D_>
struct Solver {
    Device& D;
    hipStream_t s;
    int n;
    int minpts;  // 0 = EMST
    bool hdb;
    TreeView t;
    geomst_stats_t& st;

    Solver(Device& dev, hipStream_t stream, int n_, int mp, geomst_stats_t& stats)
        : D(dev), s(stream), n(n_), minpts(mp), hdb(mp > 0), st(stats) {}

    void build_tree(const double* P) {
        int nn = 2 * n - 1;
        unsigned nbb = std::min(blocks(n, 256), 512u);
        D.part.ensure((size_t)nbb * 2 * D_ * 8);
        D.bbox.ensure(2 * D_ * 8);
        TIMED(GEOMST_K_TREE);
        k_check_input<<<std::min(blocks((size_t)n * D_, 256), 1024u), 256, 0, s>>>(P, (size_t)n * D_,
                                                                                   D.cnt.as<Counters>());
        LAUNCHCHK();
        k_bbox_partial<D_><<<nbb, 256, 0, s>>>(P, n, D.part.as<double>());
        LAUNCHCHK();
        k_bbox_final<D_><<<1, 64, 0, s>>>(D.part.as<double>(), (int)nbb, D.bbox.as<double>());
        LAUNCHCHK();
        D.key.ensure((size_t)n * 8);
        D.key2.ensure((size_t)n * 8);
        D.val.ensure((size_t)n * 4);
        D.val2.ensure((size_t)n * 4);
        D.stemp.ensure(radix_temp_bytes(n));
        k_morton<D_><<<blocks(n, 256), 256, 0, s>>>(P, n, D.bbox.as<double>(), D.key.as<u64>(), D.val.as<u32>());
        LAUNCHCHK();
        int mb = (63 / D_) > 31 ? 31 : (63 / D_);
        g_stats.sort_elems += (int64_t)n * ((mb * D_ + 7) / 8);
        int flip = radix_sort_pairs(D.key.as<u64>(), D.val.as<u32>(), D.key2.as<u64>(), D.val2.as<u32>(), n,
                                    mb * D_, D.stemp.p, s);
        LAUNCHCHK();
        const u64* skey = flip ? D.key2.as<u64>() : D.key.as<u64>();
        const u32* sval = flip ? D.val2.as<u32>() : D.val.as<u32>();
        D.X.ensure((size_t)n * D_ * 8);
        D.orig.ensure((size_t)n * 4);
        k_permute<D_><<<blocks(n, 256), 256, 0, s>>>(P, n, sval, D.X.as<double>(), D.orig.as<u32>());
        LAUNCHCHK();
        D.box.ensure((size_t)nn * 2 * D_ * 8);
        D.rad.ensure((size_t)nn * 8);
        D.rng.ensure((size_t)nn * 8);
        D.kids.ensure((size_t)std::max(n - 1, 1) * 8);
        D.npar.ensure((size_t)nn * 4);
        D.flags.ensure((size_t)nn * 4);
        D.comp.ensure((size_t)nn * 4);
        D.cdb.ensure((size_t)nn * 16);
        if (n >= 2) {
            k_karras<<<blocks(n - 1, 256), 256, 0, s>>>(skey, n, D.rng.as<int2>(), D.kids.as<int2>(),
                                                         D.npar.as<int>());
            LAUNCHCHK();
        } else {
            HIPCHK(hipMemsetAsync(D.npar.p, 0xff, 4, s));
        }
        HIPCHK(hipMemsetAsync(D.flags.p, 0, (size_t)nn * 4, s));
        k_bounds<D_><<<blocks(n, 256), 256, 0, s>>>(n, D.X.as<double>(), nullptr, D.kids.as<int2>(),
                                                    D.npar.as<int>(), D.box.as<double>(), D.rad.as<double>(),
                                                    D.cdb.as<double2>(), D.rng.as<int2>(), D.flags.as<u32>(), 1,
                                                    0);
        LAUNCHCHK();
        t.n = n;
        t.X = D.X.as<double>();
        t.orig = D.orig.as<u32>();
        t.cd2 = nullptr;
        t.box = D.box.as<double>();
        t.rad = D.rad.as<double>();
        t.rng = D.rng.as<int2>();
        t.kids = D.kids.as<int2>();
        t.cdb = D.cdb.as<double2>();
        t.comp = D.comp.as<int>();
    }

    template <int KMAX>
    void knn_k() {
        k_knn<D_, KMAX><<<blocks(n, 64), 64, 0, s>>>(t, minpts, D.cd2.as<double>(), &D.cnt.as<Counters>()->c[C_ERR]);
        LAUNCHCHK();
    }

    void core_distances() {
        D.cd2.ensure((size_t)n * 8);
        TIMED(GEOMST_K_CORE);
        if (minpts <= 8) knn_k<8>();
        else if (minpts <= 16) knn_k<16>();
        else if (minpts <= 32) knn_k<32>();
        else knn_k<64>();
        t.cd2 = D.cd2.as<double>();
        HIPCHK(hipMemsetAsync(D.flags.p, 0, (size_t)(2 * n - 1) * 4, s));
        k_bounds<D_><<<blocks(n, 256), 256, 0, s>>>(n, D.X.as<double>(), D.cd2.as<double>(), D.kids.as<int2>(),
                                                    D.npar.as<int>(), D.box.as<double>(), D.rad.as<double>(),
                                                    D.cdb.as<double2>(), D.rng.as<int2>(), D.flags.as<u32>(), 0,
                                                    1);
        LAUNCHCHK();
    }

    void refresh_components() {
        TIMED(GEOMST_K_REFRESH);
        k_uf_compress<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n, D.cnt.as<Counters>());
        LAUNCHCHK();
        k_boundaries<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n, D.bnd.as<u32>());
        LAUNCHCHK();
        scan_inclusive_u32(D.bnd.as<u32>(), D.incl.as<u32>(), n, D.stemp.p, s);
        LAUNCHCHK();
        k_node_comp<<<blocks(2 * n - 1, 256), 256, 0, s>>>(D.rng.as<int2>(), D.uf.as<u32>(), D.incl.as<u32>(),
                                                           2 * n - 1, D.comp.as<int>());
        LAUNCHCHK();
    }

    RoundArgs args(double beta2, int fo, int qo, int po) {
        RoundArgs r;
        r.cnt = D.cnt.as<Counters>();
        r.beta2 = beta2;
        r.uf = D.uf.as<u32>();
        r.fout = D.F[fo].as<PairRec>();
        r.cap_f = (u32)D.capF[fo];
        r.q = D.Q[qo].as<PairRec>();
        r.cap_q = (u32)D.capQ[qo];
        r.big = D.big.as<uint2>();
        r.cap_big = (u32)D.capBig;
        r.c = D.C.list();
        r.cap_c = (u32)D.C.cap;
        r.pout = D.P[po].list();
        r.cap_p = (u32)D.P[po].cap;
        return r;
    }

    // Grow whatever overflowed (keeping the entries that existed before the
    // step) and restore the counters so the step can run again.
    bool fix_overflow(const Counters& before, int fo, int qo, int po) {
        const Counters& c = *D.hcnt;
        if (!(c.c[C_ERR] & 1u)) return false;
        auto grow_pairs = [&](DBuf& b, size_t& cap, u32 need, u32 keep) {
            if (need > cap) {
                size_t nc = std::max<size_t>((size_t)need + need / 2, cap * 2);
                b.ensure(nc * sizeof(PairRec), (size_t)keep * sizeof(PairRec), s);
                cap = nc;
            }
        };
        grow_pairs(D.F[fo], D.capF[fo], c.c[C_F], before.c[C_F]);
        grow_pairs(D.Q[qo], D.capQ[qo], std::max(c.c[C_Q], c.c[C_QN]), 0);
        if (c.c[C_BIG] > D.capBig) {
            size_t nc = std::max<size_t>((size_t)c.c[C_BIG] * 3 / 2, D.capBig * 2);
            D.big.ensure(nc * 8, (size_t)before.c[C_BIG] * 8, s);
            D.capBig = nc;
        }
        if (c.c[C_C] > D.C.cap) D.C.ensure((size_t)c.c[C_C] * 3 / 2, before.c[C_C], s);
        if (c.c[C_P] > D.P[po].cap) D.P[po].ensure((size_t)c.c[C_P] * 3 / 2, before.c[C_P], s);
        write_counters(D, before, s);
        return true;
    }

    void run(const double* P, long long* edges, double* w, double* w2, double* cd, double* cd2out) {
        using clk = std::chrono::steady_clock;
        auto t0 = clk::now();
        HIPCHK(hipMemsetAsync(D.cnt.p, 0, sizeof(Counters), s));
        HIPCHK(hipMemsetAsync((char*)D.cnt.p + offsetof(Counters, m), 0xff, sizeof(u64) * 4, s));
        build_tree(P);
        read_counters(D, s);
        if (D.hcnt->c[C_ERR] & 2u) {
            g_err = "a coordinate is not finite or exceeds 2^500 in magnitude";
            throw Fail{GEOMST_EDOM};
        }
        auto t1 = clk::now();
        if (hdb) {
            core_distances();
            HIPCHK(hipStreamSynchronize(s));
        }
        auto t2 = clk::now();

        // union-find and node components
        D.uf.ensure((size_t)n * 4);
        D.best.ensure((size_t)n * 4);
        D.bnd.ensure((size_t)n * 4);
        D.incl.ensure((size_t)n * 4);
        D.stemp.ensure(std::max(radix_temp_bytes(n), scan_temp_bytes(n)));
        k_iota<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n);
        LAUNCHCHK();
        HIPCHK(hipMemsetAsync(D.best.p, 0xff, (size_t)n * 4, s));
        refresh_components();

        // lists
        auto initcap = [&](size_t& cap, DBuf& b, size_t want) {
            if (cap < want) {
                b.ensure(want * sizeof(PairRec));
                cap = want;
            }
        };
        size_t nf0 = (size_t)(hdb ? 8 : 4) * n + 4096;
        initcap(D.capF[0], D.F[0], nf0);
        initcap(D.capF[1], D.F[1], nf0);
        initcap(D.capQ[0], D.Q[0], (size_t)2 * n + 4096);
        initcap(D.capQ[1], D.Q[1], (size_t)2 * n + 4096);
        if (D.capBig < (size_t)n / 8 + 4096) {
            D.capBig = (size_t)n / 8 + 4096;
            D.big.ensure(D.capBig * 8);
        }
        D.C.ensure((size_t)2 * n + 4096, 0, s);
        D.P[0].ensure((size_t)n + 4096, 0, s);
        D.P[1].ensure((size_t)n + 4096, 0, s);
        D.OUT.ensure((size_t)n + 64, 0, s);

        // initial frontier: the children of every internal node
        int fc = 0, pc = 0;
        k_init_frontier<D_><<<blocks(n - 1, 256), 256, 0, s>>>(t, hdb, D.F[fc].as<PairRec>());
        LAUNCHCHK();
        k_min_positive_lb<<<blocks(n - 1, 256), 256, 0, s>>>(D.F[fc].as<PairRec>(), (u32)(n - 1),
                                                            D.cnt.as<Counters>());
        LAUNCHCHK();
        read_counters(D, s);
        u64 b0 = D.hcnt->m[M_F];
        double beta2 = (b0 == ~0ull) ? 0.0 : bits_to_double(b0);
        u32 nF = (u32)(n - 1), nP = 0;
        const double g2 = g_beta_growth * g_beta_growth;
        u64 committed = 0, maxf = nF, big_pairs = 0;
        int rounds = 0;
        u32 nout = 0;
        while (true) {
            ++rounds;
            if (rounds > 100000) {
                g_err = "round limit exceeded";
                throw Fail{GEOMST_EINTERNAL};
            }
            counters_reset_round(D, s);
            int fo = fc ^ 1, po = pc ^ 1;
            // frontier and pool split
            Counters before;
            read_counters(D, s);
            before = *D.hcnt;
            while (true) {
                RoundArgs r = args(beta2, fo, 0, po);
                {
                TIMED(GEOMST_K_SPLIT);
                if (nF) {
                    k_split_frontier<<<blocks(nF, 256), 256, 0, s>>>(t, r, D.F[fc].as<PairRec>(), nF);
                    LAUNCHCHK();
                }
                if (nP) {
                    k_split_pool<<<blocks(nP, 256), 256, 0, s>>>(r, D.P[pc].list(), nP);
                    LAUNCHCHK();
                }
                }
                read_counters(D, s);
                if (!fix_overflow(before, fo, 0, po)) break;
            }
            // expansion levels
            u32 nq = D.hcnt->c[C_Q];
            int qc = 0;
            while (nq > 0) {
                Counters b4 = *D.hcnt;
                b4.c[C_QN] = 0;
                write_counters(D, b4, s);
                while (true) {
                    RoundArgs r = args(beta2, fo, qc ^ 1, po);
                    {
                        TIMED(GEOMST_K_EXPAND);
                        k_expand<D_><<<blocks(nq, 256), 256, 0, s>>>(t, r, hdb, D.Q[qc].as<PairRec>(), nq);
                        LAUNCHCHK();
                    }
                    read_counters(D, s);
                    if (!fix_overflow(b4, fo, qc ^ 1, po)) break;
                }
                nq = D.hcnt->c[C_QN];
                qc ^= 1;
            }
            // large pairs
            u32 nbig = D.hcnt->c[C_BIG];
            if (nbig) {
                big_pairs += nbig;
                D.ntask.ensure((size_t)nbig * 4);
                D.toff.ensure((size_t)nbig * 4);
                D.stemp.ensure(std::max(scan_temp_bytes(nbig), radix_temp_bytes(n)));
                k_big_ntasks<<<blocks(nbig, 256), 256, 0, s>>>(t, D.big.as<uint2>(), nbig, D.ntask.as<u32>());
                LAUNCHCHK();
                scan_exclusive_u32(D.ntask.as<u32>(), D.toff.as<u32>(), nbig, D.stemp.p, s);
                LAUNCHCHK();
                u32 last_off = 0, last_cnt = 0;
                HIPCHK(hipMemcpyAsync(&last_off, D.toff.as<u32>() + nbig - 1, 4, hipMemcpyDeviceToHost, s));
                HIPCHK(hipMemcpyAsync(&last_cnt, D.ntask.as<u32>() + nbig - 1, 4, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                u32 ntasks = last_off + last_cnt;
                D.parts.ensure((size_t)ntasks * sizeof(PartKey));
                {
                TIMED(GEOMST_K_BCCP);
                if (hdb)
                    k_big_bccp<D_, 1><<<ntasks, 64, 0, s>>>(t, D.big.as<uint2>(), nbig, D.toff.as<u32>(),
                                                           D.parts.as<PartKey>(), D.cnt.as<Counters>());
                else
                    k_big_bccp<D_, 0><<<ntasks, 64, 0, s>>>(t, D.big.as<uint2>(), nbig, D.toff.as<u32>(),
                                                           D.parts.as<PartKey>(), D.cnt.as<Counters>());
                LAUNCHCHK();
                }
                Counters b4;
                read_counters(D, s);
                b4 = *D.hcnt;
                while (true) {
                    RoundArgs r = args(beta2, fo, 0, po);
                    TIMED(GEOMST_K_BCCP);
                    k_big_combine<<<blocks(nbig, 256), 256, 0, s>>>(r, nbig, D.toff.as<u32>(), D.ntask.as<u32>(),
                                                                    D.parts.as<PartKey>());
                    LAUNCHCHK();
                    read_counters(D, s);
                    if (!fix_overflow(b4, fo, 0, po)) break;
                }
            }
            // Kruskal on the committed edges
            u32 m = D.hcnt->c[C_C];
            committed += m;
            if (m) {
                EdgeList L = D.C.list();
                u32* perm = sort_edges(D, L, m, n, hdb, s);
                D.alive[0].ensure((size_t)m * 4);
                D.alive[1].ensure((size_t)m * 4);
                D.ru.ensure((size_t)m * 4);
                D.rv.ensure((size_t)m * 4);
                D.nalive.ensure(8);
                k_iota<<<blocks(m, 256), 256, 0, s>>>(D.alive[0].as<u32>(), m);
                LAUNCHCHK();
                k_set_u32<<<1, 1, 0, s>>>(D.nalive.as<u32>(), m);
                LAUNCHCHK();
                int ac = 0;
                while (true) {
                    u32* na_in = D.nalive.as<u32>() + ac;
                    u32* na_out = D.nalive.as<u32>() + (ac ^ 1);
                    {
                    TIMED(GEOMST_K_KRUSKAL);
                    k_set_u32<<<1, 1, 0, s>>>(na_out, 0);
                    LAUNCHCHK();
                    k_bor_pick<<<blocks(m, 256), 256, 0, s>>>(D.alive[ac].as<u32>(), na_in, perm, L, D.uf.as<u32>(),
                                                              D.best.as<u32>(), D.ru.as<u32>(), D.rv.as<u32>(),
                                                              D.cnt.as<Counters>());
                    LAUNCHCHK();
                    k_bor_hook<<<blocks(m, 256), 256, 0, s>>>(D.alive[ac].as<u32>(), na_in, perm, L, D.uf.as<u32>(),
                                                              D.best.as<u32>(), D.ru.as<u32>(), D.rv.as<u32>(),
                                                              D.alive[ac ^ 1].as<u32>(), na_out, D.OUT.list(),
                                                              (u32)D.OUT.cap, D.cnt.as<Counters>());
                    LAUNCHCHK();
                    k_bor_reset<<<blocks(m, 256), 256, 0, s>>>(na_in, D.ru.as<u32>(), D.rv.as<u32>(),
                                                               D.best.as<u32>());
                    LAUNCHCHK();
                    }
                    u32 left = 0;
                    HIPCHK(hipMemcpyAsync(&left, na_out, 4, hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                    ac ^= 1;
                    if (left == 0) break;
                }
            }
            refresh_components();
            read_counters(D, s);
            const Counters& c = *D.hcnt;
            if (c.c[C_ERR] & (1u | 4u | 8u)) {
                g_err = (c.c[C_ERR] & 8u) ? "union-find walk did not terminate"
                        : (c.c[C_ERR] & 4u) ? "k-NN stack overflow" : "output edge overflow";
                throw Fail{GEOMST_EINTERNAL};
            }
            nout = c.c[C_OUT];
            nF = c.c[C_F];
            nP = c.c[C_P];
            maxf = std::max<u64>(maxf, nF);
            fc = fo;
            pc = po;
            if (nout >= (u32)(n - 1)) break;
            double mf = c.m[M_F] == ~0ull ? kInf : bits_to_double(c.m[M_F]);
            double mp = c.m[M_P] == ~0ull ? kInf : bits_to_double(c.m[M_P]);
            double nxt = std::min(mf, mp);
            if (nxt == kInf) {
                g_err = "no pairs left before the tree was complete";
                throw Fail{GEOMST_EINTERNAL};
            }
            beta2 = std::max(beta2 * g2, nxt);
        }
        if (nout != (u32)(n - 1)) {
            g_err = "wrong number of tree edges";
            throw Fail{GEOMST_EINTERNAL};
        }
        auto t3 = clk::now();
        // output: sort the tree edges by K and write them
        EdgeList O = D.OUT.list();
        u32* perm = sort_edges(D, O, n - 1, n, hdb, s);
        {
        TIMED(GEOMST_K_OUTPUT);
        k_write_edges<<<blocks(n - 1, 256), 256, 0, s>>>(O, perm, (u32)(n - 1), edges, w, w2);
        LAUNCHCHK();
        }
        if (hdb && (cd || cd2out)) {
            TIMED(GEOMST_K_OUTPUT);
            k_write_cd<<<blocks(n, 256), 256, 0, s>>>(D.cd2.as<double>(), D.orig.as<u32>(), n, cd, cd2out);
            LAUNCHCHK();
        }
        read_counters(D, s);
        auto t4 = clk::now();
        auto ms = [](clk::time_point a, clk::time_point b) {
            return std::chrono::duration<double, std::milli>(b - a).count();
        };
        st.rounds = rounds;
        st.pair_visits = (int64_t)D.hcnt->c64[C64_VISITS];
        st.bccp_evals = (int64_t)D.hcnt->c64[C64_EVALS];
        st.bccp_pairs = (int64_t)D.hcnt->c64[C64_BCCP] + (int64_t)big_pairs;
        st.big_pairs = (int64_t)big_pairs;
        st.committed_edges = (int64_t)committed;
        st.max_frontier = (int64_t)maxf;
        st.ms_tree = ms(t0, t1);
        st.ms_core = ms(t1, t2);
        st.ms_rounds = ms(t2, t3);
        st.ms_final = ms(t3, t4);
        st.big_evals = (int64_t)D.hcnt->c64[C64_BIGEVALS];
        D.prof->finish(st);
    }
};

Device& device_ctx(int* dev_out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16) {
        g_err = "device index out of range";
        throw Fail{GEOMST_EDEVICE};
    }
    *dev_out = dev;
    return g_dev[dev];
}

void ensure_init(Device& D) {
    if (D.init) return;
    HIPCHK(hipStreamCreateWithFlags(&D.own, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void**)&D.hcnt, sizeof(Counters), hipHostMallocDefault));
    D.cnt.ensure(sizeof(Counters));
    D.prof = &g_prof[&D - g_dev];
    D.init = true;
}

int validate(const void* pts, int64_t n, int32_t d, int32_t min_pts, const void* edges) {
    if (!pts) {
        g_err = "points is NULL";
        return GEOMST_EINVAL;
    }
    if (n < 1 || n > (1ll << 26)) {
        g_err = "n must be in [1, 2^26]";
        return GEOMST_EINVAL;
    }
    if (d < 1 || d > kMaxDim) {
        g_err = "d must be in [1, 7]";
        return GEOMST_EINVAL;
    }
    if (min_pts < 0 || min_pts > 64 || (min_pts > 0 && min_pts > n)) {
        g_err = "min_pts must be in [1, min(n, 64)]";
        return GEOMST_EINVAL;
    }
    if (n > 1 && !edges) {
        g_err = "edges is NULL";
        return GEOMST_EINVAL;
    }
    return GEOMST_OK;
}

// Solve with device pointers on stream s (device context locked by caller).
void solve_dev(Device& D, hipStream_t s, const double* P, int n, int d, int minpts, long long* edges, double* w,
               double* w2, double* cd, double* cd2) {
    memset(&g_stats, 0, sizeof(g_stats));
    g_stats.n = n;
    g_stats.d = d;
    g_stats.min_pts = minpts;
    D.prof->begin(g_kernel_timing);
    auto t0 = std::chrono::steady_clock::now();
    if (n == 1) {
        // one point: no edges; its core distance is 0 (minPts = 1)
        HIPCHK(hipMemsetAsync(D.cnt.p, 0, sizeof(Counters), s));
        k_check_input<<<1, 64, 0, s>>>(P, (size_t)d, D.cnt.as<Counters>());
        LAUNCHCHK();
        read_counters(D, s);
        if (D.hcnt->c[C_ERR] & 2u) {
            g_err = "a coordinate is not finite or exceeds 2^500 in magnitude";
            throw Fail{GEOMST_EDOM};
        }
        if (cd) HIPCHK(hipMemsetAsync(cd, 0, 8, s));
        if (cd2) HIPCHK(hipMemsetAsync(cd2, 0, 8, s));
        HIPCHK(hipStreamSynchronize(s));
        return;
    }
    switch (d) {
#define CASE(K)                                                   \
    case K: {                                                     \
        Solver<K> sv(D, s, n, minpts, g_stats);                   \
        sv.run(P, edges, w, w2, cd, cd2);                         \
        break;                                                    \
    }
        CASE(1)
        CASE(2)
        CASE(3)
        CASE(4)
        CASE(5)
        CASE(6)
        CASE(7)
#undef CASE
        default:
            g_err = "unsupported dimension";
            throw Fail{GEOMST_EINVAL};
    }
    HIPCHK(hipStreamSynchronize(s));
    g_stats.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int run_dev(const double* P, int64_t n, int32_t d, int32_t minpts, long long* edges, double* w, double* w2,
            double* cd, double* cd2, void* stream) {
    g_err.clear();
    int rc = validate(P, n, d, minpts, edges);
    if (rc) return rc;
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        solve_dev(D, (hipStream_t)stream, P, (int)n, d, minpts, edges, w, w2, cd, cd2);
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int run_host(const double* P, int64_t n, int32_t d, int32_t minpts, int64_t* edges, double* w, double* cd) {
    g_err.clear();
    int rc = validate(P, n, d, minpts, edges);
    if (rc) return rc;
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        hipStream_t s = D.own;
        size_t m = (size_t)(n > 1 ? n - 1 : 0);
        D.pin.ensure((size_t)n * d * 8);
        D.eout.ensure(m * 16 + 16);
        D.wout.ensure(m * 8 + 8);
        D.cdout.ensure((size_t)n * 8);
        HIPCHK(hipMemcpyAsync(D.pin.p, P, (size_t)n * d * 8, hipMemcpyHostToDevice, s));
        solve_dev(D, s, D.pin.as<double>(), (int)n, d, minpts, D.eout.as<long long>(), w ? D.wout.as<double>() : nullptr,
                  nullptr, (minpts > 0 && cd) ? D.cdout.as<double>() : nullptr, nullptr);
        if (m) HIPCHK(hipMemcpyAsync(edges, D.eout.p, m * 16, hipMemcpyDeviceToHost, s));
        if (m && w) HIPCHK(hipMemcpyAsync(w, D.wout.p, m * 8, hipMemcpyDeviceToHost, s));
        if (minpts > 0 && cd) HIPCHK(hipMemcpyAsync(cd, D.cdout.p, (size_t)n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

}  // namespace
}  // namespace geomst

using namespace geomst;

extern "C" {

int geomst_emst(const double* points, int64_t n, int32_t d, int64_t* edges, double* weights) {
    return run_host(points, n, d, 0, edges, weights, nullptr);
}

int geomst_hdbscan(const double* points, int64_t n, int32_t d, int32_t min_pts, double* core_dist, int64_t* edges,
                   double* weights) {
    if (min_pts < 1) {
        g_err = "min_pts must be >= 1";
        return GEOMST_EINVAL;
    }
    return run_host(points, n, d, min_pts, edges, weights, core_dist);
}

int geomst_emst_dev(const double* d_points, int64_t n, int32_t d, int64_t* d_edges, double* d_weights,
                    double* d_weights_sq, void* stream) {
    return run_dev(d_points, n, d, 0, (long long*)d_edges, d_weights, d_weights_sq, nullptr, nullptr, stream);
}

int geomst_hdbscan_dev(const double* d_points, int64_t n, int32_t d, int32_t min_pts, double* d_core_dist,
                       double* d_core_dist_sq, int64_t* d_edges, double* d_weights, double* d_weights_sq,
                       void* stream) {
    if (min_pts < 1) {
        g_err = "min_pts must be >= 1";
        return GEOMST_EINVAL;
    }
    return run_dev(d_points, n, d, min_pts, (long long*)d_edges, d_weights, d_weights_sq, d_core_dist,
                   d_core_dist_sq, stream);
}

int geomst_get_stats(geomst_stats_t* out) {
    if (!out) return GEOMST_EINVAL;
    *out = g_stats;
    return GEOMST_OK;
}

int geomst_set_option(const char* name, double value) {
    if (!name) return GEOMST_EINVAL;
    if (!strcmp(name, "beta_growth")) {
        if (!(value > 1.0) || !(value < 1e6)) return GEOMST_EINVAL;
        g_beta_growth = value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "kernel_timing")) {
        if (value != 0.0 && value != 1.0) return GEOMST_EINVAL;
        g_kernel_timing = value != 0.0;
        return GEOMST_OK;
    }
    return GEOMST_EINVAL;
}

const char* geomst_last_error(void) { return g_err.c_str(); }

int geomst_version(void) { return 100; }

}  // extern "C"
