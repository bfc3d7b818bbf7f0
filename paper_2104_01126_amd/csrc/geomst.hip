// geomst C ABI and host orchestration (one solve = tree build, optional core
// distances, filtered-Kruskal rounds, output).  Every step of the solve runs
// in the kernels of this library; the host only sizes launches, reads
// counters back and decides when the rounds end.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <chrono>
#include <mutex>
#include <atomic>
#include <new>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <memory>
#include <algorithm>
#include <string>
#include <vector>
#include <algorithm>
#include <string>

#include "../../include/geomst.h"
#include "internal.h"
#include "common.h"
#include "tree_kernels.h"
#include "round_kernels.h"
#include "dendro_kernels.h"
#include "approx_kernels.h"

namespace geomst {
namespace {

thread_local std::string g_err;
thread_local hipStream_t g_cur_stream = nullptr;  // stream of the solve running on this thread
thread_local geomst_stats_t g_stats;
double g_beta_growth = 0.0;  // 0: 2 for EMST, sqrt(2) for HDBSCAN*
double g_separation = 2.0;   // s of the sphere separation test
int g_sep_mode = 0;          // 0: geometric or mutually unreachable (Sec. 3.2.2); 1: geometric only
// Round schedule: 0 distance thresholds (default); 1 Naive (one round, all
// pairs); 2 GFK (Alg. 2: cardinality beta, BCCPs of every pair up to beta);
// 3 MemoGFK (Alg. 3: cardinality beta, pairs retrieved up to rho_hi).
int g_sched = 0;
int g_bccp_chunk = kBigBDefault;  // B points per large-pair BCCP task
double g_capacity_scale = 1.0;
double g_beta_start = 0.0;  // fraction of the initial pair bounds below the first threshold (0: the smallest)
int g_beta_plain = 0;        // 1: the threshold grows by exactly g every round (no early-round acceleration)
double g_share_scale = 1.0;  // server workers: scale of the workspace share a batch may grow to (testing aid)
constexpr int kMaxKeyLevels = 6;  // Morton key words per point (see k_morton_level)
constexpr int kLevelBatch = 6;    // expansion levels launched between host checks
// refresh node components once a round merged n / this many (the default
// means about every round that merged anything: the splits and the levels
// drop connected pairs by these labels, so fresh ones pay for the refresh)
constexpr u32 kRefreshDefault = 1048576;
u32 g_refresh_div = kRefreshDefault;
u32 g_small_switch = 2048;  // queues up to kRegions times this go to the per-region level kernel
u32 g_small_max = 4096;     // ... whose workgroups keep going while their levels stay this small
u32 g_wide_switch = 2048;   // queues up to kRegions * kSub times this go to the wide level kernel (0: off)
u32 g_wide_max = 4096;      // ... whose workgroups keep going while their levels stay this small
constexpr int kBoruvkaBatch = 4;  // Boruvka steps launched between host checks
// beta grows faster while the tree has fewer than n / this many edges
// (HDBSCAN*, whose larger early rounds cost more, and EMST)
constexpr u32 kSparseDivHdb = 64;
constexpr u32 kSparseDivEmst = 16;
const bool g_trace = getenv("GEOMST_TRACE") != nullptr;

// Options of one solve: the process-wide values (geomst_set_option) read
// once under a lock when the solve starts, so a change made meanwhile never
// reaches a running solve; knobs still at their built-in defaults take the
// loaded tuning table's value for the solve's (kind, d, log2 n) instead.
struct Opts {
    double beta_growth, separation, capacity_scale, beta_start;
    int bccp_chunk, beta_plain, sep_mode, sched;
    u32 refresh_div, small_switch, small_max, wide_switch, wide_max;
    bool tuned = false;
};

struct TuneEntry {
    int kind, d, nlog2;  // kind 0 EMST, 1 HDBSCAN*
    int bccp_chunk = 0;
    u32 small_switch = 0, small_max = 0, refresh_div = 0;
    double beta_growth = 0.0, beta_start = -1.0;
};

std::mutex g_opt_mu;
std::vector<TuneEntry> g_tuning;

int log2_floor(int64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

Opts snapshot_options(int kind, int d, int64_t n) {
    std::lock_guard<std::mutex> lk(g_opt_mu);
    Opts o;
    o.beta_growth = g_beta_growth;
    o.separation = g_separation;
    o.capacity_scale = g_capacity_scale;
    o.beta_start = g_beta_start;
    o.bccp_chunk = g_bccp_chunk;
    o.beta_plain = g_beta_plain;
    o.sep_mode = g_sep_mode;
    o.sched = g_sched;
    o.refresh_div = g_refresh_div;
    o.small_switch = g_small_switch;
    o.small_max = g_small_max;
    o.wide_switch = g_wide_switch;
    o.wide_max = std::max(g_wide_max, g_wide_switch);
    // HDBSCAN* from d = 4 keeps its mid-size levels on the whole grid: its
    // expansions there are uneven enough that the wide kernel's slowest
    // workgroup sets the pace (2M 5-D mixture 85 -> 106 ms with it; EMST and
    // HDBSCAN* up to d = 3 gain 2 to 8 %)
    if (kind == 1 && d >= 4 && o.wide_switch == 2048 && o.wide_max == 4096) o.wide_switch = o.wide_max = 0;
    // the entry of the same kind and d whose log2 n is nearest (within 2)
    const TuneEntry* best = nullptr;
    const int nl = log2_floor(n);
    for (const TuneEntry& e : g_tuning) {
        if (e.kind != kind || e.d != d || std::abs(e.nlog2 - nl) > 2) continue;
        if (!best || std::abs(e.nlog2 - nl) < std::abs(best->nlog2 - nl)) best = &e;
    }
    if (best) {
        if (best->bccp_chunk && o.bccp_chunk == kBigBDefault) o.bccp_chunk = best->bccp_chunk;
        if (best->small_switch && o.small_switch == 2048 && o.small_max == 4096) {
            o.small_switch = best->small_switch;
            o.small_max = std::max(best->small_max, best->small_switch);
        }
        if (best->refresh_div && o.refresh_div == kRefreshDefault) o.refresh_div = best->refresh_div;
        if (best->beta_growth > 0.0 && o.beta_growth == 0.0) o.beta_growth = best->beta_growth;
        if (best->beta_start >= 0.0 && o.beta_start == 0.0) o.beta_start = best->beta_start;
        o.tuned = true;
    }
    return o;
}

struct Fail {
    int code;
};

// The device counters block: the Counters record followed by the few words
// the host reads back with it, so that one copy serves each host check.
constexpr size_t kAuxLstate = (sizeof(Counters) + 63) / 64 * 64;   // pairs left by a small-level launch (1 word)
constexpr size_t kAuxNalive = kAuxLstate + 64;                     // Boruvka alive counts (2 words)
constexpr size_t kAuxRing = (kAuxNalive + 64 + 255) / 256 * 256;   // level-queue count ring
constexpr size_t kCntBytes = kAuxRing + (size_t)kQRing * kSlotWords * 4;

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

// A fixed device region carved by bumping an offset (the no-allocation entry
// point's scratch).  While a solve on this thread has one installed, every
// buffer a solve grows comes from it instead of hipMalloc; a buffer that is
// the region's last carve grows in place, others move up and abandon their
// old range until the region is reset for the next call.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, top = 0;
    void* last = nullptr;
};
thread_local Arena* g_arena = nullptr;

// Device-memory accounting of the workspace a solve on this thread grows
// (set by the server's workers): growth beyond `limit` bytes fails with
// ENOMEM before any allocation is made.
struct WsBudget {
    std::atomic<size_t> held{0};
    size_t limit = ~(size_t)0;
};
thread_local WsBudget* g_ws_budget = nullptr;

// Grow-only device buffer.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool fixed = false;  // carved from an Arena: never freed
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() {
        if (p && !fixed) (void)hipFree(p);
    }
    void ensure(size_t need, size_t keep = 0, hipStream_t s = 0) {
        if (need <= bytes) return;
        size_t nb = std::max(need, bytes + bytes / 2);
        nb = (nb + 255) & ~(size_t)255;
        if (g_arena) {
            carve(*g_arena, nb, keep, s);
            return;
        }
        if (g_ws_budget) {
            if (g_ws_budget->held - bytes + nb > g_ws_budget->limit) {
                g_err = "the worker's workspace would exceed its share of the device-memory budget";
                throw Fail{GEOMST_ENOMEM};
            }
        }
        void* q = nullptr;
        // queued kernels of this solve may still use p (solves leave no work
        // queued behind them, so this solve's stream is the only one to wait for)
        if (p) HIPCHK(hipStreamSynchronize(g_cur_stream));
        HIPCHK(hipMalloc(&q, nb));
        if (keep && p) {
            HIPCHK(hipMemcpyAsync(q, p, std::min(keep, bytes), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        if (p) HIPCHK(hipFree(p));
        if (g_ws_budget) g_ws_budget->held = g_ws_budget->held - bytes + nb;
        p = q;
        bytes = nb;
    }
    template <class T>
    T* as() const {
        return (T*)p;
    }
    void carve(Arena& A, size_t nb, size_t keep, hipStream_t s) {
        if (p && !fixed) {
            g_err = "internal: a heap buffer met the fixed scratch";
            throw Fail{GEOMST_EINTERNAL};
        }
        if (p && p == A.last && (size_t)((char*)p - A.base) + nb <= A.cap) {
            A.top = (size_t)((char*)p - A.base) + nb;  // the last carve grows in place
            bytes = nb;
            return;
        }
        if (A.top + nb > A.cap) {
            g_err = "the solve needs more than the " + std::to_string(A.cap >> 20) +
                    " MiB of fixed device scratch of the no-allocation entry point";
            throw Fail{GEOMST_ENOMEM};
        }
        void* q = A.base + A.top;
        if (keep && p) {
            HIPCHK(hipMemcpyAsync(q, p, std::min(keep, bytes), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        A.top += nb;
        A.last = q;
        p = q;
        bytes = nb;
        fixed = true;
    }
};

// Optional device timing of kernel families: event pairs recorded on the
// solve's stream around each launch group, resolved after the final sync.
struct Prof {
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, size_t>> pend;  // (family, first event index)
    size_t used = 0;
    bool on = false;
    u32 mask = 0;  // families timed while on
    ~Prof() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
    void begin(u32 families) {
        on = families != 0;
        mask = families;
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

// Workspace of the dendrogram call (see dendro_kernels.h).
struct DendroBufs {
    DBuf eu, ev, key[2], val[2], pos, first, nx[2], dd[2], near, pedge, lab, sz, P, MX, SZ, OWN, par[2], off[2], err;
};

struct Device {
    std::mutex mu;
    bool init = false;
    hipStream_t own = nullptr;
    Counters* hcnt = nullptr;  // pinned mirror of the counters block (kCntBytes)
    u32* hpin = nullptr;       // pinned words read back together with the counters
    DBuf cnt;
    // input staging (host API)
    DBuf pin, eout, wout, cdout;
    // tree
    DBuf keysA, keysB, gflag, gincl, gid, gstart, gbox, hflag;
    DBuf part, bbox, key, val, key2, val2, stemp, X, xc, orig, cd2, nodes, npar, flags, cdr, btop, nrange;
    // union-find / component refresh
    DBuf uf, best, bnd, incl, ncomp;
    // rounds
    DBuf F[2], Q[3], big, ntask, toff, parts, ubest, tdone, lbhist;
    size_t qmax_seen = 0;
    size_t capF[2] = {0, 0}, capQ[3] = {0, 0, 0}, capBig = 0, capTiny = 0;
    DBuf tiny;  // small separated pairs of the current round
    DBuf rq[2], rho, rhocnt;  // GetRho traversal of the cardinality schedules
    DBuf bb64;                // boxes of the aligned 64-point blocks (large-pair BCCP pruning)
    DBuf FF[2];  // far frontier (see the round loop)
    size_t capFF[2] = {0, 0};
    EdgeBufs C, P[2], OUT;
    // Kruskal
    DBuf kid, ke2, kw2, perm[2], alive[2], apos[2], ru, rv, minmax;
    DBuf birange, bik, browinst;  // batched solves: instance table and row -> instance
    DendroBufs dg;
    Prof profm;
    Prof* prof = nullptr;
    bool noalloc = false;     // buffers come from the fixed scratch; no event timing
    WsBudget budget;          // bytes held by this workspace's buffers (server workers)
    double list_scale = 1.0;  // scale of the initial pair and edge list capacities
    ~Device() {
        if (own) (void)hipStreamDestroy(own);
        if (hcnt) (void)hipHostFree(hcnt);
        if (hpin) (void)hipHostFree(hpin);
    }
};

// Per-device workspaces of the plain and batched calls; never destroyed (the
// runtime may already be gone at static destruction).
Device* const g_dev = new Device[16];
u32 g_kernel_timing = 0;                    // families timed (bit per GEOMST_K_*); 0 = off
u32 g_kernel_timing_families = 0xffffffffu;  // restriction set by "kernel_timing_families"



struct TimedScope {
    Prof& P;
    hipStream_t s;
    int fam;
    size_t a = 0;
    bool on;
    TimedScope(Prof& p, hipStream_t st, int f) : P(p), s(st), fam(f), on(p.on && ((p.mask >> f) & 1u)) {
        if (on) a = P.rec(s);
    }
    ~TimedScope() {
        // never throws: a failed record only loses this sample
        if (on && P.used < P.pool.size() + 1) {
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

// Timing of back-to-back launches of one family: one event between
// consecutive launches closes the previous sample and opens the next, so a
// batch of k launches records k + 1 events instead of 2k.
struct TimedChain {
    Prof& P;
    hipStream_t s;
    int fam;
    bool on;
    size_t last = 0;
    TimedChain(Prof& p, hipStream_t st, int f) : P(p), s(st), fam(f), on(p.on && ((p.mask >> f) & 1u)) {
        if (on) last = P.rec(s);
    }
    void tick() {
        if (!on) return;
        const size_t e = P.rec(s);  // events are numbered in record order
        P.pend.push_back({fam, last});
        last = e;
    }
};

// Reads the first `bytes` of the counters block into its pinned mirror.
void read_counters(Device& D, hipStream_t s, size_t bytes = sizeof(Counters)) {
    HIPCHK(hipMemcpyAsync(D.hcnt, D.cnt.p, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

u32* aux_dev(Device& D, size_t off) { return (u32*)((char*)D.cnt.p + off); }
const u32* aux_host(const Device& D, size_t off) { return (const u32*)((const char*)D.hcnt + off); }

// Queues a copy of c to the device counters.  The pinned mirror is the copy
// source, so the host leaves it alone until the next read_counters.
void write_counters(Device& D, const Counters& c, hipStream_t s) {
    *D.hcnt = c;
    HIPCHK(hipMemcpyAsync(D.cnt.p, D.hcnt, sizeof(Counters), hipMemcpyHostToDevice, s));
}

// Error flags the kernels raise (bit 1 list overflow is handled by round
// restarts before this is reached).
void check_errors(Device& D) {
    u32 e = D.hcnt->c[C_ERR];
    if (e & (1u | 4u | 8u)) {
        g_err = (e & 8u) ? "union-find walk did not terminate"
                : (e & 4u) ? "k-NN stack overflow" : "output edge overflow";
        throw Fail{GEOMST_EINTERNAL};
    }
}

double bits_to_double(u64 b) {
    double x;
    memcpy(&x, &b, 8);
    return x;
}

const double kInf = __builtin_inf();
constexpr int kPinWords = 2048;  // pinned read-back words per device (the bound histogram is the largest use)

int id_bits(int n) {
    u32 m = (u32)(n - 1);
    int b = 0;
    while (m) {
        ++b;
        m >>= 1;
    }
    return b < 1 ? 1 : b;
}

// Sort m edges of L by K = (w2, d2, lo, hi); returns the permutation (sorted
// rank -> edge).  Each key word is gathered once and then sorted as (key,
// index) pairs with sequential passes, least significant word first, over
// only the bits below the highest bit where the word's min and max differ
// (every key shares the bits above).  Fast path: sort by the leading bits of
// w2 alone (about log2 m + 8 of the bits that vary, in whole 8-bit passes)
// and keep that order when no two such keys are equal, else order each run
// of equal leading bits by (w2, d2, ids) in place.
u32* sort_edges(Device& D, const EdgeList& L, u32 m, int n, bool hdb, hipStream_t s, const u32* pinst = nullptr) {
    D.kid.ensure((size_t)m * 8);
    D.kw2.ensure((size_t)m * 8);
    D.perm[0].ensure((size_t)m * 4);
    D.perm[1].ensure((size_t)m * 4);
    D.stemp.ensure(radix_temp_bytes(m));
    D.minmax.ensure(64);
    int B = id_bits(n);
    TIMED(GEOMST_K_SORT);
    u64* ka = D.kid.as<u64>();
    u64* kb = D.kw2.as<u64>();
    u32* va = D.perm[0].as<u32>();
    u32* vb = D.perm[1].as<u32>();
    unsigned gg = std::min(blocks(m, kBlock), (unsigned)kGrid);
    u64* mm = D.minmax.as<u64>();
    u32* longrun = D.minmax.as<u32>() + 9;
    int* lead_sh = (int*)(D.minmax.as<u32>() + 10);  // first w2 bit of the fast path's sort
    // one word: gather through the current permutation (in place), then sort
    // on the bits that vary
    auto word = [&](const u32* perm, int kind) {
        k_sort_init<<<1, kWave, 0, s>>>(mm, longrun - 1);
        LAUNCHCHK();
        k_gather_word<<<gg, kBlock, 0, s>>>(L, perm, m, kind, B, pinst, ka, va, mm);
        LAUNCHCHK();
        u64* h = (u64*)D.hpin;  // pinned
        HIPCHK(hipMemcpyAsync(h, mm, 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        u64 diff = h[0] ^ h[1];
        int bits = 0;
        while (bits < 64 && (diff >> bits)) ++bits;
        g_stats.sort_elems += (int64_t)m * ((bits + 7) / 8);
        if (radix_sort_pairs(ka, va, kb, vb, m, bits, D.stemp.p, s)) {
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        LAUNCHCHK();
    };
    // Batched output: the instance is the most significant word.
    auto finish = [&]() -> u32* {
        if (pinst) word(va, 3);
        return va;
    };
    // a short list: the whole order in one workgroup, no host round trip
    if (!pinst && m <= (u32)kSmallSort) {
        k_sort_small<<<1, kSmallSortBlock, 0, s>>>(L, m, va);
        LAUNCHCHK();
        return va;
    }
    // Fast path, one host round trip: sort by the leading `lead` varying bits
    // of w2 (the first of them found on the device), then order each run of
    // keys equal in those bits by (w2, d2, ids) in place.  A run too long
    // for that sends the list to the full order, least significant word
    // first.
    int lg = 0;
    while (lg < 32 && (1u << lg) < m) ++lg;
    const int lead = 8 * ((lg + 8 + 7) / 8);
    k_sort_init<<<1, kWave, 0, s>>>(mm, longrun - 1);
    LAUNCHCHK();
    k_gather_word<<<gg, kBlock, 0, s>>>(L, nullptr, m, 2, B, pinst, ka, va, mm);
    LAUNCHCHK();
    k_sort_lead<<<1, kWave, 0, s>>>(mm, lead, lead_sh);
    LAUNCHCHK();
    g_stats.sort_elems += (int64_t)m * (lead / 8);
    if (radix_sort_pairs(ka, va, kb, vb, m, lead, D.stemp.p, s, 0, lead_sh)) {
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    LAUNCHCHK();
    D.ke2.ensure((size_t)m * 8);
    k_run_keys<<<gg, kBlock, 0, s>>>(L, ka, va, m, kb, D.ke2.as<u64>(), lead_sh);
    LAUNCHCHK();
    k_fix_runs<<<gg, kBlock, 0, s>>>(ka, va, kb, D.ke2.as<u64>(), m, vb, longrun, lead_sh);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(D.hpin, longrun, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (D.hpin[0] == 0) {
        std::swap(va, vb);
        return finish();
    }
    word(nullptr, 0);
    if (hdb) word(va, 1);
    word(va, 2);
    return finish();
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
    int key_levels = 1;
    // batched solve (forest of instances); all null for a single instance
    int ninst = 1;
    const u32* pinst = nullptr;   // instance of each row / sorted position
    const int2* irange = nullptr; // (first row, rows) per instance
    const int* ik = nullptr;      // k-NN k per instance
    u32 target_edges = 0;         // edges of the whole forest

    Opts o;                       // this solve's options (snapshot)

    Solver(Device& dev, hipStream_t stream, int n_, int mp, geomst_stats_t& stats, const Opts& opts)
        : D(dev), s(stream), n(n_), minpts(mp), hdb(mp > 0), st(stats), target_edges((u32)(n_ - 1)), o(opts) {}

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
        k_bbox_final<D_><<<1, kBboxFinal, 0, s>>>(D.part.as<double>(), (int)nbb, D.bbox.as<double>());
        LAUNCHCHK();
        D.key.ensure((size_t)n * 8);
        D.key2.ensure((size_t)n * 8);
        D.val.ensure((size_t)n * 4);
        D.val2.ensure((size_t)n * 4);
        D.stemp.ensure(std::max(radix_temp_bytes(n), scan_temp_bytes(n)));
        int mb = (63 / D_) > 31 ? 31 : (63 / D_);
        int bits0 = mb * D_;
        if (pinst) {
            k_inst_key<<<blocks(n, 256), 256, 0, s>>>(pinst, n, D.key.as<u64>(), D.val.as<u32>());
            bits0 = id_bits(ninst);
        } else {
            k_morton<D_><<<blocks(n, 256), 256, 0, s>>>(P, n, D.bbox.as<double>(), D.key.as<u64>(), D.val.as<u32>());
        }
        LAUNCHCHK();
        g_stats.sort_elems += (int64_t)n * ((bits0 + 7) / 8);
        int flip = radix_sort_pairs(D.key.as<u64>(), D.val.as<u32>(), D.key2.as<u64>(), D.val2.as<u32>(), n,
                                    bits0, D.stemp.p, s);
        LAUNCHCHK();
        // multi-level keys: keysA holds L words per position, level-major
        D.keysA.ensure((size_t)kMaxKeyLevels * n * 8);
        D.keysB.ensure((size_t)kMaxKeyLevels * n * 8);
        u64* keys = D.keysA.as<u64>();
        u64* keysB = D.keysB.as<u64>();
        u32* vala = flip ? D.val2.as<u32>() : D.val.as<u32>();
        u32* valb = flip ? D.val.as<u32>() : D.val2.as<u32>();
        HIPCHK(hipMemcpyAsync(keys, flip ? D.key2.p : D.key.p, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        int L = 1;
        D.gflag.ensure((size_t)n * 4);
        D.gincl.ensure((size_t)n * 4);
        D.gid.ensure((size_t)n * 4);
        D.gstart.ensure((size_t)n * 4);
        D.perm[0].ensure((size_t)n * 4);
        D.perm[1].ensure((size_t)n * 4);
        D.hflag.ensure(16);
        while (L < kMaxKeyLevels && n > 1) {
            HIPCHK(hipMemsetAsync(D.hflag.p, 0, 16, s));
            k_key_flags<<<blocks(n, 256), 256, 0, s>>>(keys, n, L, D.gflag.as<u32>(), D.hflag.as<u32>());
            LAUNCHCHK();
            scan_inclusive_u32(D.gflag.as<u32>(), D.gincl.as<u32>(), n, D.stemp.p, s);
            LAUNCHCHK();
            u32* hv = D.hpin;  // pinned
            HIPCHK(hipMemcpyAsync(hv, D.hflag.p, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hv + 1, D.gincl.as<u32>() + n - 1, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (!hv[0]) break;  // every key is unique
            u32 ngroups = hv[1];
            D.gbox.ensure((size_t)ngroups * 2 * D_ * 8);
            k_group_ids<<<blocks(n, 256), 256, 0, s>>>(D.gincl.as<u32>(), n, D.gid.as<u32>(), D.gstart.as<u32>());
            LAUNCHCHK();
            k_group_box<D_><<<blocks(ngroups, 4), 256, 0, s>>>(P, vala, n, D.gstart.as<u32>(), ngroups,
                                                                D.gbox.as<double>(), D.hflag.as<u32>() + 1);
            LAUNCHCHK();
            HIPCHK(hipMemcpyAsync(D.hpin, D.hflag.as<u32>() + 1, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (!D.hpin[0]) break;  // the remaining equal keys belong to coincident points
            u64* kl = keys + (size_t)L * n;
            k_morton_level<D_><<<blocks(n, 256), 256, 0, s>>>(P, vala, n, D.gid.as<u32>(), D.gstart.as<u32>(),
                                                               ngroups, D.gbox.as<double>(), kl);
            LAUNCHCHK();
            // stable order by (group, new word): positions sorted by the new
            // word, then stably by the group id gathered through that order
            // (key-value sorts on contiguous keys)
            u32* pa = D.perm[0].as<u32>();
            u32* pb = D.perm[1].as<u32>();
            u64* ka = D.key.as<u64>();
            u64* kb = D.key2.as<u64>();
            k_iota<<<blocks(n, 256), 256, 0, s>>>(pa, n);
            LAUNCHCHK();
            HIPCHK(hipMemcpyAsync(ka, kl, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
            if (radix_sort_pairs(ka, pa, kb, pb, n, mb * D_, D.stemp.p, s)) {
                std::swap(ka, kb);
                std::swap(pa, pb);
            }
            LAUNCHCHK();
            k_gather_u32_u64<<<blocks(n, 256), 256, 0, s>>>(D.gid.as<u32>(), pa, n, ka);
            LAUNCHCHK();
            if (radix_sort_pairs(ka, pa, kb, pb, n, id_bits((int)ngroups), D.stemp.p, s)) {
                std::swap(ka, kb);
                std::swap(pa, pb);
            }
            LAUNCHCHK();
            g_stats.sort_elems += (int64_t)n * ((mb * D_ + 7) / 8 + (id_bits((int)ngroups) + 7) / 8);
            k_apply_perm<<<blocks(n, 256), 256, 0, s>>>(pa, n, L + 1, vala, valb, keys, keysB);
            LAUNCHCHK();
            std::swap(keys, keysB);
            std::swap(vala, valb);
            ++L;
        }
        key_levels = L;
        const u64* skey = keys;
        const u32* sval = vala;
        D.X.ensure((size_t)n * D_ * 8);
        D.orig.ensure((size_t)n * 4);
        k_permute<D_><<<blocks(n, 256), 256, 0, s>>>(P, n, sval, D.X.as<double>(), D.orig.as<u32>());
        LAUNCHCHK();
        D.nodes.ensure((size_t)nn * sizeof(NodeRec<D_>));
        D.npar.ensure((size_t)nn * 4);
        D.flags.ensure((size_t)nn * 4);
        NodeRec<D_>* nodes = D.nodes.as<NodeRec<D_>>();
        k_karras<D_><<<blocks(n - 1, 256), 256, 0, s>>>(skey, n, L, nodes, D.npar.as<int>());
        LAUNCHCHK();
        bounds(false);
        t.n = n;
        t.X = D.X.as<double>();
        t.orig = D.orig.as<u32>();
        t.cd2 = nullptr;
        t.nodes = nodes;
        t.cdr = nullptr;
        t.XC = nullptr;
    }

    // Node boxes (and, with cd2, core-distance ranges): block-local phase,
    // then one workgroup for the nodes spanning blocks.
    void bounds(bool cd) {
        const u32 nsb = blocks(n, kBoundsSpan);
        D.btop.ensure(((size_t)nsb * kBoundsSpanCap + (size_t)n + 64) * 4);
        D.flags.ensure(((size_t)n + nsb + 2) * 4);
        u32* ntop = D.flags.as<u32>() + n;  // per super-block counters after the arrival flags
        u32* ntop2 = ntop + nsb;
        u32* top2 = D.btop.as<u32>() + (size_t)nsb * kBoundsSpanCap;
        HIPCHK(hipMemsetAsync(D.flags.p, 0, ((size_t)n + nsb + 1) * 4, s));
        if (cd) D.cdr.ensure((size_t)(2 * n - 1) * 16);
        k_bounds_local<D_><<<blocks(n, kBoundsBlock), kBoundsBlock, 0, s>>>(
            n, D.X.as<double>(), cd ? D.cd2.as<double>() : nullptr, D.npar.as<int>(), D.nodes.as<NodeRec<D_>>(),
            cd ? D.cdr.as<double2>() : nullptr, cd ? 0 : 1, D.btop.as<u32>(), ntop);
        LAUNCHCHK();
        k_bounds_top<D_><<<nsb, kBoundsTop, 0, s>>>(n, D.npar.as<int>(), D.nodes.as<NodeRec<D_>>(),
                                                    cd ? D.cdr.as<double2>() : nullptr, cd ? 0 : 1, cd ? 1 : 0,
                                                    D.btop.as<u32>(), ntop, D.flags.as<u32>(), top2, ntop2);
        LAUNCHCHK();
        k_bounds_top<D_><<<1, kBoundsTop, 0, s>>>(n, D.npar.as<int>(), D.nodes.as<NodeRec<D_>>(),
                                                  cd ? D.cdr.as<double2>() : nullptr, cd ? 0 : 1, cd ? 1 : 0, top2,
                                                  ntop2, D.flags.as<u32>(), nullptr, nullptr);
        LAUNCHCHK();
    }

    template <int KMAX>
    void knn_k() {
        k_knn<D_, KMAX><<<blocks(n, 64), 64, 0, s>>>(t, minpts, pinst, irange, ik, D.cd2.as<double>(),
                                                      &D.cnt.as<Counters>()->c[C_ERR]);
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
        D.xc.ensure((size_t)n * (D_ + 1) * 8);
        k_append_cd<D_><<<blocks(n, 256), 256, 0, s>>>(D.X.as<double>(), D.cd2.as<double>(), D.xc.as<double>(), n);
        LAUNCHCHK();
        t.XC = D.xc.as<double>();
        bounds(true);
        t.cdr = D.cdr.as<double2>();
    }

    void refresh_components() {
        TIMED(GEOMST_K_REFRESH);
        k_uf_compress<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n, D.cnt.as<Counters>());
        LAUNCHCHK();
        k_boundaries<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n, D.bnd.as<u32>());
        LAUNCHCHK();
        scan_inclusive_u32(D.bnd.as<u32>(), D.incl.as<u32>(), n, D.stemp.p, s);
        LAUNCHCHK();
        k_node_comp<D_><<<blocks(2 * n - 1, 256), 256, 0, s>>>(D.nodes.as<NodeRec<D_>>(), D.ncomp.as<int>(),
                                                               D.nrange.as<int2>(), D.uf.as<u32>(),
                                                               D.incl.as<u32>(), 2 * n - 1);
        LAUNCHCHK();
    }

    u32 gfk_card = 0;     // GFK schedule: this round's cardinality beta (0 otherwise)

    // GetRho (Alg. 3; rho_hi of Alg. 2): the smallest weight lower bound of
    // the well-separated pairs below the waiting pairs (near list F[fc] and
    // far list FF[ffc]) with |A| + |B| > beta_card that are not connected,
    // by a pruned breadth-first traversal; +inf when there is none.
    double get_rho(u32 beta_card, int fc, u32 nF, int ffc, u32 nFF) {
        if ((u64)nF + nFF == 0) return kInf;
        TIMED(GEOMST_K_EXPAND);
        D.rho.ensure(8);
        D.rhocnt.ensure(4);
        u64* rho = D.rho.as<u64>();
        u32* cnt = D.rhocnt.as<u32>();
        k_set_u64<<<1, 1, 0, s>>>(rho, 0x7ff0000000000000ull);
        LAUNCHCHK();
        HIPCHK(hipMemsetAsync(cnt, 0, 4, s));
        size_t nin = (size_t)nF + nFF;
        D.rq[0].ensure(2 * nin * sizeof(PairRec));
        const int mutual = o.sep_mode == 0;
        const PairRec* lists[2] = {D.F[fc].as<PairRec>(), D.FF[ffc].as<PairRec>()};
        const u32 counts[2] = {nF, nFF};
        for (int l = 0; l < 2; ++l) {
            if (!counts[l]) continue;
            k_rho_level<D_><<<blocks(counts[l], kBlock), kBlock, 0, s>>>(t, hdb, mutual, o.separation, lists[l],
                                                                         counts[l], D.rq[0].as<PairRec>(), cnt,
                                                                         beta_card, rho);
            LAUNCHCHK();
        }
        int c = 0;
        while (true) {
            HIPCHK(hipMemcpyAsync(D.hpin, cnt, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            nin = D.hpin[0];
            if (!nin) break;
            D.rq[c ^ 1].ensure(2 * nin * sizeof(PairRec));
            HIPCHK(hipMemsetAsync(cnt, 0, 4, s));
            k_rho_level<D_><<<blocks(nin, kBlock), kBlock, 0, s>>>(t, hdb, mutual, o.separation,
                                                                   D.rq[c].as<PairRec>(), (u32)nin,
                                                                   D.rq[c ^ 1].as<PairRec>(), cnt, beta_card, rho);
            LAUNCHCHK();
            c ^= 1;
        }
        HIPCHK(hipMemcpyAsync(D.hpin, rho, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        u64 b;
        memcpy(&b, D.hpin, 8);
        return bits_to_double(b);
    }

    double t_near = 0.0;  // edge of the near frontier band
    u32 bstamp = 0;       // Boruvka step stamp (decreases by one per step)
    int ffo = 0;          // far list receiving appends this round

    // Diagnostic (GEOMST_TRACE): size classes of the round's large pairs and
    // how well their BCCP tasks fill the lanes.
    void trace_big_pairs(u32 nbig, u32 ntasks) {
        std::vector<uint2> bp(nbig);
        std::vector<NodeRec<D_>> nd((size_t)2 * n - 1);
        HIPCHK(hipMemcpyAsync(bp.data(), D.big.p, (size_t)nbig * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(nd.data(), D.nodes.p, nd.size() * sizeof(NodeRec<D_>), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double mid_ev = 0, big_ev = 0, slots = 0;
        u64 nmid = 0, nlarge = 0;
        u64 hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // large pairs by min side: <64,<256,<1k,<4k,<16k,<64k,more
        double hev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (u32 i = 0; i < nbig; ++i) {
            double a = nd[bp[i].x].count, b = nd[bp[i].y].count;
            if (b > a) std::swap(a, b);
            double w = a * b;
            if (w <= kMidMax) {
                ++nmid;
                mid_ev += w;
                continue;
            }
            ++nlarge;
            big_ev += w;
            double ta = std::ceil(a / kBigA), tbn = std::ceil(b / o.bccp_chunk);
            slots += ta * kBigA * (tbn > 1 ? b : b);  // lanes x B points each task row covers
            int h = b < 64 ? 0 : b < 256 ? 1 : b < 1024 ? 2 : b < 4096 ? 3 : b < 16384 ? 4 : b < 65536 ? 5 : 6;
            ++hist[h];
            hev[h] += w;
        }
        fprintf(stderr,
                "[geomst]   big pairs: %u (%llu medium, %.3g evals; %llu large, %.3g evals, A-lane fill %.2f) "
                "tasks %u; large by smaller side <64/<256/<1k/<4k/<16k/<64k/more:",
                nbig, (unsigned long long)nmid, mid_ev, (unsigned long long)nlarge, big_ev,
                slots > 0 ? big_ev / slots : 0.0, ntasks);
        for (int h = 0; h < 7; ++h) fprintf(stderr, " %llu(%.2g)", (unsigned long long)hist[h], hev[h]);
        fprintf(stderr, "\n");
    }

    RoundArgs args(double beta2, int fo, int qo, int po) {
        RoundArgs r;
        r.cnt = D.cnt.as<Counters>();
        r.beta2 = beta2;
        r.sep = o.separation;
        r.mutual = o.sep_mode == 0;
        r.beta_card = gfk_card;
        r.t_near = t_near;
        r.ffar = D.FF[ffo].as<PairRec>();
        r.cap_far = (u32)D.capFF[ffo];
        r.uf = D.uf.as<u32>();
        r.fout = D.F[fo].as<PairRec>();
        r.cap_f = (u32)D.capF[fo];
        r.q = D.Q[qo].as<PairRec>();
        r.cap_q = (u32)(D.capQ[qo] / kRegions);  // per region
        r.big = D.big.as<uint2>();
        r.cap_big = (u32)D.capBig;
        r.tiny = D.tiny.as<uint4>();
        r.cap_tiny = (u32)D.capTiny;
        r.c = D.C.list();
        r.cap_c = (u32)D.C.cap;
        r.pout = D.P[po].list();
        r.cap_p = (u32)D.P[po].cap;
        r.labels = D.ncomp.as<int>();
        return r;
    }

    // Total and largest region count of level-queue ring slot `slot`, read
    // together with the counters (one host round trip for both).
    void read_slot(int slot, u32& total, u32& largest) {
        const size_t off = kAuxRing + (size_t)slot * kSlotWords * 4;
        read_counters(D, s, off + kSlotWords * 4);
        const u32* h = aux_host(D, off);
        total = largest = 0;
        for (int x = 0; x < kRegions; ++x) {
            total += h[x * kRegionStride];
            largest = std::max(largest, h[x * kRegionStride]);
        }
    }

    // List lengths are counted in 32 bits on the device.
    static constexpr size_t kMaxListCap = 0xffffff00u;

    // After an overflow: grow the round's output lists that ran out.  Their
    // contents are not kept (the round restarts); the round's input frontier
    // F[fc] and input pool P[pc] are never touched.
    void grow_lists(int fo, int po, size_t keep_far) {
        const Counters& c = *D.hcnt;
        if (g_trace)
            fprintf(stderr,
                    "[geomst] need/cap per point: F %.3f/%.3f far %.3f/%.3f queue %.3f/%.3f big %.4f/%.4f "
                    "C %.3f/%.3f P %.3f/%.3f tiny %.3f/%.3f\n",
                    (double)c.c[C_F] / n, (double)D.capF[fo] / n, (double)c.c[C_FAR] / n, (double)D.capFF[ffo] / n,
                    (double)D.qmax_seen / n, (double)std::max(D.capQ[0], D.capQ[1]) / n, (double)c.c[C_BIG] / n,
                    (double)D.capBig / n, (double)c.c[C_C] / n, (double)D.C.cap / n, (double)c.c[C_P] / n,
                    (double)D.P[po].cap / n, (double)c.c[C_TINY] / n, (double)D.capTiny / n);
        // A count read at an overflow only bounds the round's need from below
        // (the round stopped early); lists grow to 1.25 times the count, and
        // at least double.  The frontier and the level queues carry the same
        // pairs level by level, so when either overflows both grow to the
        // larger need.
        auto grow_pairs = [&](DBuf& b, size_t& cap, size_t need) {
            if (need > cap) {
                size_t nc = std::min<size_t>(std::max<size_t>(need + need / 4, cap * 2), kMaxListCap) / kRegions * kRegions;
                b.ensure(nc * sizeof(PairRec));
                cap = nc;
            }
        };
        // level queues (kRegions equal regions; qmax_seen is kRegions times the
        // largest region count seen): the split's counts are exact; an
        // overflowing level's count may already be cleared, so then they double
        size_t qneed = D.qmax_seen;
        if (c.c[C_ERR] & 16u) qneed = std::max(qneed, std::max(D.capQ[0], D.capQ[1]) + 1);
        size_t fneed = c.c[C_F];
        if (fneed > D.capF[fo] || qneed > std::min(D.capQ[0], D.capQ[1])) fneed = qneed = std::max(fneed, qneed);
        grow_pairs(D.F[fo], D.capF[fo], fneed);
        if (c.c[C_FAR] > D.capFF[ffo]) {  // keeps the far pairs retained from earlier rounds
            size_t nc = std::min<size_t>(std::max<size_t>((size_t)c.c[C_FAR] + c.c[C_FAR] / 4, D.capFF[ffo] * 2), kMaxListCap);
            D.FF[ffo].ensure(nc * sizeof(PairRec), keep_far * sizeof(PairRec), s);
            D.capFF[ffo] = nc;
        }
        for (int i = 0; i < 2; ++i) grow_pairs(D.Q[i], D.capQ[i], qneed);
        if (c.c[C_TINY] > D.capTiny) {
            size_t nc = std::min<size_t>(std::max<size_t>((size_t)c.c[C_TINY] + c.c[C_TINY] / 4, D.capTiny * 2), kMaxListCap);
            D.tiny.ensure(nc * sizeof(uint4));
            D.capTiny = nc;
        }
        if (c.c[C_BIG] > D.capBig) {
            size_t nc = std::max<size_t>((size_t)c.c[C_BIG] * 5 / 4, D.capBig * 2);
            D.big.ensure(nc * 8);
            D.capBig = nc;
        }
        if (c.c[C_C] > D.C.cap) D.C.ensure(std::max<size_t>((size_t)c.c[C_C] * 5 / 4, D.C.cap * 2), 0, s);
        if (c.c[C_P] > D.P[po].cap) D.P[po].ensure(std::max<size_t>((size_t)c.c[C_P] * 5 / 4, D.P[po].cap * 2), 0, s);
    }

    // Kruskal on m edges of L: sorted by K, then Boruvka steps on the ranks
    // until no edge joins two components (Sec. 3.1.2); tree edges go to OUT.
    void kruskal(const EdgeList& L, u32 m) {
        u32* perm = sort_edges(D, L, m, n, hdb, s);
        D.alive[0].ensure((size_t)m * 4);
        D.alive[1].ensure((size_t)m * 4);
        D.apos[0].ensure((size_t)m * 8);
        D.apos[1].ensure((size_t)m * 8);
        D.ru.ensure((size_t)m * 4);
        D.rv.ensure((size_t)m * 4);
        u32* nalive = aux_dev(D, kAuxNalive);
        unsigned gk = std::min(blocks(m, kBlock), (unsigned)kGrid);
        k_alive_init<<<gk, kBlock, 0, s>>>(perm, L, m, D.alive[0].as<u32>(), D.apos[0].as<u64>());
        LAUNCHCHK();
        k_set_u32<<<1, 1, 0, s>>>(nalive, m);
        LAUNCHCHK();
        int ac = 0;
        while (true) {
            for (int j = 0; j < kBoruvkaBatch; ++j) {
                TIMED(GEOMST_K_KRUSKAL);
                u32* na_in = nalive + ac;
                u32* na_out = nalive + (ac ^ 1);
                const u32 stamp = --bstamp;  // decreasing: this step's keys beat older ones
                k_bor_pick<<<gk, kBlock, 0, s>>>(D.alive[ac].as<u32>(), D.apos[ac].as<u64>(), na_in, m,
                                                D.uf.as<u32>(), D.best.as<u64>(), stamp, D.ru.as<u32>(),
                                                D.rv.as<u32>(), na_out, D.cnt.as<Counters>());
                LAUNCHCHK();
                k_bor_hook<<<std::min(blocks(m, kHookTile), 256u), kHookBlock, 0, s>>>(
                    D.alive[ac].as<u32>(), na_in, m, perm, L, D.uf.as<u32>(),
                    D.best.as<u64>(), stamp, D.ru.as<u32>(), D.rv.as<u32>(), D.alive[ac ^ 1].as<u32>(),
                    D.apos[ac ^ 1].as<u64>(), na_out, D.OUT.list(), (u32)D.OUT.cap, D.cnt.as<Counters>());
                LAUNCHCHK();
                ac ^= 1;
            }
            read_counters(D, s, kAuxNalive + 8);  // the counters and the alive count
            if (aux_host(D, kAuxNalive)[ac] == 0) break;
        }
    }

    // Kruskal over the m approximate-OPTICS candidates in D.C by weight
    // buckets: the candidates are scattered once into buckets cut at
    // quantiles of a strided sample of their weights (the lightest ~3n
    // candidates, then up to 1/16, 1/4, 1/2, 5/8, 3/4 and 7/8 of them, then
    // the rest);
    // bucket 0 goes to Kruskal as it is, every later bucket first drops the
    // edges whose ends the lighter buckets have already joined (cycle
    // property), and the buckets stop once the tree is complete.
    void kruskal_filtered(u32 m) {
        const u64 slice_min = std::max<u64>((u64)3 * (u64)n, 1u << 16);
        if ((u64)m <= 2 * slice_min) {
            kruskal(D.C.list(), m);
            return;
        }
        constexpr u32 kSample = 1u << 16;
        D.minmax.ensure(kSample * 8);
        const u64 step = (u64)m / kSample;
        const u32 ns = (u32)std::min<u64>(kSample, (u64)m / step);
        k_sample_w2<<<blocks(ns, 256), 256, 0, s>>>(D.C.w2.as<double>(), m, step, ns, D.minmax.as<double>());
        LAUNCHCHK();
        std::vector<double> smp(ns);
        HIPCHK(hipMemcpyAsync(smp.data(), D.minmax.p, (size_t)ns * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::sort(smp.begin(), smp.end());
        const double fr[7] = {std::max((double)slice_min / (double)m, 1.0 / 128.0), 1.0 / 16.0, 0.25, 0.5, 0.625,
                              0.75, 0.875};
        Buckets bk{};
        bk.nt = 0;
        for (double f : fr) {
            const size_t q = std::min<size_t>(ns - 1, (size_t)(f * (double)ns));
            u64 tb;
            memcpy(&tb, &smp[q], 8);
            ++tb;  // bucket below: w2 <= the quantile
            if (bk.nt == 0 || tb > bk.t[bk.nt - 1]) bk.t[bk.nt++] = tb;
        }
        const int nbk = bk.nt + 1;
        u32* cnt = aux_dev(D, kAuxLstate);  // 2 words there, then room up to the alive counts
        static_assert(kAuxNalive - kAuxLstate >= 2 * kMaxBuckets * 4, "bucket counters fit the state words");
        u32* cur = cnt + kMaxBuckets;
        HIPCHK(hipMemsetAsync(cnt, 0, 2 * kMaxBuckets * 4, s));
        {
            TIMED(GEOMST_K_KRUSKAL);
            k_bucket_count<<<std::min(blocks(m, kPartBlock), 4096u), kPartBlock, 0, s>>>(D.C.w2.as<double>(), m, bk,
                                                                                        cnt);
            LAUNCHCHK();
        }
        read_counters(D, s, kAuxLstate + 2 * kMaxBuckets * 4);
        u32 count[kMaxBuckets], off[kMaxBuckets];
        Buckets base{};
        base.nt = bk.nt;
        u32 run = 0;
        for (int b = 0; b < nbk; ++b) {
            count[b] = aux_host(D, kAuxLstate)[b];
            off[b] = run;
            if (b) base.t[b - 1] = run;
            run += count[b];
        }
        if (run != m) {
            g_err = "candidate buckets lost entries";
            throw Fail{GEOMST_EINTERNAL};
        }
        D.P[0].ensure((size_t)m, 0, s);
        {
            TIMED(GEOMST_K_KRUSKAL);
            k_bucket_scatter<<<std::min(blocks(m, kPartBlock), 4096u), kPartBlock, 0, s>>>(D.C.list(), m, bk,
                                                                                          D.P[0].list(), base, cur);
            LAUNCHCHK();
        }
        u32 maxb = 0;
        for (int b = 1; b < nbk; ++b) maxb = std::max(maxb, count[b]);
        if (maxb) D.P[1].ensure((size_t)maxb, 0, s);
        for (int b = 0; b < nbk; ++b) {
            if (!count[b]) continue;
            EdgeList L = D.P[0].list();
            EdgeList seg{L.w2 + off[b], L.e2 + off[b], L.ids + off[b], L.pos + off[b]};
            if (b == 0) {
                kruskal(seg, count[b]);
                continue;
            }
            read_counters(D, s);
            if (D.hcnt->c[C_OUT] >= target_edges) break;
            HIPCHK(hipMemsetAsync(&D.cnt.as<Counters>()->c[C_C], 0, 4, s));
            {
                TIMED(GEOMST_K_KRUSKAL);
                // tbits 0: every candidate takes the heavy test (ends in
                // different components), none is light
                k_partition_cand<<<std::min(blocks(count[b], kPartBlock), 4096u), kPartBlock, 0, s>>>(
                    seg, count[b], 0ull, D.P[1].list(), 0u, D.P[1].list(), D.uf.as<u32>(), D.cnt.as<Counters>());
                LAUNCHCHK();
            }
            read_counters(D, s);
            const u32 kept = D.hcnt->c[C_C];
            if (g_trace)
                fprintf(stderr, "[geomst] filtered kruskal: bucket %d of %d: %u candidates, %u kept\n", b, nbk,
                        count[b], kept);
            if (kept) kruskal(D.P[1].list(), kept);
        }
    }

    // Approximate OPTICS (paper Appendix; see approx_kernels.h): the whole
    // decomposition level by level, each separated pair's candidate edge,
    // then one Kruskal pass over the candidates.  Room for a level's appends
    // (two children and one candidate per input pair) is made before its
    // launch, so no append can overflow.
    void run_approx(const double* P, double rho, long long* edges, double* w, double* w2, double* cd,
                    double* cd2out) {
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
        core_distances();
        HIPCHK(hipStreamSynchronize(s));
        auto t2 = clk::now();
        D.uf.ensure((size_t)n * 4);
        D.best.ensure((size_t)n * 8);
        k_iota<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n);
        LAUNCHCHK();
        HIPCHK(hipMemsetAsync(D.best.p, 0xff, (size_t)n * 8, s));
        bstamp = 0xffffffffu;
        D.OUT.ensure((size_t)n + 64, 0, s);

        const double sep = std::sqrt(8.0 / rho);
        ApproxArgs a;
        a.cnt = D.cnt.as<Counters>();
        a.K = (sep + 2.0) * (sep + 2.0);
        a.q = (1.0 + rho) * (1.0 + rho);
        a.min_pts = minpts;
        int b = 0;
        u64 nq = (u64)(n - 1), m = 0;
        D.Q[0].ensure(nq * sizeof(PairRec), 0, s);
        k_init_frontier<D_><<<blocks(n - 1, 256), 256, 0, s>>>(t, 1, nullptr, D.Q[0].as<PairRec>());
        LAUNCHCHK();
        int levels = 0;
        while (nq) {
            if (m + nq >= 0x80000000ull || 2 * nq >= 0x80000000ull) {
                g_err = "the decomposition has more than 2^31 pairs (choose a larger rho)";
                throw Fail{GEOMST_ENOMEM};
            }
            D.Q[b ^ 1].ensure((size_t)(2 * nq) * sizeof(PairRec), 0, s);
            D.C.ensure((size_t)(m + nq), (size_t)m, s);
            a.qout = D.Q[b ^ 1].as<PairRec>();
            a.c = D.C.list();
            HIPCHK(hipMemsetAsync(&D.cnt.as<Counters>()->c[C_QN], 0, 4, s));
            {
                TIMED(GEOMST_K_EXPAND);
                k_approx_level<D_><<<std::min(blocks(nq, kApproxBlock), 4096u), kApproxBlock, 0, s>>>(
                    t, a, D.Q[b].as<PairRec>(), (u32)nq);
                LAUNCHCHK();
            }
            read_counters(D, s);
            ++levels;
            nq = D.hcnt->c[C_QN];
            m = D.hcnt->c[C_C];
            b ^= 1;
        }
        kruskal_filtered((u32)m);
        read_counters(D, s);
        check_errors(D);
        if (D.hcnt->c[C_OUT] != target_edges) {
            g_err = "wrong number of tree edges";
            throw Fail{GEOMST_EINTERNAL};
        }
        auto t3 = clk::now();
        EdgeList O = D.OUT.list();
        u32* perm = sort_edges(D, O, target_edges, n, true, s);
        {
            TIMED(GEOMST_K_OUTPUT);
            k_write_edges<<<blocks(target_edges, 256), 256, 0, s>>>(O, perm, target_edges, nullptr, nullptr, edges,
                                                                    w, w2);
            LAUNCHCHK();
            if (cd || cd2out) {
                k_write_cd<<<blocks(n, 256), 256, 0, s>>>(D.cd2.as<double>(), D.orig.as<u32>(), n, cd, cd2out);
                LAUNCHCHK();
            }
        }
        read_counters(D, s);
        check_errors(D);
        auto t4 = clk::now();
        auto ms = [](clk::time_point x, clk::time_point y) {
            return std::chrono::duration<double, std::milli>(y - x).count();
        };
        st.rounds = levels;
        st.pair_visits = (int64_t)D.hcnt->c64[C64_VISITS];
        st.bccp_evals = (int64_t)D.hcnt->c64[C64_EVALS];
        st.bccp_evals_done = st.bccp_evals;
        st.bccp_pairs = (int64_t)D.hcnt->c64[C64_BCCP];
        st.committed_edges = (int64_t)m;
        st.ms_tree = ms(t0, t1);
        st.ms_core = ms(t1, t2);
        st.ms_rounds = ms(t2, t3);
        st.ms_final = ms(t3, t4);
        D.prof->finish(st);
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
        if (g_trace) fprintf(stderr, "[geomst] key levels %d\n", key_levels);
        if (hdb) {
            core_distances();
            HIPCHK(hipStreamSynchronize(s));
        }
        auto t2 = clk::now();

        // boxes of the aligned 64-point blocks for the large-pair BCCP
        {
            TIMED(GEOMST_K_BCCP_LARGE);
            const u32 nb64 = (u32)((n + 63) / 64);
            D.bb64.ensure((size_t)nb64 * (2 * D_ + 1) * 8);
            k_block_boxes<D_><<<blocks(nb64, kBlock), kBlock, 0, s>>>(t, hdb, D.bb64.as<double>());
            LAUNCHCHK();
        }
        // union-find and node components
        D.nrange.ensure((size_t)(2 * n - 1) * 8);
        // compact label copy; a value no label takes, so the first refresh
        // writes every record
        D.ncomp.ensure((size_t)(2 * n - 1) * 4);
        HIPCHK(hipMemsetAsync(D.ncomp.p, 0x80, (size_t)(2 * n - 1) * 4, s));
        k_node_ranges<D_><<<blocks(2 * n - 1, 256), 256, 0, s>>>(D.nodes.as<NodeRec<D_>>(), 2 * n - 1,
                                                                 D.nrange.as<int2>());
        LAUNCHCHK();
        D.uf.ensure((size_t)n * 4);
        D.best.ensure((size_t)n * 8);
        D.bnd.ensure((size_t)n * 4);
        D.incl.ensure((size_t)n * 4);
        D.stemp.ensure(std::max(radix_temp_bytes(n), scan_temp_bytes(n)));
        k_iota<<<blocks(n, 256), 256, 0, s>>>(D.uf.as<u32>(), n);
        LAUNCHCHK();
        HIPCHK(hipMemsetAsync(D.best.p, 0xff, (size_t)n * 8, s));
        bstamp = 0xffffffffu;
        refresh_components();

        // lists
        auto initcap = [&](size_t& cap, DBuf& b, size_t want) {
            if (cap < want) {
                b.ensure(want * sizeof(PairRec));
                cap = want;
            }
        };
        auto sc = [&](double per_point) {
            return std::max<size_t>(64, (size_t)(o.capacity_scale * D.list_scale * (per_point * n + 4096)));
        };
        if (o.capacity_scale != 1.0) {  // testing aid: start from the given capacities
            for (int i = 0; i < 2; ++i) {
                D.capF[i] = D.capQ[i] = D.capFF[i] = 0;
                D.P[i].cap = 0;
            }
            D.capBig = 0;
            D.capTiny = 0;
            D.C.cap = 0;
        }
        // frontier and queue: pairs per point they typically reach (they grow
        // with d), so that a first solve seldom restarts rounds to grow them
        static const double kInitPairs[8] = {0, 4, 4, 12, 16, 24, 48, 96};
        const double fq = std::max(kInitPairs[D_], hdb ? 4.0 : 2.0);
        initcap(D.capF[0], D.F[0], sc(fq));
        initcap(D.capF[1], D.F[1], sc(fq));
        static const double kInitFar[8] = {0, 4, 4, 4, 8, 16, 32, 64};
        initcap(D.capFF[0], D.FF[0], sc(kInitFar[D_] * (hdb ? 2 : 1)));
        initcap(D.capFF[1], D.FF[1], sc(kInitFar[D_] * (hdb ? 2 : 1)));
        // a thin-level chain keeps its queue in one region: room for a level
        // of up to small_max pairs and its children
        const size_t qmin = (size_t)(std::min(o.capacity_scale, 1.0) * kRegions * (2 * (double)o.small_max + 2048));
        initcap(D.capQ[0], D.Q[0], (std::max(sc(fq), qmin) + kRegions - 1) / kRegions * kRegions);
        initcap(D.capQ[1], D.Q[1], (std::max(sc(fq), qmin) + kRegions - 1) / kRegions * kRegions);
        if (D.capTiny < sc(hdb ? 8 : 3)) {
            D.capTiny = sc(hdb ? 8 : 3);
            D.tiny.ensure(D.capTiny * sizeof(uint4));
        }
        if (D.capBig < sc(0.125)) {
            D.capBig = sc(0.125);
            D.big.ensure(D.capBig * 8);
        }
        D.C.ensure(sc(hdb ? 6 : 3), 0, s);
        D.P[0].ensure(sc(1), 0, s);
        D.P[1].ensure(sc(1), 0, s);
        D.OUT.ensure((size_t)n + 64, 0, s);

        // initial frontier: the children of every internal node
        // Waiting pairs live in two lists: "near" (bound up to t_near, due
        // within a few rounds; streamed every round) and "far" (re-split, with
        // connectivity pruning, only when beta passes t_near).  The initial
        // pairs start in the far list.
        int fc = 0, pc = 0, ffc = 0;
        k_init_frontier<D_><<<blocks(n - 1, 256), 256, 0, s>>>(t, hdb, pinst, D.FF[ffc].as<PairRec>());
        LAUNCHCHK();
        const bool want_hist = o.beta_start > 0.0;
        if (want_hist) {
            D.lbhist.ensure(kExpBins * 4);
            HIPCHK(hipMemsetAsync(D.lbhist.p, 0, kExpBins * 4, s));
        }
        k_min_positive_lb<<<std::min(blocks(n - 1, kBlock), (unsigned)kGrid), kBlock, 0, s>>>(
            D.FF[ffc].as<PairRec>(), (u32)(n - 1), D.cnt.as<Counters>(), want_hist ? D.lbhist.as<u32>() : nullptr);
        LAUNCHCHK();
        const u32* lbh = D.hpin;  // pinned
        if (want_hist) HIPCHK(hipMemcpyAsync(D.hpin, D.lbhist.p, kExpBins * 4, hipMemcpyDeviceToHost, s));
        read_counters(D, s);
        u64 b0 = D.hcnt->m[M_F];
        double beta2 = (b0 == ~0ull) ? 0.0 : bits_to_double(b0);
        const double far_first = beta2;
        // The first threshold: the low edge of the binade in which the given
        // fraction of the initial pairs' positive bounds is reached (never
        // below the smallest bound).  Rounds below it would commit almost
        // nothing; any start gives the same tree.
        if (o.beta_start > 0.0 && beta2 > 0.0) {
            u64 total = 0;
            for (int e = 0; e < kExpBins; ++e) total += lbh[e];
            const double target = std::max(1.0, std::ceil(o.beta_start * (double)total));
            u64 cum = 0;
            for (int e = 0; e < kExpBins; ++e) {
                cum += lbh[e];
                if ((double)cum >= target) {
                    beta2 = std::max(beta2, bits_to_double((u64)e << 52));
                    break;
                }
            }
        }
        // Naive: one round over every pair.  Cardinality schedules (single
        // instance): each round's threshold is GetRho of its beta.
        const int sched = pinst ? 0 : o.sched;
        if (sched == 1) beta2 = kInf;
        u32 beta_card = 2;
        u32 nF = 0, nFF = (u32)(n - 1), nP = 0;
        t_near = -1.0;  // the first round starts a band
        double far_min = far_first;
        const double growth = o.beta_growth > 0.0 ? o.beta_growth : (hdb ? 1.4142135623730951 : 2.0);
        const double g2 = growth * growth;
        u64 committed = 0, maxf = nF, big_pairs = 0;
        int rounds = 0;
        u32 nout = 0;
        int stale_rounds = 0;
        u32* ring = aux_dev(D, kAuxRing);
        while (true) {
            ++rounds;
            if (rounds > 100000) {
                g_err = "round limit exceeded";
                throw Fail{GEOMST_EINTERNAL};
            }
            int fo = fc ^ 1, po = pc ^ 1;
            if (sched >= 2) {
                // GetRho on current components: rho_hi of this round's
                // cardinality beta (an empty weight range only advances beta)
                if (stale_rounds) {
                    refresh_components();
                    stale_rounds = 0;
                }
                beta2 = std::max(beta2, get_rho(beta_card, fc, nF, ffc, nFF));
                gfk_card = sched == 2 ? beta_card : 0;
            }
            const bool epoch = beta2 > t_near;
            if (epoch) t_near = beta2 * g2 * g2;  // the band covers about two rounds
            ffo = epoch ? (ffc ^ 1) : ffc;
            // per-round counters reset on the device (error flags raised by
            // the previous round's last kernels stay for the next read), and
            // mirrored in the host copy, which a restart writes back
            const u32 far_keep = epoch ? 0u : nFF;  // far appends go after the retained pairs
            k_round_reset<<<1, kWave, 0, s>>>(D.cnt.as<Counters>(), far_keep, ring);
            LAUNCHCHK();
            for (int i = 0; i < C_OUT; ++i) D.hcnt->c[i] = 0;
            for (int i = 0; i < M_NUM; ++i) D.hcnt->m[i] = ~0ull;
            D.hcnt->c[C_FAR] = far_keep;
            D.hcnt->c[C_TINY] = 0;
            const Counters round_start = *D.hcnt;
            int levels = 0;
            u32 nbig = 0;
            bool restart;
            int restarts = 0;
            do {
                restart = false;
                levels = 0;
                D.qmax_seen = 0;
                if (restarts) HIPCHK(hipMemsetAsync(ring, 0, kQRing * kSlotWords * 4, s));  // else k_round_reset
                // frontier and pool split
                {
                    TIMED(GEOMST_K_SPLIT);
                    RoundArgs r = args(beta2, fo, 0, po);
                    if (nF)
                        k_split_frontier<D_><<<std::min(blocks(nF, kSplitTile), (unsigned)kGrid), kBlock, 0, s>>>(
                            t, r, D.F[fc].as<PairRec>(), nF, ring);
                    LAUNCHCHK();
                    if (nP)
                        k_split_pool<<<std::min(blocks(nP, kSplitTile), (unsigned)kGrid), kBlock, 0, s>>>(
                            r, D.P[pc].list(), nP);
                    LAUNCHCHK();
                    if (epoch && nFF)
                        k_split_far<D_><<<std::min(blocks(nFF, kSplitTile), (unsigned)kGrid), kBlock, 0, s>>>(
                            t, r, D.FF[ffc].as<PairRec>(), nFF, ring);
                    LAUNCHCHK();
                }
                u32 nq = 0, nq_region = 0;
                read_slot(0, nq, nq_region);
                D.hcnt->c[C_Q] = nq;
                D.qmax_seen = (size_t)kRegions * nq_region;
                if (D.hcnt->c[C_ERR] & 1u) {
                    restart = true;
                } else {
                    // breadth-first levels: thin chains run inside one
                    // workgroup; wide levels run grid-wide in batches launched
                    // without host syncs.  Q[lv & 1] holds the queue and
                    // ring[lv % 4] its count.
                    int lv = 0;
                    int sub = 1;  // layout of the current queue (kSub after the wide kernel)
                    // the wide kernel's workgroups need room for a level of
                    // wide_max pairs and its children in each part
                    const size_t wpart = 2 * (size_t)o.wide_max + 64;
                    const bool wide_ok = !D.noalloc && o.wide_switch > 0 &&
                                         std::min(D.capQ[0], D.capQ[1]) / kRegions / kSub >= wpart;
                    while (nq > 0) {
                        const bool regional = nq <= (u32)kRegions * o.small_switch;
                        if (regional || (wide_ok && nq <= (u64)kRegions * kSub * o.wide_switch)) {
                            const int groups = regional ? 1 : kSub;
                            if (groups > 1 && D.capQ[2] < kRegions * kSub * wpart) {
                                D.capQ[2] = kRegions * kSub * wpart;
                                D.Q[2].ensure(D.capQ[2] * sizeof(PairRec));
                            }
                            {
                                TIMED(GEOMST_K_EXPAND);
                                RoundArgs r = args(beta2, fo, 0, po);
                                HIPCHK(hipMemsetAsync(aux_dev(D, kAuxLstate), 0, 4, s));
                                PairRec* qt = groups > 1 ? D.Q[2].as<PairRec>() : D.Q[0].as<PairRec>();
                                const u32 capt = groups > 1 ? (u32)(D.capQ[2] / kRegions) : 0u;
                                k_level_small<D_><<<kRegions * groups, SmallBlock<D_>::value, 0, s>>>(
                                    t, r, hdb, D.Q[0].as<PairRec>(), (u32)(D.capQ[0] / kRegions), D.Q[1].as<PairRec>(),
                                    (u32)(D.capQ[1] / kRegions), qt, capt, lv & 1, sub, groups, ring,
                                    (u32)(lv % kQRing), groups > 1 ? o.wide_max : o.small_max, aux_dev(D, kAuxLstate));
                                LAUNCHCHK();
                            }
                            read_counters(D, s, kAuxLstate + 8);
                            ++levels;
                            ++g_stats.level_launches[groups > 1 ? 2 : 1];
                            if (D.hcnt->c[C_ERR] & 1u) {
                                restart = true;
                                break;
                            }
                            nq = aux_host(D, kAuxLstate)[0];
                            ++lv;  // the remaining pairs: slot lv % kQRing, buffer lv & 1
                            sub = groups;
                            D.qmax_seen = std::max<size_t>(D.qmax_seen, (size_t)kRegions * nq);  // at most all in one region
                            continue;
                        }
                        TimedChain chain(*D.prof, s, GEOMST_K_EXPAND);
                        for (int j = 0; j < kLevelBatch; ++j, ++lv, ++levels) {
                            RoundArgs r = args(beta2, fo, (lv + 1) & 1, po);
                            k_level<D_><<<LevelShape<D_>::grid, LevelShape<D_>::block, 0, s>>>(t, r, hdb, D.Q[lv & 1].as<PairRec>(),
                                                                 (u32)(D.capQ[lv & 1] / kRegions), j == 0 ? sub : 1,
                                                                 ring + (lv % kQRing) * kSlotWords,
                                                                 ring + ((lv + 1) % kQRing) * kSlotWords,
                                                                 ring + ((lv + 2) % kQRing) * kSlotWords);
                            LAUNCHCHK();
                            chain.tick();
                            ++g_stats.level_launches[0];
                        }
                        sub = 1;
                        read_slot(lv % kQRing, nq, nq_region);
                        D.qmax_seen = std::max<size_t>(D.qmax_seen, (size_t)kRegions * nq_region);
                        if (D.hcnt->c[C_ERR] & 1u) {
                            restart = true;
                            break;
                        }
                        if (levels > 1000000) {
                            g_err = "level limit exceeded";
                            throw Fail{GEOMST_EINTERNAL};
                        }
                    }
                }
                if (!restart) {
                    // small separated pairs: brute-force BCCP, one pair per thread
                    const u32 ntiny = std::min<u32>(D.hcnt->c[C_TINY], (u32)D.capTiny);
                    if (ntiny) {
                        TIMED(GEOMST_K_BCCP);
                        RoundArgs r = args(beta2, fo, 0, po);
                        k_tiny_bccp<D_><<<std::min(blocks(ntiny, kTinyTile), (unsigned)kTinyGrid), kTinyBlock, 0, s>>>(
                            t, r, hdb, D.tiny.as<uint4>(), ntiny);
                        LAUNCHCHK();
                    }
                    nbig = D.hcnt->c[C_BIG];
                    if (!nbig && ntiny) {
                        read_counters(D, s);
                        if (D.hcnt->c[C_ERR] & 1u) restart = true;
                    }
                    if (nbig) {
                        D.ntask.ensure((size_t)nbig * 4);
                        D.toff.ensure((size_t)nbig * 4);
                        D.stemp.ensure(std::max(scan_temp_bytes(nbig), radix_temp_bytes(n)));
                        HIPCHK(hipMemsetAsync(&D.cnt.as<Counters>()->c64[C64_TASKS], 0, 8, s));
                        k_big_ntasks<D_><<<blocks(nbig, 256), 256, 0, s>>>(t, D.big.as<uint2>(), nbig,
                                                                            D.ntask.as<u32>(), o.bccp_chunk,
                                                                            D.cnt.as<Counters>());
                        LAUNCHCHK();
                        scan_exclusive_u32(D.ntask.as<u32>(), D.toff.as<u32>(), nbig, D.stemp.p, s);
                        LAUNCHCHK();
                        u32 last_off = 0, last_cnt = 0;
                        HIPCHK(hipMemcpyAsync(D.hpin, D.toff.as<u32>() + nbig - 1, 4, hipMemcpyDeviceToHost, s));
                        HIPCHK(hipMemcpyAsync(D.hpin + 1, D.ntask.as<u32>() + nbig - 1, 4, hipMemcpyDeviceToHost, s));
                        read_counters(D, s);  // synchronises
                        last_off = D.hpin[0];
                        last_cnt = D.hpin[1];
                        if (D.hcnt->c64[C64_TASKS] >= (1ull << 31)) {
                            g_err = "the separated pairs of one round need more than 2^31 BCCP tasks";
                            throw Fail{GEOMST_EINTERNAL};
                        }
                        u32 ntasks = last_off + last_cnt;
                        if (g_trace) trace_big_pairs(nbig, ntasks);
                        D.parts.ensure((size_t)ntasks * sizeof(PartKey));
                        D.ubest.ensure((size_t)nbig * 8);
                        D.tdone.ensure((size_t)ntasks * 4);
                        {
                            TIMED(GEOMST_K_BCCP_LARGE);
                            HIPCHK(hipMemsetAsync(D.ubest.p, 0xff, (size_t)nbig * 8, s));  // no weight yet
                            if (hdb)
                                k_big_bccp<D_, 1><<<ntasks, 64, 0, s>>>(t, D.big.as<uint2>(), nbig, D.toff.as<u32>(),
                                                                       D.parts.as<PartKey>(), D.cnt.as<Counters>(),
                                                                       o.bccp_chunk, D.ubest.as<u64>(), D.tdone.as<u32>(),
                                                                       D.bb64.as<double>());
                            else
                                k_big_bccp<D_, 0><<<ntasks, 64, 0, s>>>(t, D.big.as<uint2>(), nbig, D.toff.as<u32>(),
                                                                       D.parts.as<PartKey>(), D.cnt.as<Counters>(),
                                                                       o.bccp_chunk, D.ubest.as<u64>(), D.tdone.as<u32>(),
                                                                       D.bb64.as<double>());
                            LAUNCHCHK();
                            // the per-pair best weights are dead after k_big_bccp: the
                            // same array then holds each pair's evaluation count
                            k_big_reduce<<<blocks(nbig, kBlock / kWave), kBlock, 0, s>>>(
                                nbig, D.toff.as<u32>(), D.ntask.as<u32>(), D.parts.as<PartKey>(), D.tdone.as<u32>(),
                                D.ubest.as<unsigned long long>());
                            LAUNCHCHK();
                            RoundArgs r = args(beta2, fo, 0, po);
                            k_big_combine<<<std::min(blocks(nbig, kBlock), (unsigned)kGrid), kBlock, 0, s>>>(
                                r, nbig, D.toff.as<u32>(), D.parts.as<PartKey>(), D.ubest.as<unsigned long long>());
                            LAUNCHCHK();
                        }
                        read_counters(D, s);
                        if (D.hcnt->c[C_ERR] & 1u) restart = true;
                    }
                }
                if (restart) {
                    if (++restarts > 64) {
                        g_err = "internal lists kept overflowing";
                        throw Fail{GEOMST_EINTERNAL};
                    }
                    if (g_trace) fprintf(stderr, "[geomst] round %d: list overflow, growing and restarting\n", rounds);
                    if (D.hcnt->c[C_ERR] & (4u | 8u)) check_errors(D);  // not an overflow: report it
                    grow_lists(fo, po, epoch ? 0 : nFF);
                    write_counters(D, round_start, s);
                }
            } while (restart);
            big_pairs += nbig;
            // Kruskal on the committed edges
            u32 m = D.hcnt->c[C_C];
            committed += m;
            if (m) kruskal(D.C.list(), m);
            // The counters read last (after the Kruskal steps, or after the
            // expansion when nothing was committed) are this round's final
            // values.  Refresh the node components unless this round merged
            // almost nothing (stale labels only miss some pruning: components
            // only grow, so a node labelled with one component still is in
            // one); its error flags are checked at the next read.
            const Counters& c = *D.hcnt;
            check_errors(D);
            u32 merged = c.c[C_OUT] - nout;
            if ((u64)merged * o.refresh_div >= (u64)n || stale_rounds >= 3 || c.c[C_OUT] >= target_edges) {
                refresh_components();
                stale_rounds = 0;
            } else {
                ++stale_rounds;
            }
            nout = c.c[C_OUT];
            nF = c.c[C_F];
            nFF = c.c[C_FAR];
            ffc = ffo;
            double mfar = c.m[M_FAR] == ~0ull ? kInf : bits_to_double(c.m[M_FAR]);
            far_min = epoch ? mfar : std::min(far_min, mfar);
            nP = c.c[C_P];
            maxf = std::max<u64>(maxf, (u64)nF + nFF);
            fc = fo;
            pc = po;
            if (g_trace) {
                fprintf(stderr,
                        "[geomst] round %d beta2=%.6g levels=%d visits=%llu F=%u+%u P=%u C=%u big=%u out=%u "
                        "t=%.2fms\n",
                        rounds, beta2, levels, (unsigned long long)c.c64[C64_VISITS], nF, nFF, nP, m, nbig, nout,
                        std::chrono::duration<double, std::milli>(clk::now() - t2).count());
            }
            if (nout >= target_edges) break;
            double mf = c.m[M_F] == ~0ull ? kInf : bits_to_double(c.m[M_F]);
            double mp = c.m[M_P] == ~0ull ? kInf : bits_to_double(c.m[M_P]);
            double nxt = std::min(std::min(mf, mp), far_min);
            if (nxt == kInf) {
                g_err = "no pairs left before the tree was complete";
                throw Fail{GEOMST_EINTERNAL};
            }
            // While the tree is nearly empty (the first rounds: the smallest
            // pair bounds lie far below the bulk of the tree's weights) a
            // round costs its fixed work for few edges, so the threshold then
            // grows by g^2 at once.  Later rounds that merge little (the gaps
            // between clusters) keep the plain growth: there, larger steps
            // put more inter-cluster pairs into one round, before their
            // components are known.  Any schedule gives the same tree.
            // For EMST, a round that found no edge at all (nothing committed,
            // pooled or queued as a large pair, before the first edge) grows
            // it by g^4: on the same grid of thresholds, it skips rounds that
            // would only split pairs.  (For HDBSCAN* the larger first round
            // this leads to cost more than the rounds it saves.)
            if (sched >= 2) {  // Alg. 2 / Alg. 3: beta doubles
                beta_card = beta_card >= 0x80000000u ? 0xffffffffu : beta_card * 2;
                continue;
            }
            const bool sparse = !o.beta_plain && (u64)nout * (hdb ? kSparseDivHdb : kSparseDivEmst) < (u64)n;
            const bool empty = !o.beta_plain && !hdb && nout == 0 && m == 0 && nP == 0 && nbig == 0;
            beta2 = std::max(beta2 * (empty ? g2 * g2 * g2 * g2 : sparse ? g2 * g2 : g2), nxt);
        }
        if (nout != target_edges) {
            g_err = "wrong number of tree edges";
            throw Fail{GEOMST_EINTERNAL};
        }
        auto t3 = clk::now();
        // output: sort the tree edges by K and write them
        EdgeList O = D.OUT.list();
        u32* perm = target_edges ? sort_edges(D, O, target_edges, n, hdb, s, pinst) : nullptr;
        {
        TIMED(GEOMST_K_OUTPUT);
        if (target_edges) {
            k_write_edges<<<blocks(target_edges, 256), 256, 0, s>>>(O, perm, target_edges, pinst, irange, edges, w,
                                                                    w2);
            LAUNCHCHK();
        }
        }
        if (hdb && (cd || cd2out)) {
            TIMED(GEOMST_K_OUTPUT);
            k_write_cd<<<blocks(n, 256), 256, 0, s>>>(D.cd2.as<double>(), D.orig.as<u32>(), n, cd, cd2out);
            LAUNCHCHK();
        }
        read_counters(D, s);
        check_errors(D);
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
        st.bccp_evals_done =
            (int64_t)(D.hcnt->c64[C64_EVALS] - D.hcnt->c64[C64_BIGWORK] + D.hcnt->c64[C64_BIGEVALS]);
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
    HIPCHK(hipHostMalloc((void**)&D.hcnt, kCntBytes, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&D.hpin, kPinWords * sizeof(u32), hipHostMallocDefault));
    D.cnt.ensure(kCntBytes);
    D.prof = &D.profm;
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
               double* w2, double* cd, double* cd2, double rho = 0.0) {
    g_cur_stream = s;
    memset(&g_stats, 0, sizeof(g_stats));
    g_stats.n = n;
    g_stats.d = d;
    g_stats.min_pts = minpts;
    D.prof->begin(D.noalloc ? 0u : (g_kernel_timing & g_kernel_timing_families));
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
    const Opts opts = snapshot_options(minpts > 0 ? 1 : 0, d, n);
    g_stats.tuning_applied = opts.tuned ? 1 : 0;
    switch (d) {
#define CASE(K)                                                   \
    case K: {                                                     \
        Solver<K> sv(D, s, n, minpts, g_stats, opts);             \
        if (rho > 0.0)                                            \
            sv.run_approx(P, rho, edges, w, w2, cd, cd2);         \
        else                                                      \
            sv.run(P, edges, w, w2, cd, cd2);                     \
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

// Batched solve over a packed device arena (see geomst_batch_dev).
void solve_batch_dev(Device& D, hipStream_t s, const double* P, int stride, const geomst_batch_item_t* items,
                     int64_t count, long long* edges, double* w, double* w2, double* cd, double* cd2) {
    g_cur_stream = s;
    memset(&g_stats, 0, sizeof(g_stats));
    D.prof->begin(g_kernel_timing & g_kernel_timing_families);
    auto t0 = std::chrono::steady_clock::now();
    int64_t N = 0;
    int maxk = 0;
    bool hdb = false;
    std::vector<int2> hr((size_t)count);
    std::vector<int> hk((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        hr[i] = make_int2((int)items[i].offset, (int)items[i].n);
        N += items[i].n;
        hdb |= items[i].min_pts > 0;
        maxk = std::max(maxk, (int)items[i].min_pts);
    }
    for (int64_t i = 0; i < count; ++i) hk[i] = items[i].min_pts > 0 ? items[i].min_pts : 1;
    g_stats.n = N;
    g_stats.d = stride;
    g_stats.min_pts = maxk;
    D.birange.ensure((size_t)count * 8);
    D.bik.ensure((size_t)count * 4);
    D.browinst.ensure((size_t)N * 4);
    HIPCHK(hipMemcpyAsync(D.birange.p, hr.data(), (size_t)count * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(D.bik.p, hk.data(), (size_t)count * 4, hipMemcpyHostToDevice, s));
    k_row_instance<<<blocks(N, 256), 256, 0, s>>>(D.birange.as<int2>(), (u32)count, (u32)N, D.browinst.as<u32>());
    LAUNCHCHK();
    if (N == count) {
        // every instance is a single point: no edges, core distances 0
        if (cd) HIPCHK(hipMemsetAsync(cd, 0, (size_t)N * 8, s));
        if (cd2) HIPCHK(hipMemsetAsync(cd2, 0, (size_t)N * 8, s));
        HIPCHK(hipStreamSynchronize(s));
        return;
    }
    const Opts opts = snapshot_options(hdb ? 1 : 0, stride, N);
    g_stats.tuning_applied = opts.tuned ? 1 : 0;
    switch (stride) {
#define CASE(K)                                                   \
    case K: {                                                     \
        Solver<K> sv(D, s, (int)N, hdb ? maxk : 0, g_stats, opts); \
        sv.ninst = (int)count;                                    \
        sv.pinst = D.browinst.as<u32>();                          \
        sv.irange = D.birange.as<int2>();                         \
        sv.ik = D.bik.as<int>();                                  \
        sv.target_edges = (u32)(N - count);                       \
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
            g_err = "unsupported stride";
            throw Fail{GEOMST_EINVAL};
    }
    HIPCHK(hipStreamSynchronize(s));
    g_stats.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int validate_batch(int32_t stride, const geomst_batch_item_t* items, int64_t count) {
    if (!items || count < 1) {
        g_err = "items is NULL or count < 1";
        return GEOMST_EINVAL;
    }
    if (stride < 1 || stride > kMaxDim) {
        g_err = "stride must be in [1, 7]";
        return GEOMST_EINVAL;
    }
    int64_t off = 0;
    for (int64_t i = 0; i < count; ++i) {
        const geomst_batch_item_t& it = items[i];
        bool bad = it.offset != off || it.n < 1 || it.d < 1 || it.d > stride || it.min_pts < 0 || it.min_pts > 64 ||
                   it.min_pts > it.n;
        if (bad) {
            g_err = "batch item " + std::to_string(i) +
                    " is invalid (items must be packed in order; n >= 1; 1 <= d <= stride; 0 <= min_pts <= "
                    "min(n, 64))";
            return GEOMST_EINVAL;
        }
        off += it.n;
    }
    if (off > (1ll << 26)) {
        g_err = "total points must be at most 2^26";
        return GEOMST_EINVAL;
    }
    return GEOMST_OK;
}

// One instance of a host-side batch: caller-owned arrays.
struct HostItem {
    const double* points;
    int64_t n;
    int d, min_pts;
    int64_t* edges;
    double* weights;
    double* core_dist;
};

// Host-side check of one instance: GEOMST_OK, GEOMST_EINVAL for a bad shape
// or pointer, GEOMST_EDOM for a coordinate that is not finite or exceeds 2^500.
int check_host_item(const HostItem& q) {
    if (!q.points || q.n < 1 || q.n > (1ll << 26) || q.d < 1 || q.d > kMaxDim || q.min_pts < 0 || q.min_pts > 64 ||
        q.min_pts > q.n || (q.n > 1 && !q.edges))
        return GEOMST_EINVAL;
    for (int64_t j = 0; j < q.n * q.d; ++j)
        if (!(fabs(q.points[j]) <= 0x1p500)) return GEOMST_EDOM;
    return GEOMST_OK;
}

// Packs host instances into one arena (stride = largest d, missing columns
// 0.0), solves them as one forest on the workspace's stream and scatters the
// edges (local ids), weights and core distances back. Throws Fail.
void solve_host_items(Device& D, const HostItem* it, int64_t count) {
    int stride = 0;
    int64_t N = 0;
    for (int64_t i = 0; i < count; ++i) {
        stride = std::max(stride, it[i].d);
        N += it[i].n;
    }
    std::vector<double> host((size_t)N * stride, 0.0);
    std::vector<geomst_batch_item_t> items((size_t)count);
    int64_t off = 0;
    for (int64_t i = 0; i < count; ++i) {
        const HostItem& q = it[i];
        for (int64_t r = 0; r < q.n; ++r)
            for (int k = 0; k < q.d; ++k) host[(size_t)(off + r) * stride + k] = q.points[r * q.d + k];
        items[i] = geomst_batch_item_t{off, q.n, q.d, q.min_pts};
        off += q.n;
    }
    if (int rc = validate_batch(stride, items.data(), count)) throw Fail{rc};
    hipStream_t s = D.own;
    g_cur_stream = s;
    size_t m = (size_t)(N - count);
    D.pin.ensure((size_t)N * stride * 8);
    D.eout.ensure(m * 16 + 16);
    D.wout.ensure(m * 8 + 8);
    D.cdout.ensure((size_t)N * 8);
    HIPCHK(hipMemcpyAsync(D.pin.p, host.data(), (size_t)N * stride * 8, hipMemcpyHostToDevice, s));
    solve_batch_dev(D, s, D.pin.as<double>(), stride, items.data(), count, D.eout.as<long long>(),
                    D.wout.as<double>(), nullptr, D.cdout.as<double>(), nullptr);
    std::vector<long long> e(m * 2);
    std::vector<double> w(m), cd((size_t)N);
    if (m) {
        HIPCHK(hipMemcpyAsync(e.data(), D.eout.p, m * 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(w.data(), D.wout.p, m * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipMemcpyAsync(cd.data(), D.cdout.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t i = 0; i < count; ++i) {
        const HostItem& q = it[i];
        size_t eo = (size_t)(items[i].offset - i);
        for (int64_t k = 0; k < q.n - 1; ++k) {
            q.edges[2 * k] = e[2 * (eo + k)];
            q.edges[2 * k + 1] = e[2 * (eo + k) + 1];
            if (q.weights) q.weights[k] = w[eo + k];
        }
        if (q.core_dist)
            for (int64_t r = 0; r < q.n; ++r) q.core_dist[r] = q.min_pts > 0 ? cd[items[i].offset + r] : 0.0;
    }
}

int run_dev(const double* P, int64_t n, int32_t d, int32_t minpts, long long* edges, double* w, double* w2,
            double* cd, double* cd2, void* stream, double rho = 0.0) {
    g_err.clear();
    int rc = validate(P, n, d, minpts, edges);
    if (rc) return rc;
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        solve_dev(D, (hipStream_t)stream, P, (int)n, d, minpts, edges, w, w2, cd, cd2, rho);
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int run_host(const double* P, int64_t n, int32_t d, int32_t minpts, int64_t* edges, double* w, double* cd,
             double rho = 0.0) {
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
                  nullptr, (minpts > 0 && cd) ? D.cdout.as<double>() : nullptr, nullptr, rho);
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

// One line of a tuning cache: a flat JSON object such as
// {"kind": "emst", "d": 3, "nlog2": 25, "bccp_chunk": 1024,
//  "small_level_switch": 2048, "small_level_max": 4096, "beta_growth": 2.0,
//  "refresh_divisor": 1024, "beta_start_quantile": 0.0}
// (other keys the tuner records, e.g. measured times, are ignored).  Blank
// lines and lines starting with '#' are skipped.  Returns false on a
// malformed line or an out-of-range value.
bool parse_tune_line(const char* line, std::vector<TuneEntry>& out) {
    std::string t(line);
    size_t a = t.find_first_not_of(" \t\r\n");
    if (a == std::string::npos || t[a] == '#') return true;
    size_t b = t.find_last_not_of(" \t\r\n");
    if (t[a] != '{' || t[b] != '}') return false;
    std::string body = t.substr(a + 1, b - a - 1);
    TuneEntry e{};
    e.kind = -1;
    e.d = 0;
    e.nlog2 = -1;
    size_t p = 0;
    while (p < body.size()) {
        size_t q1 = body.find('"', p);
        if (q1 == std::string::npos) break;
        size_t q2 = body.find('"', q1 + 1);
        size_t colon = q2 == std::string::npos ? q2 : body.find(':', q2);
        if (colon == std::string::npos) return false;
        std::string key = body.substr(q1 + 1, q2 - q1 - 1);
        size_t v0 = body.find_first_not_of(" \t", colon + 1);
        if (v0 == std::string::npos) return false;
        size_t v1;
        std::string val;
        if (body[v0] == '"') {
            v1 = body.find('"', v0 + 1);
            if (v1 == std::string::npos) return false;
            val = body.substr(v0 + 1, v1 - v0 - 1);
            ++v1;
        } else {
            v1 = body.find(',', v0);
            if (v1 == std::string::npos) v1 = body.size();
            val = body.substr(v0, v1 - v0);
        }
        char* endp = nullptr;
        const double x = strtod(val.c_str(), &endp);
        const bool num = endp && endp != val.c_str();
        if (key == "kind") {
            if (val == "emst") e.kind = 0;
            else if (val == "hdbscan") e.kind = 1;
            else return false;
        } else if (key == "d") {
            if (!num || x < 1 || x > kMaxDim || x != (int)x) return false;
            e.d = (int)x;
        } else if (key == "nlog2") {
            if (!num || x < 0 || x > 26 || x != (int)x) return false;
            e.nlog2 = (int)x;
        } else if (key == "bccp_chunk") {
            if (!num || x < 64 || x > 65536 || x != 64.0 * (int)(x / 64.0)) return false;
            e.bccp_chunk = (int)x;
        } else if (key == "small_level_switch" || key == "small_level_max") {
            if (!num || x < 0 || x > 1048576 || x != (u32)x) return false;
            (key == "small_level_switch" ? e.small_switch : e.small_max) = (u32)x;
        } else if (key == "refresh_divisor") {
            if (!num || x < 1 || x > 1048576 || x != (u32)x) return false;
            e.refresh_div = (u32)x;
        } else if (key == "beta_growth") {
            if (!num || !(x > 1.0) || !(x < 1e6)) return false;
            e.beta_growth = x;
        } else if (key == "beta_start_quantile") {
            if (!num || !(x >= 0.0) || !(x <= 1.0)) return false;
            e.beta_start = x;
        }
        p = body.find(',', v1);
        if (p == std::string::npos) break;
        ++p;
    }
    if (e.kind < 0 || e.d < 1 || e.nlog2 < 0) return false;
    out.push_back(e);
    return true;
}

// ------------------------------------------------------------ dendrogram
int ceil_log2(u64 x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

// Ordered dendrogram and reachability plot of a spanning tree whose n-1
// edges come in their total order (see dendro_kernels.h for the steps).
void dendrogram_dev(Device& D, hipStream_t s, const long long* edges, const double* w, int n, int start,
                    long long* children, long long* size, long long* order, double* reach) {
    g_cur_stream = s;
    memset(&g_stats, 0, sizeof(g_stats));
    g_stats.n = n;
    D.prof->begin(D.noalloc ? 0u : (g_kernel_timing & g_kernel_timing_families));
    auto t0 = std::chrono::steady_clock::now();
    DendroBufs& B = D.dg;
    B.err.ensure(4);
    u32* err = B.err.as<u32>();
    HIPCHK(hipMemsetAsync(err, 0, 4, s));
    auto check = [&](const char* stage) {
        HIPCHK(hipMemcpyAsync(D.hpin, err, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const u32 e = D.hpin[0];
        if (e & (kDgErrIds | kDgErrTree)) {
            g_err = (e & kDgErrIds) ? "an edge has an endpoint outside [0, n) or joins a point to itself"
                                    : "the edges do not form a spanning tree of the n points";
            throw Fail{GEOMST_EINVAL};
        }
        if (e) {
            g_err = std::string("internal error in the dendrogram (") + stage + ")";
            throw Fail{GEOMST_EINTERNAL};
        }
    };
    if (n == 1) {
        k_dg_single<<<1, 1, 0, s>>>(order, reach);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(s));
        return;
    }
    const u32 m = (u32)(n - 1), na = 2 * m, nn = 2 * (u32)n - 1;
    B.eu.ensure((size_t)m * 4);
    B.ev.ensure((size_t)m * 4);
    for (int i = 0; i < 2; ++i) {
        B.key[i].ensure((size_t)na * 8);
        B.val[i].ensure((size_t)na * 4);
        B.nx[i].ensure((size_t)na * 4);
        B.dd[i].ensure((size_t)na * 4);
        B.par[i].ensure((size_t)nn * 4);
        B.off[i].ensure((size_t)nn * 4);
    }
    B.pos.ensure((size_t)na * 4);
    B.first.ensure((size_t)n * 4);
    B.near.ensure(m);
    B.pedge.ensure((size_t)n * 4);
    B.lab.ensure((size_t)na * 4);
    B.sz.ensure((size_t)na * 4);
    B.P.ensure((size_t)nn * 4);
    B.MX.ensure((size_t)nn * 4);
    B.SZ.ensure((size_t)nn * 4);
    B.OWN.ensure((size_t)nn * 4);
    D.stemp.ensure(std::max(radix_temp_bytes(na), scan_temp_bytes(na)));
    int c = 0;
    {
        TIMED(GEOMST_K_DENDRO);
        // 1. root the tree at the start: Euler tour and list ranking
        k_dg_load<<<blocks(m, 256), 256, 0, s>>>(edges, m, (u32)n, B.eu.as<u32>(), B.ev.as<u32>(),
                                                 B.key[0].as<u64>(), B.val[0].as<u32>(), err);
        LAUNCHCHK();
        const int flip = radix_sort_pairs(B.key[0].as<u64>(), B.val[0].as<u32>(), B.key[1].as<u64>(),
                                          B.val[1].as<u32>(), na, id_bits(n), D.stemp.p, s);
        LAUNCHCHK();
        const u64* skey = B.key[flip].as<u64>();
        const u32* sarc = B.val[flip].as<u32>();
        HIPCHK(hipMemsetAsync(B.first.p, 0xff, (size_t)n * 4, s));
        k_dg_adj<<<blocks(na, 256), 256, 0, s>>>(skey, sarc, na, B.pos.as<u32>(), B.first.as<u32>());
        LAUNCHCHK();
        k_dg_succ<<<blocks(na, 256), 256, 0, s>>>(skey, sarc, B.pos.as<u32>(), B.first.as<u32>(), na, (u32)start,
                                                  B.nx[0].as<u32>(), B.dd[0].as<u32>(), err);
        LAUNCHCHK();
        for (int r = 0, rounds = id_bits((int)na) + 1; r < rounds; ++r, c ^= 1) {
            k_dg_jump<<<blocks(na, 256), 256, 0, s>>>(B.nx[c].as<u32>(), B.dd[c].as<u32>(), B.nx[c ^ 1].as<u32>(),
                                                      B.dd[c ^ 1].as<u32>(), na);
            LAUNCHCHK();
        }
        k_dg_orient<<<blocks(m, 256), 256, 0, s>>>(B.eu.as<u32>(), B.ev.as<u32>(), B.nx[c].as<u32>(),
                                                   B.dd[c].as<u32>(), m, B.near.as<unsigned char>(),
                                                   B.pedge.as<u32>(), err);
        LAUNCHCHK();
    }
    check("rooting");
    {
        TIMED(GEOMST_K_DENDRO);
        // 2. children by heavy/light halving
        u32* lab = B.lab.as<u32>();
        u32* sz = B.sz.as<u32>();
        HIPCHK(hipMemcpyAsync(lab, B.eu.p, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(lab + m, B.ev.p, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
        k_dg_fill_u32<<<blocks(na, 256), 256, 0, s>>>(sz, na, 1u);
        LAUNCHCHK();
        for (int j = ceil_log2(m); j >= 1; --j) {
            k_dg_level_reset<<<blocks(na, 256), 256, 0, s>>>(lab, m, B.P.as<u32>(), B.MX.as<u32>(), B.SZ.as<u32>(),
                                                             B.OWN.as<u32>());
            LAUNCHCHK();
            k_dg_level_union<<<blocks(m, 256), 256, 0, s>>>(lab, m, j, B.P.as<u32>());
            LAUNCHCHK();
            k_dg_level_info<<<blocks(m, 256), 256, 0, s>>>(lab, sz, m, j, B.P.as<u32>(), B.MX.as<u32>(),
                                                            B.SZ.as<u32>(), B.OWN.as<u32>());
            LAUNCHCHK();
            k_dg_level_rename<<<blocks(m, 256), 256, 0, s>>>(lab, sz, m, (u32)n, j, B.P.as<u32>(), B.MX.as<u32>(),
                                                              B.SZ.as<u32>());
            LAUNCHCHK();
        }
        // 3. orientation, then in-order positions by pointer jumping
        k_dg_children<<<blocks(m, 256), 256, 0, s>>>(lab, sz, B.near.as<unsigned char>(), m, (u32)n, children, size,
                                                     B.par[0].as<u32>(), B.off[0].as<u32>());
        LAUNCHCHK();
        int q = 0;
        for (int r = 0, rounds = id_bits((int)nn) + 1; r < rounds; ++r, q ^= 1) {
            k_dg_jump<<<blocks(nn, 256), 256, 0, s>>>(B.par[q].as<u32>(), B.off[q].as<u32>(), B.par[q ^ 1].as<u32>(),
                                                      B.off[q ^ 1].as<u32>(), nn);
            LAUNCHCHK();
        }
        k_dg_plot<<<blocks(n, 256), 256, 0, s>>>(B.off[q].as<u32>(), B.pedge.as<u32>(), w, (u32)n, (u32)start, order,
                                                 reach, err);
        LAUNCHCHK();
    }
    check("positions");
    g_stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    D.prof->finish(g_stats);
}

int validate_dendro(const void* edges, const void* w, int64_t n, int64_t start, const void* order, const void* reach) {
    if (n < 1 || n > (1ll << 26)) {
        g_err = "n must be in [1, 2^26]";
        return GEOMST_EINVAL;
    }
    if (start < 0 || start >= n) {
        g_err = "start must be in [0, n)";
        return GEOMST_EINVAL;
    }
    if (!order || !reach || (n > 1 && (!edges || !w))) {
        g_err = "edges, weights, order or reach is NULL";
        return GEOMST_EINVAL;
    }
    return GEOMST_OK;
}

// ------------------------------------------------- no-allocation entry point
// geomst_emst_dev_noalloc runs the same solve as geomst_emst_dev with every
// device buffer carved from the fixed array `scratch` (below) and the counter
// read-backs in static host memory, so it calls no hipMalloc, hipHostMalloc,
// hipEventCreate or hipStreamCreate.  Per device: the array's device address
// (taken once with that device current), a lock that serialises the calls,
// and storage for a workspace that is rebuilt empty at every call.
constexpr size_t kNoAllocBytes = (size_t)GEOMST_NOALLOC_SCRATCH_MIB << 20;

struct NoAllocSlot {
    std::mutex mu;
    char* ptr = nullptr;  // device address of `scratch` on this device
    bool live = false;    // store holds a constructed workspace
    alignas(Device) unsigned char store[sizeof(Device)];
    alignas(256) unsigned char hcnt[kCntBytes];
    u32 hpin[kPinWords];
};
NoAllocSlot g_noalloc[16];

struct ArenaScope {
    explicit ArenaScope(Arena* a) { g_arena = a; }
    ~ArenaScope() { g_arena = nullptr; }
};

}  // namespace
}  // namespace geomst

// The no-allocation entry point's scratch (one copy per device, resident
// while the library is loaded).  Host code never passes this name to a
// kernel: it only stands in for the symbol; the device address comes from
// hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[geomst::kNoAllocBytes];

namespace geomst {
namespace {

int run_dev_noalloc(const double* P, int64_t n, int32_t d, long long* edges, double* w, double* w2, void* stream) {
    g_err.clear();
    int rc = validate(P, n, d, 0, edges);
    if (rc) return rc;
    if (n > GEOMST_NOALLOC_MAX_POINTS) {
        g_err = "n exceeds GEOMST_NOALLOC_MAX_POINTS (" + std::to_string(GEOMST_NOALLOC_MAX_POINTS) +
                ") for the no-allocation entry point";
        return GEOMST_EINVAL;
    }
    try {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        if (dev < 0 || dev >= 16) {
            g_err = "device index out of range";
            throw Fail{GEOMST_EDEVICE};
        }
        NoAllocSlot& S = g_noalloc[dev];
        std::lock_guard<std::mutex> lk(S.mu);
        if (!S.ptr) {
            void* a = nullptr;
            HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
            if (!a) {
                g_err = "hipGetSymbolAddress returned no address for the scratch array";
                throw Fail{GEOMST_EDEVICE};
            }
            S.ptr = (char*)a;
        }
        if (S.live) {
            Device* old = (Device*)S.store;
            old->hcnt = nullptr;  // static host memory, not pinned: nothing to free
            old->hpin = nullptr;
            old->~Device();
            S.live = false;
        }
        Device& D = *new (S.store) Device();
        S.live = true;
        D.hcnt = (Counters*)S.hcnt;
        D.hpin = S.hpin;
        D.noalloc = true;
        D.list_scale = 0.25;
        D.prof = &D.profm;
        Arena A;
        A.base = S.ptr;
        A.cap = kNoAllocBytes;
        ArenaScope scope(&A);
        D.cnt.ensure(kCntBytes);
        D.init = true;
        solve_dev(D, (hipStream_t)stream, P, (int)n, d, 0, edges, w, w2, nullptr, nullptr);
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

// ------------------------------------------------------------ serving
// Continuous batching: requests queue up with their arrival time; each worker
// thread owns a workspace and a stream, takes what is queued at the front (up
// to its share of the device-memory budget and the batch limits) and solves it
// as one forest batch. Batches of different workers overlap on the device, and
// requests that arrive meanwhile form the next batch.
using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    std::vector<double> pts;  // copied at submit
    HostItem item{};
    size_t footprint = 0;
    int status = GEOMST_OK;
    int lane = 0;
    std::string err;  // the worker's error message when status != OK
    bool started = false, done = false;
    Clock::time_point t_arrive, t_start, t_done;
    int batch_requests = 0;
    int64_t batch_points = 0;
};

// Device-memory estimate of one request inside a batch: staged points and
// outputs, multi-level sort keys and temporaries, 2n node records, union-find
// and component arrays, the edge pools at their initial capacities, for
// HDBSCAN* core distances and node core-distance ranges, and the waiting and
// queued pairs (16 bytes each) that the frontier, far and queue lists hold at
// their peak.  The pair count per point grows steeply with d (measured peaks
// on uniform inputs with growth headroom: about 1,600 at d = 7 against 64 at
// d = 3).
size_t request_footprint(int64_t n, int d, int min_pts) {
    static const size_t kListPairs[8] = {0, 24, 24, 64, 100, 200, 600, 1600};
    size_t node = d <= 3 ? 64 : 128;
    return (size_t)n * (720 + 2 * node + 16 * (size_t)d + (min_pts > 0 ? 640 : 0) + 16 * kListPairs[d]);
}

struct Server {
    int device = 0;
    size_t budget = 0, cap_per_worker = 0;
    int max_req = 0;
    int64_t max_pts = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> lane[2];  // 0: small requests (batched), 1: large requests (one at a time)
    int64_t small_max = 0;         // requests with n <= this go to the small lane
    std::unordered_map<uint64_t, Request*> all;
    std::unordered_set<uint64_t> withdrawn;  // cancelled tickets not yet reported by a wait
    std::vector<std::thread> workers;
    std::vector<std::unique_ptr<Device>> ws;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::atomic<int> want_release{0};  // workers solving a request alone that needs the others' memory
    geomst_server_stats_t st{};
};

// Releases a worker's workspace (waits for its queued work first).
void release_workspace(Device& D) {
    if (D.own) (void)hipStreamSynchronize(D.own);
    D.~Device();
    new (&D) Device();
}

// Solves a taken batch as forests of equal dimension and kind (EMST or
// HDBSCAN*), so that no instance pays for padded coordinates or for the
// other kind's separation test; the groups run in the order of their oldest
// request; each group's requests are done as soon as the group is.
void run_batch(Server* S, Device& D, std::vector<Request*>& batch) {
    std::vector<std::vector<Request*>> groups;
    std::vector<int> gkey;
    for (Request* r : batch) {
        int k = r->item.d * 2 + (r->item.min_pts > 0);
        size_t gi = std::find(gkey.begin(), gkey.end(), k) - gkey.begin();
        if (gi == gkey.size()) {
            gkey.push_back(k);
            groups.emplace_back();
        }
        groups[gi].push_back(r);
    }
    for (auto& grp : groups) {
        std::vector<HostItem> it(grp.size());
        int64_t N = 0;
        for (size_t i = 0; i < grp.size(); ++i) {
            it[i] = grp[i]->item;
            N += it[i].n;
        }
        auto solve = [&](HostItem* items, int64_t count, size_t limit) -> int {
            g_err.clear();
            D.budget.limit = limit;
            g_ws_budget = &D.budget;
            struct Reset {
                ~Reset() { g_ws_budget = nullptr; }
            } reset;
            try {
                ensure_init(D);
                solve_host_items(D, items, count);
            } catch (const Fail& f) {
                return f.code;
            } catch (const std::bad_alloc&) {
                return GEOMST_ENOMEM;
            } catch (...) {
                g_err = "unexpected exception in a server worker";
                return GEOMST_EINTERNAL;
            }
            return GEOMST_OK;
        };
        std::vector<int> status(grp.size(),
                                solve(it.data(), (int64_t)it.size(), (size_t)((double)S->cap_per_worker * g_share_scale)));
        std::vector<std::string> err(grp.size(), g_err);
        if (status[0] == GEOMST_ENOMEM) {
            // The workspace outgrew the device (the admission estimate does
            // not cover the pair lists of high-dimensional inputs): release
            // it and solve the requests one at a time.
            release_workspace(D);  // nothing of the failed solve may still run
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->st.enomem_batches += 1;
            }
            auto others_hold = [&] {
                size_t o = 0;
                for (auto& w : S->ws)
                    if (w.get() != &D) o += w->budget.held.load(std::memory_order_relaxed);
                return o;
            };
            for (size_t i = 0; i < grp.size(); ++i) {
                // one request may use the whole budget less what the other
                // workers hold now; when that is not enough it is solved
                // alone in whatever device memory is free (the budget is a
                // soft admission limit; such solves count in
                // enomem_batches); if the device itself runs out, the other
                // workers are asked to release their workspaces after their
                // current batch (idle ones at once), this worker releases its
                // own, and the request is solved again once they have (or
                // after two minutes) with what is then free
                size_t others = others_hold();
                status[i] = solve(&it[i], 1, S->budget > others ? S->budget - others : 0);
                err[i] = g_err;
                if (status[i] == GEOMST_ENOMEM) {
                    status[i] = solve(&it[i], 1, ~(size_t)0);
                    err[i] = g_err;
                }
                bool asked = false;
                for (int attempt = 0; attempt < 8 && status[i] == GEOMST_ENOMEM; ++attempt) {
                    if (asked && others == 0) break;
                    if (!asked) {
                        asked = true;
                        S->want_release.fetch_add(1);
                        std::lock_guard<std::mutex> lk(S->mu);
                        S->cv_work.notify_all();
                    }
                    release_workspace(D);
                    const auto t0 = Clock::now();
                    while (others_hold() != 0 && Clock::now() - t0 < std::chrono::seconds(120))
                        std::this_thread::sleep_for(std::chrono::milliseconds(20));
                    others = others_hold();
                    status[i] = solve(&it[i], 1, S->budget > others ? S->budget - others : ~(size_t)0);
                    err[i] = g_err;
                }
                if (asked) S->want_release.fetch_sub(1);
            }
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            auto now = Clock::now();
            for (size_t i = 0; i < grp.size(); ++i) {
                Request* r = grp[i];
                r->status = status[i];
                if (status[i]) r->err = err[i].empty() ? "batch failed" : err[i];
                r->batch_requests = (int)grp.size();
                r->batch_points = N;
                r->done = true;
                r->t_done = now;
            }
            S->st.running -= (int64_t)grp.size();
            S->st.completed += (int64_t)grp.size();
        }
        S->cv_done.notify_all();
    }
}

// Size-class lanes: small requests are solved as forests (one launch
// sequence for many instances, which is what pays for them), large ones one
// at a time, since a forest is only as fast as its slowest member and large
// instances already fill the device.  With several workers, worker 0 prefers
// the small lane and the others the large lane; each takes from the other
// lane when its own is empty, so no worker idles while requests wait.  A
// single worker takes the requests in arrival order.
void worker_loop(Server* S, int wi) {
    (void)hipSetDevice(S->device);
    Device& D = *S->ws[wi];
    const bool single = S->ws.size() == 1;
    const int pref = wi == 0 ? 0 : 1;
    while (true) {
        std::vector<Request*> batch;
        size_t fp = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            const auto release_asked = [&] {
                return S->want_release.load() > 0 && D.budget.held.load(std::memory_order_relaxed) > 0;
            };
            S->cv_work.wait(lk, [&] {
                return S->stop || !S->lane[0].empty() || !S->lane[1].empty() || release_asked();
            });
            if (S->stop) break;
            if (S->lane[0].empty() && S->lane[1].empty()) {  // woken only to let go of the workspace
                lk.unlock();
                release_workspace(D);
                continue;
            }
            int ln;
            if (S->lane[0].empty()) ln = 1;
            else if (S->lane[1].empty()) ln = 0;
            else if (single) ln = S->lane[0].front()->ticket < S->lane[1].front()->ticket ? 0 : 1;
            else ln = pref;
            std::deque<Request*>& q = S->lane[ln];
            const int max_req = ln == 0 ? S->max_req : 1;
            int64_t pts = 0;
            auto now = Clock::now();
            while (!q.empty()) {
                Request* r = q.front();
                bool fits = fp + r->footprint <= S->cap_per_worker && (int)batch.size() < max_req &&
                            pts + r->item.n <= S->max_pts;
                if (!batch.empty() && !fits) break;  // the first request always fits (checked at submit)
                q.pop_front();
                r->started = true;
                r->t_start = now;
                batch.push_back(r);
                fp += r->footprint;
                pts += r->item.n;
            }
            S->st.queued -= (int64_t)batch.size();
            S->st.running += (int64_t)batch.size();
            S->st.batches += 1;
            S->st.reserved_bytes += (int64_t)fp;
            S->st.peak_reserved_bytes = std::max(S->st.peak_reserved_bytes, S->st.reserved_bytes);
            S->st.max_batch_requests = std::max<int64_t>(S->st.max_batch_requests, (int64_t)batch.size());
            S->st.max_batch_points = std::max(S->st.max_batch_points, pts);
        }
        if (!batch.empty()) {
            run_batch(S, D, batch);
            // another worker solving a request alone ran out of device
            // memory: let go of this workspace (a grown workspace is
            // otherwise kept: regrowing it costs list restarts)
            if (S->want_release.load() > 0) release_workspace(D);
        }
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.reserved_bytes -= (int64_t)fp;
    }
}

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace
}  // namespace geomst

using namespace geomst;

struct geomst_server : Server {};

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

int geomst_dendrogram_dev(const int64_t* d_edges, const double* d_weights, int64_t n, int64_t start,
                          int64_t* d_children, int64_t* d_size, int64_t* d_order, double* d_reach, void* stream) {
    g_err.clear();
    int rc = validate_dendro(d_edges, d_weights, n, start, d_order, d_reach);
    if (rc) return rc;
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        dendrogram_dev(D, (hipStream_t)stream, (const long long*)d_edges, d_weights, (int)n, (int)start,
                       (long long*)d_children, (long long*)d_size, (long long*)d_order, d_reach);
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int geomst_dendrogram(const int64_t* edges, const double* weights, int64_t n, int64_t start, int64_t* children,
                      int64_t* size, int64_t* order, double* reach) {
    g_err.clear();
    int rc = validate_dendro(edges, weights, n, start, order, reach);
    if (rc) return rc;
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        hipStream_t s = D.own;
        const size_t m = (size_t)(n - 1);
        // staging: edges and children share one buffer, weights / reach and
        // sizes / order the others
        D.pin.ensure(std::max<size_t>(m * 16, 16));
        D.wout.ensure(std::max<size_t>(m * 8, (size_t)n * 8));
        D.eout.ensure(std::max<size_t>(m * 16, 16) + (size_t)n * 8 + m * 8);
        long long* de = D.pin.as<long long>();
        double* dw = D.wout.as<double>();
        long long* dch = D.eout.as<long long>();
        long long* dorder = dch + 2 * m;
        long long* dsize = dorder + n;
        D.cdout.ensure((size_t)n * 8);
        double* dreach = D.cdout.as<double>();
        if (m) {
            HIPCHK(hipMemcpyAsync(de, edges, m * 16, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(dw, weights, m * 8, hipMemcpyHostToDevice, s));
        }
        dendrogram_dev(D, s, de, dw, (int)n, (int)start, children ? dch : nullptr, size ? dsize : nullptr, dorder,
                       dreach);
        if (m && children) HIPCHK(hipMemcpyAsync(children, dch, m * 16, hipMemcpyDeviceToHost, s));
        if (m && size) HIPCHK(hipMemcpyAsync(size, dsize, m * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(order, dorder, (size_t)n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(reach, dreach, (size_t)n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int geomst_emst_dev_noalloc(const double* d_points, int64_t n, int32_t d, int64_t* d_edges, double* d_weights,
                            double* d_weights_sq, void* stream) {
    return run_dev_noalloc(d_points, n, d, (long long*)d_edges, d_weights, d_weights_sq, stream);
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

namespace {
int check_approx(int32_t min_pts, double rho) {
    if (min_pts < 1) {
        g_err = "min_pts must be >= 1";
        return GEOMST_EINVAL;
    }
    if (!(rho > 0.0) || !(rho < 1e300)) {
        g_err = "rho must be positive and finite";
        return GEOMST_EINVAL;
    }
    return GEOMST_OK;
}
}  // namespace

int geomst_optics_approx_dev(const double* d_points, int64_t n, int32_t d, int32_t min_pts, double rho,
                             double* d_core_dist, double* d_core_dist_sq, int64_t* d_edges, double* d_weights,
                             double* d_weights_sq, void* stream) {
    g_err.clear();
    int rc = check_approx(min_pts, rho);
    if (rc) return rc;
    return run_dev(d_points, n, d, min_pts, (long long*)d_edges, d_weights, d_weights_sq, d_core_dist,
                   d_core_dist_sq, stream, rho);
}

int geomst_optics_approx(const double* points, int64_t n, int32_t d, int32_t min_pts, double rho,
                         double* core_dist, int64_t* edges, double* weights) {
    g_err.clear();
    int rc = check_approx(min_pts, rho);
    if (rc) return rc;
    return run_host(points, n, d, min_pts, edges, weights, core_dist, rho);
}

int geomst_batch_dev(const double* d_points, int32_t stride, const geomst_batch_item_t* items, int64_t count,
                     int64_t* d_edges, double* d_weights, double* d_weights_sq, double* d_core_dist,
                     double* d_core_dist_sq, void* stream) {
    g_err.clear();
    if (!d_points) {
        g_err = "points is NULL";
        return GEOMST_EINVAL;
    }
    int rc = validate_batch(stride, items, count);
    if (rc) return rc;
    int64_t N = items[count - 1].offset + items[count - 1].n;
    if (N > count && !d_edges) {
        g_err = "edges is NULL";
        return GEOMST_EINVAL;
    }
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        solve_batch_dev(D, (hipStream_t)stream, d_points, stride, items, count, (long long*)d_edges, d_weights,
                        d_weights_sq, d_core_dist, d_core_dist_sq);
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int geomst_batch(geomst_instance_t* inst, int64_t count) {
    g_err.clear();
    if (!inst || count < 1) {
        g_err = "inst is NULL or count < 1";
        return GEOMST_EINVAL;
    }
    std::vector<HostItem> it((size_t)count);
    int bad = 0;
    for (int64_t i = 0; i < count; ++i) {
        geomst_instance_t& q = inst[i];
        it[i] = HostItem{q.points, q.n, q.d, q.min_pts, q.edges, q.weights, q.core_dist};
        q.status = check_host_item(it[i]);
        bad += q.status != GEOMST_OK;
    }
    if (bad) {
        g_err = "invalid batch items (see their status)";
        for (int64_t i = 0; i < count; ++i)
            if (inst[i].status == GEOMST_EDOM) return GEOMST_EDOM;
        return GEOMST_EINVAL;
    }
    try {
        int dev;
        Device& D = device_ctx(&dev);
        std::lock_guard<std::mutex> lk(D.mu);
        ensure_init(D);
        solve_host_items(D, it.data(), count);
    } catch (const Fail& f) {
        for (int64_t i = 0; i < count; ++i) inst[i].status = f.code;
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int geomst_server_create(const geomst_server_cfg_t* cfg, geomst_server_t** out) {
    g_err.clear();
    if (!out) {
        g_err = "out is NULL";
        return GEOMST_EINVAL;
    }
    *out = nullptr;
    geomst_server_cfg_t c{};
    if (cfg) c = *cfg;
    if (c.workers < 0 || c.workers > 16 || c.max_batch_requests < 0 || c.small_max_points < 0 || c.max_batch_points < 0 ||
        c.max_batch_points > (1ll << 26) || c.device < -1 || c.device >= 16) {
        g_err = "bad server configuration";
        return GEOMST_EINVAL;
    }
    int dev = c.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        g_err = "no current HIP device";
        return GEOMST_EDEVICE;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) {
        g_err = "device index out of range";
        return GEOMST_EDEVICE;
    }
    try {
        std::unique_ptr<geomst_server> S(new geomst_server());
        S->device = dev;
        int w = c.workers ? c.workers : 2;
        S->small_max = c.small_max_points ? c.small_max_points : 32768;
        if (c.tuning_cache) {
            int trc = geomst_load_tuning(c.tuning_cache);
            if (trc) return trc;
        }
        S->budget = c.hbm_budget_bytes ? (size_t)c.hbm_budget_bytes : (size_t)200e9;
        S->cap_per_worker = S->budget / (size_t)w;
        S->max_req = c.max_batch_requests ? c.max_batch_requests : 4096;
        S->max_pts = c.max_batch_points ? c.max_batch_points : (1ll << 20);
        for (int i = 0; i < w; ++i) S->ws.emplace_back(new Device());
        for (int i = 0; i < w; ++i) S->workers.emplace_back(worker_loop, S.get(), i);
        *out = S.release();
    } catch (const std::exception& e) {
        g_err = std::string("server start failed: ") + e.what();
        return GEOMST_ENOMEM;
    }
    return GEOMST_OK;
}

int geomst_submit(geomst_server_t* srv, geomst_instance_t* req, uint64_t* ticket) {
    g_err.clear();
    if (!srv || !req || !ticket) {
        g_err = "srv, req or ticket is NULL";
        return GEOMST_EINVAL;
    }
    HostItem it{req->points, req->n, req->d, req->min_pts, req->edges, req->weights, req->core_dist};
    int rc = check_host_item(it);
    if (rc) {
        g_err = rc == GEOMST_EDOM ? "a coordinate is not finite or exceeds 2^500 in magnitude"
                                  : "invalid request (n, d, min_pts or a NULL pointer)";
        req->status = rc;
        return rc;
    }
    size_t fp = request_footprint(it.n, it.d, it.min_pts);
    if (fp > srv->cap_per_worker || (it.n <= srv->small_max && it.n > srv->max_pts)) {
        g_err = "request exceeds a worker's share of the memory budget or the batch point limit";
        req->status = GEOMST_ENOMEM;
        return GEOMST_ENOMEM;
    }
    try {
        std::unique_ptr<Request> r(new Request());
        r->pts.assign(it.points, it.points + it.n * it.d);
        r->item = it;
        r->item.points = r->pts.data();
        r->footprint = fp;
        r->t_arrive = Clock::now();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->stop) {
                g_err = "server is stopping";
                return GEOMST_EINVAL;
            }
            r->ticket = srv->next_ticket++;
            *ticket = r->ticket;
            srv->all[r->ticket] = r.get();
            // forests pay for small EMST requests; HDBSCAN* forests that mix
            // minPts values and densities ran slower than their members
            // solved one by one, so HDBSCAN* requests take the large lane
            r->lane = (it.n <= srv->small_max && it.min_pts == 0) ? 0 : 1;
            srv->lane[r->lane].push_back(r.get());
            srv->st.submitted += 1;
            srv->st.queued += 1;
            r.release();
        }
        srv->cv_work.notify_one();
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        req->status = GEOMST_ENOMEM;
        return GEOMST_ENOMEM;
    }
    req->status = GEOMST_OK;
    return GEOMST_OK;
}

int geomst_wait(geomst_server_t* srv, uint64_t ticket, int64_t timeout_us, geomst_request_info_t* info) {
    g_err.clear();
    if (!srv) {
        g_err = "srv is NULL";
        return GEOMST_EINVAL;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    // the ticket is looked up again after every wake-up: another thread's
    // wait or cancel may have released it meanwhile
    auto ready = [&] {
        auto f = srv->all.find(ticket);
        return f == srv->all.end() || f->second->done;
    };
    if (timeout_us < 0)
        srv->cv_done.wait(lk, ready);
    else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return GEOMST_ETIMEDOUT;
    auto f = srv->all.find(ticket);
    if (f == srv->all.end()) {
        if (srv->withdrawn.erase(ticket)) {
            g_err = "the request was cancelled";
            return GEOMST_ECANCELED;
        }
        g_err = "unknown ticket";
        return GEOMST_ENOENT;
    }
    Request* r = f->second;
    srv->all.erase(f);
    lk.unlock();
    int rc = r->status;
    if (info) {
        info->status = rc;
        info->batch_requests = r->batch_requests;
        info->batch_points = r->batch_points;
        info->queue_ms = ms_between(r->t_arrive, r->t_start);
        info->service_ms = ms_between(r->t_start, r->t_done);
        info->latency_ms = ms_between(r->t_arrive, r->t_done);
    }
    if (rc) g_err = r->err;
    delete r;
    srv->cv_done.notify_all();  // wake other waiters of this ticket
    return rc;
}

int geomst_cancel(geomst_server_t* srv, uint64_t ticket) {
    g_err.clear();
    if (!srv) {
        g_err = "srv is NULL";
        return GEOMST_EINVAL;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] {
        auto f = srv->all.find(ticket);
        return f == srv->all.end() || !f->second->started || f->second->done;
    });
    auto f = srv->all.find(ticket);
    if (f == srv->all.end()) {
        g_err = "unknown ticket";
        return GEOMST_ENOENT;
    }
    Request* r = f->second;
    if (!r->started) {
        auto& q = srv->lane[r->lane];
        q.erase(std::find(q.begin(), q.end(), r));
        srv->st.queued -= 1;
    }
    srv->all.erase(f);
    srv->withdrawn.insert(ticket);
    lk.unlock();
    delete r;
    srv->cv_done.notify_all();
    return GEOMST_OK;
}

int geomst_server_stats(geomst_server_t* srv, geomst_server_stats_t* out) {
    if (!srv || !out) return GEOMST_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    out->workspace_bytes = 0;
    for (auto& w : srv->ws) out->workspace_bytes += (int64_t)w->budget.held.load(std::memory_order_relaxed);
    return GEOMST_OK;
}

void geomst_server_destroy(geomst_server_t* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->lane[0].clear();
        srv->lane[1].clear();
    }
    srv->cv_work.notify_all();
    for (auto& t : srv->workers) t.join();
    for (auto& kv : srv->all) delete kv.second;
    int cur = 0;
    bool have = hipGetDevice(&cur) == hipSuccess;
    (void)hipSetDevice(srv->device);
    srv->ws.clear();
    if (have) (void)hipSetDevice(cur);
    delete srv;
}

int geomst_get_stats(geomst_stats_t* out) {
    if (!out) return GEOMST_EINVAL;
    *out = g_stats;
    return GEOMST_OK;
}

int geomst_set_option(const char* name, double value) {
    if (!name) return GEOMST_EINVAL;
    std::lock_guard<std::mutex> lk(g_opt_mu);
    if (!strcmp(name, "beta_growth")) {
        if (value != 0.0 && (!(value > 1.0) || !(value < 1e6))) return GEOMST_EINVAL;
        g_beta_growth = value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "refresh_divisor")) {
        if (!(value >= 1.0) || !(value <= 1048576.0) || value != (double)(u32)value) return GEOMST_EINVAL;
        g_refresh_div = (u32)value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "small_level_switch") || !strcmp(name, "small_level_max")) {
        if (!(value >= 0.0) || !(value <= 1048576.0) || value != (double)(u32)value) return GEOMST_EINVAL;
        (name[12] == 's' ? g_small_switch : g_small_max) = (u32)value;
        if (g_small_max < g_small_switch) g_small_max = g_small_switch;
        return GEOMST_OK;
    }
    if (!strcmp(name, "wide_level_switch") || !strcmp(name, "wide_level_max")) {
        if (!(value >= 0.0) || !(value <= 65536.0) || value != (double)(u32)value) return GEOMST_EINVAL;
        (name[11] == 's' ? g_wide_switch : g_wide_max) = (u32)value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "bccp_chunk")) {
        if (value == 0.0) value = kBigBDefault;
        if (!(value >= 64.0) || !(value <= 65536.0) || value != (double)(64 * (int)(value / 64.0))) return GEOMST_EINVAL;
        g_bccp_chunk = (int)value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "schedule")) {
        if (value != 0.0 && value != 1.0 && value != 2.0 && value != 3.0) return GEOMST_EINVAL;
        g_sched = (int)value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "separation_mode")) {
        if (value != 0.0 && value != 1.0) return GEOMST_EINVAL;
        g_sep_mode = (int)value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "separation")) {
        if (!(value >= 0.0) || !(value <= 16.0)) return GEOMST_EINVAL;
        g_separation = value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "beta_start_quantile")) {
        if (!(value >= 0.0 && value <= 1.0)) return GEOMST_EINVAL;
        g_beta_start = value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "server_share_scale")) {
        if (!(value > 0.0) || !(value <= 1.0)) return GEOMST_EINVAL;
        g_share_scale = value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "beta_schedule")) {
        if (value != 0.0 && value != 1.0) return GEOMST_EINVAL;
        g_beta_plain = value != 0.0;
        return GEOMST_OK;
    }
    if (!strcmp(name, "list_capacity_scale")) {
        if (!(value > 0.0) || !(value <= 1.0)) return GEOMST_EINVAL;
        g_capacity_scale = value;
        return GEOMST_OK;
    }
    if (!strcmp(name, "kernel_timing")) {
        if (value != 0.0 && value != 1.0) return GEOMST_EINVAL;
        g_kernel_timing = value != 0.0 ? 0xffffffffu : 0u;
        return GEOMST_OK;
    }
    if (!strcmp(name, "kernel_timing_families")) {
        if (!(value >= 0.0) || !(value < (double)(1u << GEOMST_K_COUNT)) || value != (double)(u32)value)
            return GEOMST_EINVAL;
        g_kernel_timing_families = value == 0.0 ? 0xffffffffu : (u32)value;
        return GEOMST_OK;
    }
    return GEOMST_EINVAL;
}

int geomst_load_tuning(const char* path) {
    g_err.clear();
    if (!path) {
        std::lock_guard<std::mutex> lk(g_opt_mu);
        g_tuning.clear();
        return GEOMST_OK;
    }
    FILE* fh = fopen(path, "r");
    if (!fh) {
        g_err = std::string("cannot open tuning cache ") + path;
        return GEOMST_ENOENT;
    }
    std::vector<TuneEntry> table;
    char line[4096];
    int lineno = 0;
    int rc = GEOMST_OK;
    while (rc == GEOMST_OK && fgets(line, sizeof line, fh)) {
        ++lineno;
        if (!parse_tune_line(line, table)) {
            g_err = std::string("tuning cache ") + path + ": bad entry on line " + std::to_string(lineno);
            rc = GEOMST_EINVAL;
        }
    }
    fclose(fh);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_opt_mu);
    g_tuning.swap(table);
    return GEOMST_OK;
}

const char* geomst_last_error(void) { return g_err.c_str(); }

int geomst_version(void) { return 100; }

}  // extern "C"
