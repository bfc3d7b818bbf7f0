// Generic device primitives: prefix sums and stable LSD radix sorts (gfx950).
//
// The radix sort is the classic three-step pass (per-tile digit histograms,
// an exclusive scan of the digit-major histogram table, a stable scatter),
// three launches per 8-bit digit.
// Stability inside a tile comes from processing the tile in (iteration,
// wave, lane) order, which is the element order, and ranking equal digits
// inside a wave with ballots; the scatter stages the ranked tile in LDS and
// writes each digit's run with coalesced stores.
#include <hip/hip_runtime.h>
#include "internal.h"
#include "common.h"

namespace geomst {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // 2048 elements per block
constexpr int kWaves = kThreads / kWave;

inline size_t cdiv(size_t a, size_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- scan
__device__ __forceinline__ u32 wave_incl_scan(u32 v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        u32 t = __shfl_up(v, o);
        if (lane_id() >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ u32 block_excl_scan(u32 v, u32* total) {
    __shared__ u32 wsum[kWaves];
    u32 inc = wave_incl_scan(v);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = inc;
    __syncthreads();
    u32 off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        u32 s = wsum[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const u32* in, u32* sums, size_t count) {
    size_t base = (size_t)blockIdx.x * kTile;
    u32 s = 0;
    for (int it = 0; it < kItems; ++it) {
        size_t e = base + (size_t)it * kThreads + threadIdx.x;
        if (e < count) s += in[e];
    }
    u32 tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scan each tile with its block offset; thread t owns elements t*kItems..+kItems.
__global__ void __launch_bounds__(kThreads) k_scan_apply(const u32* in, u32* out, const u32* offs, size_t count,
                                                         int inclusive) {
    size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kItems;
    u32 v[kItems];
    u32 s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (base + i < count) ? in[base + i] : 0u;
        s += v[i];
    }
    u32 tot;
    u32 run = block_excl_scan(s, &tot) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        u32 x = v[i];
        if (base + i < count) out[base + i] = inclusive ? run + x : run;
        run += x;
    }
}

void scan_impl(const u32* in, u32* out, size_t count, u32* temp, int inclusive, hipStream_t s) {
    if (count == 0) return;
    size_t nb = cdiv(count, kTile);
    if (nb == 1) {
        k_scan_apply<<<1, kThreads, 0, s>>>(in, out, nullptr, count, inclusive);
        return;
    }
    u32* sums = temp;
    u32* rest = temp + cdiv(nb, 64) * 64;
    k_scan_reduce<<<(unsigned)nb, kThreads, 0, s>>>(in, sums, count);
    scan_impl(sums, sums, nb, rest, 0, s);
    k_scan_apply<<<(unsigned)nb, kThreads, 0, s>>>(in, out, sums, count, inclusive);
}

// ---------------------------------------------------------------- radix
struct PairKeys {
    const u64* key;
    __device__ __forceinline__ u32 digit(size_t e, int shift) const { return (u32)(key[e] >> shift) & 255u; }
};
// Per-tile digit counts into the digit-major table.
template <class K>
__global__ void __launch_bounds__(kThreads) k_radix_hist(K keys, size_t count, int shift, const int* dshift, u32* hist,
                                                         u32 nblocks) {
    __shared__ u32 h[256];
    if (dshift) shift += *dshift;
    h[threadIdx.x] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * kTile;
    for (int it = 0; it < kItems; ++it) {
        size_t e = base + (size_t)it * kThreads + threadIdx.x;
        if (e < count) atomicAdd(&h[keys.digit(e, shift)], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Block d scans row d of the table (digit d's per-tile counts) in place and
// stores the digit's total; the scatter adds the totals of the smaller digits.
// One launch and no atomics.
__global__ void __launch_bounds__(kThreads) k_radix_rowscan(u32* hist, u32 nblocks, u32* totals) {
    const u32 d = blockIdx.x;
    u32 run = 0;
    u32* row = hist + (size_t)d * nblocks;
    for (u32 c0 = 0; c0 < nblocks; c0 += kTile) {
        const u32 b = c0 + threadIdx.x * kItems;
        u32 v[kItems];
        u32 sum = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            v[i] = b + i < nblocks ? row[b + i] : 0u;
            sum += v[i];
        }
        u32 tot;
        u32 off = run + block_excl_scan(sum, &tot);
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            if (b + i < nblocks) row[b + i] = off;
            off += v[i];
        }
        run += tot;
    }
    if (threadIdx.x == 0) totals[d] = run;
}

// Key-value scatter through LDS: the tile is first ranked into digit order in
// LDS (stable, as above), then written out so that consecutive threads write
// consecutive slots of one digit's run: coalesced stores instead of one
// scattered store per element.
__global__ void __launch_bounds__(kThreads) k_radix_scatter_lds(const u64* ki, const u32* vi, u64* ko, u32* vo,
                                                                size_t count, int shift, const int* dshift,
                                                                const u32* offs, u32 nblocks, const u32* totals) {
    if (dshift) shift += *dshift;
    __shared__ u64 sk[kTile];
    __shared__ u32 sv[kTile];
    __shared__ u32 lstart[256], gbase[256], run[256];
    __shared__ u32 wcnt[kWaves][256];
    const int t = threadIdx.x;
    const int w = t / kWave;
    const size_t base = (size_t)blockIdx.x * kTile;
    const u32 ntile = (u32)((count - base) < (size_t)kTile ? (count - base) : (size_t)kTile);
    u64 key[kItems];
    u32 val[kItems], dg[kItems];
    run[t] = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) wcnt[i][t] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const u32 le = (u32)it * kThreads + t;
        key[it] = 0;
        val[it] = 0;
        if (le < ntile) {
            key[it] = ki[base + le];
            val[it] = vi[base + le];
            atomicAdd(&run[(u32)(key[it] >> shift) & 255u], 1u);
        }
        dg[it] = (u32)(key[it] >> shift) & 255u;
    }
    __syncthreads();
    u32 tot;
    const u32 ex = block_excl_scan(run[t], &tot);
    const u32 dbase = block_excl_scan(totals[t], &tot);  // elements of the smaller digits
    lstart[t] = ex;
    run[t] = ex;
    gbase[t] = dbase + offs[(size_t)t * nblocks + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const bool valid = (u32)it * kThreads + t < ntile;
        const u32 d = dg[it];
        const u64 vmask = __ballot(valid);
        u64 peers = valid ? vmask : ~vmask;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const u64 bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const u32 rank = (u32)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = (u32)__popcll(peers);
        __syncthreads();
        if (valid) {
            u32 pos = run[d] + rank;
            for (int i = 0; i < w; ++i) pos += wcnt[i][d];
            sk[pos] = key[it];
            sv[pos] = val[it];
        }
        __syncthreads();
        u32 add = 0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) {
            add += wcnt[i][t];
            wcnt[i][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
    for (u32 j = t; j < ntile; j += kThreads) {
        const u64 k = sk[j];
        const u32 d = (u32)(k >> shift) & 255u;
        const size_t gp = (size_t)gbase[d] + (j - lstart[d]);
        ko[gp] = k;
        vo[gp] = sv[j];
    }
}

}  // namespace

size_t scan_temp_bytes(size_t count) {
    size_t tot = 0;
    size_t c = count;
    while (c > (size_t)kTile) {
        c = cdiv(c, kTile);
        tot += cdiv(c, 64) * 64;
    }
    return (tot + 64) * sizeof(u32);
}

size_t radix_temp_bytes(size_t count) {
    size_t nb = cdiv(count ? count : 1, kTile);
    size_t h = nb * 256;
    return (cdiv(h, 64) * 64 + 256) * sizeof(u32);
}

void scan_exclusive_u32(const u32* in, u32* out, size_t count, void* temp, hipStream_t s) {
    scan_impl(in, out, count, (u32*)temp, 0, s);
}
void scan_inclusive_u32(const u32* in, u32* out, size_t count, void* temp, hipStream_t s) {
    scan_impl(in, out, count, (u32*)temp, 1, s);
}

int radix_sort_pairs(u64* key, u32* val, u64* key2, u32* val2, size_t count, int bits, void* temp,
                     hipStream_t s, int lo_bit, const int* dshift) {
    bits = std::min(bits, 64);
    if (count <= 1 || bits <= lo_bit) return 0;
    u32 nb = (u32)cdiv(count, kTile);
    u32* hist = (u32*)temp;
    u32* totals = hist + cdiv((size_t)nb * 256, 64) * 64;  // 256 digit totals
    const int passes = (bits - lo_bit + 7) / 8;
    int flip = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = lo_bit + 8 * p;
        u64* ki = flip ? key2 : key;
        u32* vi = flip ? val2 : val;
        u64* ko = flip ? key : key2;
        u32* vo = flip ? val : val2;
        PairKeys K{ki};
        k_radix_hist<<<nb, kThreads, 0, s>>>(K, count, shift, dshift, hist, nb);
        k_radix_rowscan<<<256, kThreads, 0, s>>>(hist, nb, totals);
        k_radix_scatter_lds<<<nb, kThreads, 0, s>>>(ki, vi, ko, vo, count, shift, dshift, hist, nb, totals);
        flip ^= 1;
    }
    return flip;
}

}  // namespace geomst
