// Device-side building blocks shared by the geomst kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace geomst {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int32_t i32;

constexpr int kWave = 64;
constexpr u32 kNone = 0xffffffffu;
constexpr int kMaxDim = 7;

// Positive doubles (and +0) order like their bit patterns as unsigned ints.
__device__ __forceinline__ u64 dbits(double x) { return (u64)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(u64 b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ u64 lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Wave-aggregated append: every active lane calls it; lanes with pred get a
// distinct slot base+k (k = rank among predicated lanes), others get kNone.
__device__ __forceinline__ u32 wave_append(u32* counter, bool pred) {
    u64 mask = __ballot(pred);
    if (mask == 0) return kNone;
    int leader = __ffsll((long long)mask) - 1;
    u32 base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (u32)__popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + (u32)__popcll(mask & lanemask_lt()) : kNone;
}

// A value known to be equal in every active lane, moved to scalar registers.
__device__ __forceinline__ double wave_uniform_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Wave-wide minimum of a u64 (all 64 lanes must be active).
__device__ __forceinline__ u64 wave_min_u64(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u64 w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double w = __shfl_xor(v, o);
        v = fmin(w, v);
    }
    return v;
}

// atomic minimum of a non-negative double through its bit pattern
__device__ __forceinline__ void atomic_min_pos_f64(u64* addr, double v) {
    atomicMin((unsigned long long*)addr, (unsigned long long)dbits(v));
}

// Edge key K = (w2, e2, lo, hi) compared lexicographically; lo < hi are the
// caller's row indices.  For EMST w2 == e2.
struct EKey {
    double w2, e2;
    u32 lo, hi;
};

__device__ __forceinline__ bool key_less(const EKey& a, const EKey& b) {
    if (a.w2 != b.w2) return a.w2 < b.w2;
    if (a.e2 != b.e2) return a.e2 < b.e2;
    if (a.lo != b.lo) return a.lo < b.lo;
    return a.hi < b.hi;
}

__device__ __forceinline__ EKey key_none() {
    EKey k;
    k.w2 = __longlong_as_double(0x7ff0000000000000ll);  // +inf
    k.e2 = k.w2;
    k.lo = kNone;
    k.hi = kNone;
    return k;
}

__device__ __forceinline__ EKey shfl_key(const EKey& k, int src) {
    EKey r;
    r.w2 = __shfl(k.w2, src);
    r.e2 = __shfl(k.e2, src);
    r.lo = __shfl(k.lo, src);
    r.hi = __shfl(k.hi, src);
    return r;
}

__device__ __forceinline__ EKey wave_min_key(EKey k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        EKey w;
        w.w2 = __shfl_xor(k.w2, o);
        w.e2 = __shfl_xor(k.e2, o);
        w.lo = __shfl_xor(k.lo, o);
        w.hi = __shfl_xor(k.hi, o);
        if (key_less(w, k)) k = w;
    }
    return k;
}

}  // namespace geomst
