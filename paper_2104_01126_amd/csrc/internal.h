// Internal interface between the geomst orchestration and its generic
// primitives (scan, radix sort) which live in their own translation unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace geomst {

typedef uint64_t u64;
typedef uint32_t u32;

// Scratch bytes needed by the scans / sorts below for `count` elements.
size_t scan_temp_bytes(size_t count);
size_t radix_temp_bytes(size_t count);

void scan_exclusive_u32(const u32* in, u32* out, size_t count, void* temp, hipStream_t s);
void scan_inclusive_u32(const u32* in, u32* out, size_t count, void* temp, hipStream_t s);

// Stable LSD sort of (key, val) pairs on key bits [lo_bit, bits) (keys equal
// in those bits keep their input order), every bit position moved up by the
// device word *dshift when dshift is not null (0 <= *dshift <= 64 - bits).
// Ping-pongs between (key, val) and (key2, val2); returns 1 when the sorted
// result ends in (key2, val2) and 0 when it ends in (key, val).
int radix_sort_pairs(u64* key, u32* val, u64* key2, u32* val2, size_t count, int bits, void* temp,
                     hipStream_t s, int lo_bit = 0, const int* dshift = nullptr);


}  // namespace geomst
