// Device helpers shared by the kernels of libdbg (internal header).
#pragma once

#include "dbg_kernels.h"

namespace dbgk {


constexpr uint64_t kAllOnes = ~0ull;

// SplitMix64 output function (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): a bijective 64-bit mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

// Home slot in [0, cap): high 64 bits of h * cap (Lemire's multiply-shift
// range reduction, "Fast random integer generation in an interval", 2019).
__device__ __forceinline__ uint64_t home_slot(uint64_t h, uint64_t cap) {
    return __umul64hi(h, cap);
}

__device__ __forceinline__ bool valid_letter(uint32_t c) {
    const uint32_t lc = c | 0x20u;
    return lc == 'a' || lc == 'c' || lc == 'g' || lc == 't';
}

__device__ __forceinline__ uint32_t atomic_or_u32(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_add_u64(uint64_t *p, uint64_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Instance owning a global read index: the last i with read_begin <= r.
__device__ __forceinline__ uint32_t instance_of_read(const Instance *inst, uint32_t m, uint64_t r) {
    uint32_t lo = 0, hi = m;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (inst[mid].read_begin <= r) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t instance_of_byte(const Instance *inst, uint32_t m, uint64_t b) {
    uint32_t lo = 0, hi = m;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (inst[mid].byte_begin <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// The 32 bases starting at base position p, first base in bits 63..62.
__device__ __forceinline__ uint64_t bases_at(const uint64_t *__restrict__ packed, uint64_t p) {
    const uint64_t wi = p >> 5;
    const uint32_t sh = (uint32_t)(p & 31) * 2;
    const uint64_t hi = packed[wi];
    if (sh == 0) return hi;
    const uint64_t lo = packed[wi + 1];
    return (hi << sh) | (lo >> (64 - sh));
}

// 64 bases from base position p, first base in bits 63..62 of x0 (reads
// up to three words: the packed array has two words of padding).
__device__ __forceinline__ void bases128_at(const uint64_t *__restrict__ packed, uint64_t p,
                                            uint64_t &x0, uint64_t &x1) {
    const uint64_t wi = p >> 5;
    const uint32_t sh = (uint32_t)(p & 31) * 2;
    const uint64_t w0 = packed[wi], w1 = packed[wi + 1];
    if (sh == 0) {
        x0 = w0;
        x1 = w1;
        return;
    }
    const uint64_t w2 = packed[wi + 2];
    x0 = (w0 << sh) | (w1 >> (64 - sh));
    x1 = (w1 << sh) | (w2 >> (64 - sh));
}

// The (k-1)-mer K of a window of 32 < k <= 64 as (K >> 64, K mod 2^64), and
// the letter after it, from the window's 128 bits x0:x1.
__device__ __forceinline__ void wide_window(uint64_t x0, uint64_t x1, uint32_t km1, uint64_t &khi,
                                            uint64_t &klo, uint32_t &letter) {
    const uint32_t r = 128 - 2 * km1;  // 2 .. 64: the key ends r bits above x1's end
    klo = r == 64 ? x0 : (x1 >> r) | (x0 << (64 - r));
    khi = r == 64 ? 0 : x0 >> r;
    letter = (uint32_t)(x1 >> (r - 2)) & 3u;
}

__device__ __forceinline__ uint64_t wave_inclusive_scan(uint64_t v) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim <= 1024).
// Returns the exclusive prefix; *total receives the block sum.
__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t *total) {
    __shared__ uint64_t s_wave[16];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nwaves = (blockDim.x + 63) >> 6;
    const uint64_t inc = wave_inclusive_scan(v);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        uint64_t x = lane < nwaves ? s_wave[lane] : 0;
        x = wave_inclusive_scan(x);
        if (lane < nwaves) s_wave[lane] = x;
    }
    __syncthreads();
    const uint64_t before = wave ? s_wave[wave - 1] : 0;
    *total = s_wave[nwaves - 1];
    __syncthreads();
    return before + inc - v;
}


// ---------------------------------------------------------------- binned key images

// Binned tables and records hold a key's image under a bijection of the
// 60-bit key space (keys of k <= 31 have at most 60 bits): a multiply by an
// odd constant modulo 2^60, then an xorshift by 30, which undoes itself on 60
// bits.  A window's key is hashed once, in pass 1; everything after works on
// the image: the segment is a pair of mixed-radix digits of its top 32 bits
// (the level-1 bucket, then the segment inside the bucket), the home slot
// inside the segment is its low bits, and extraction maps it back.
constexpr uint64_t kKey60 = (1ull << 60) - 1;
constexpr uint64_t kKeyMul = 0x0E3779B97F4A7C15ull;  // odd; the golden-ratio constant's low 60 bits

constexpr uint64_t inverse_mod_2_64(uint64_t a) {  // Newton's iteration, 6 steps
    uint64_t x = a;
    for (int i = 0; i < 6; ++i) x *= 2 - a * x;
    return x;
}
constexpr uint64_t kKeyMulInv = inverse_mod_2_64(kKeyMul);
static_assert(kKeyMul * kKeyMulInv == 1, "inverse of the key multiplier");

__device__ __forceinline__ uint64_t key_image(uint64_t key) {
    const uint64_t x = (key * kKeyMul) & kKey60;
    return x ^ (x >> 30);
}

__device__ __forceinline__ uint64_t key_of_image(uint64_t x) {
    x ^= x >> 30;
    return (x * kKeyMulInv) & kKey60;
}

// Top 32 bits of an image: the digits of its segment.
__device__ __forceinline__ uint32_t image_top(uint64_t x) { return (uint32_t)(x >> 28); }

// Level-1 bucket of an image: the first digit, in [0, d1).
__device__ __forceinline__ uint32_t bucket_of(uint32_t top, uint32_t d1) { return __umulhi(top, d1); }

// Segment inside its bucket: the second digit, in [0, fan).
__device__ __forceinline__ uint32_t child_of(uint32_t top, uint32_t d1, uint32_t fan) {
    return __umulhi(top * d1, fan);
}

// A segment of a binned table is kSegSlots entries of EW words, stored as
// arrays: the image words (image | kOccupied) of its vertices, packed at
// [0, seg_count), then their four counters (16 bytes each); with 32-byte
// entries of short keys the last quarter is unused.  Each is written and read by
// consecutive lanes as one contiguous run.
// Long keys: the words ih | kOccupied, then il, then the counters.
template <uint32_t RW = 1>
__device__ __forceinline__ uint4 *seg_counts(uint64_t *seg) {
    return reinterpret_cast<uint4 *>(seg + RW * kSegSlots);
}
template <uint32_t RW = 1>
__device__ __forceinline__ const uint4 *seg_counts(const uint64_t *seg) {
    return reinterpret_cast<const uint4 *>(seg + RW * kSegSlots);
}

// Home slot inside a segment: the image's low bits.
__device__ __forceinline__ uint32_t seg_home(uint64_t x) { return (uint32_t)x & (kSegSlots - 1); }

}  // namespace dbgk
