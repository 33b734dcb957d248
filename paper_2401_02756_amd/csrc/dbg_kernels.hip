// HIP kernels of the A-Bruijn graph build for gfx950 (MI355X).
//
// The per-k-mer work is the paper's makeGraph body (Methods, "Lock-free graph
// creation algorithm", Algorithms 2-4): look the source (k-1)-mer up, add it
// if absent, raise its counter for the k-mer's last letter; for the target
// (k-1)-mer only make sure it exists.  Both halves are expressed per window:
// window j of a read with L >= k is its (k-1)-mer at offset j, for
// j = 0 .. L-k+1; every window is found-or-claimed, and every window but the
// last also raises one counter.  Window j's target is window j+1 of the same
// read, so claiming every window is exactly "add left and right vertex".
//
// Differences from the paper's CPU structure, for the device:
//   * open addressing with linear probing instead of chained buckets: a slot
//     goes from empty to one key once, by a 64-bit compare-and-swap (the
//     paper's CAS, Algorithm 1), and never changes key afterwards, so a
//     non-empty value read once is final and no list has to be walked;
//   * the key is the packed (k-1)-mer itself, so the paper's string compare
//     (Algorithm 4) is one 64-bit compare and no read has to stay resident;
//   * the out-edge pointers are not stored: the target of (v, c) is
//     (v << 2 | c) masked to 2(k-1) bits;
//   * counters are uint32, not uint8 (255 is exceeded by repeat-rich inputs).
#include "dbg_device.h"

#include <algorithm>

namespace dbgk {
namespace {
// ---------------------------------------------------------------- prepare

__global__ void k_prepare(const PassArgs *__restrict__ args, Instance *inst, InstStatus *st,
                          CallState *cs) {
    const uint32_t m = args->m;
    const uint64_t n = args->n_reads;
    const uint64_t *off = args->off;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        st[i].err = inst[i].skip ? kErrSkip : 0u;
        st[i].pad = 0;
        st[i].claimed = 0;
        st[i].inserts = 0;
        st[i].windows = 0;
        st[i].emitted = 0;
        // byte range of the instance, relative to the first read's first byte
        if (n) {
            const uint64_t off0 = off[0];
            const uint64_t rb = min(inst[i].read_begin, n), re = min(inst[i].read_end, n);
            inst[i].byte_begin = off[rb] - off0;
            inst[i].byte_end = off[re] - off0;
        }
    }
    if (i == 0) {
        cs->cursor = 0;
        cs->windows = 0;
    }
}

__global__ void k_fill_zero(uint64_t *__restrict__ words, uint64_t n_words) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t pairs = n_words >> 1;
    ulonglong2 *w2 = reinterpret_cast<ulonglong2 *>(words);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs; i += stride)
        w2[i] = make_ulonglong2(0ull, 0ull);
    if ((n_words & 1) && blockIdx.x == 0 && threadIdx.x == 0) words[n_words - 1] = 0;
}

__global__ void k_gather_u64(const uint64_t *__restrict__ src, const uint64_t *__restrict__ idx, uint64_t n,
                             uint64_t *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = src[idx[i]];
}

// ---------------------------------------------------------------- pack

// One thread per output word: 32 bases, letter code (c >> 1) & 3, first base
// in bits 63..62.  Words past the input are zero (the build reads one word
// beyond the last base of a window).
__global__ __launch_bounds__(256) void k_pack(const PassArgs *__restrict__ args,
                                             uint64_t *__restrict__ packed,
                                             const Instance *__restrict__ inst, InstStatus *st) {
    const uint8_t *__restrict__ ascii = args->reads;
    const uint64_t n = args->reads_len;
    const uint64_t n_words = packed_words(n);
    const uint32_t m = args->m;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const bool aligned = (reinterpret_cast<uintptr_t>(ascii) & 15) == 0;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n_words; w += stride) {
        const uint64_t b0 = w * 32;
        uint64_t v = 0;
        uint32_t bad = 0;  // bit i: byte b0 + i is not a letter
        if (aligned && b0 + 32 <= n) {
            const uint4 *src = reinterpret_cast<const uint4 *>(ascii + b0);
            const uint4 lo = src[0], hi = src[1];
            const uint32_t q[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const uint32_t c = (q[i >> 2] >> (8 * (i & 3))) & 0xffu;
                v |= (uint64_t)((c >> 1) & 3u) << (62 - 2 * i);
                bad |= (valid_letter(c) ? 0u : 1u) << i;
            }
        } else {
            for (int i = 0; i < 32; ++i) {
                if (b0 + i >= n) break;
                const uint32_t c = ascii[b0 + i];
                v |= (uint64_t)((c >> 1) & 3u) << (62 - 2 * i);
                bad |= (valid_letter(c) ? 0u : 1u) << i;
            }
        }
        packed[w] = v;
        while (bad) {
            const int i = __builtin_ctz(bad);
            bad &= bad - 1;
            const uint32_t t = (m == 1) ? 0u : instance_of_byte(inst, m, b0 + i);
            atomic_or_u32(&st[t].err, kErrBase);
        }
    }
}

// ---------------------------------------------------------------- scan

// Windows and k-mers of one read.  A read with bad offsets has none (the
// instance is flagged and the build skips it).
struct ReadCount {
    uint64_t windows, kmers;
    bool bad;
};

__device__ __forceinline__ ReadCount count_read(const uint64_t *off, uint64_t off0, uint64_t r,
                                                uint64_t n, uint64_t len, bool check_ends,
                                                uint32_t k) {
    ReadCount rc{0, 0, false};
    const uint64_t a = off[r], b = off[r + 1];
    if (b < a || a < off0 || b - off0 > len) {
        rc.bad = true;
        return rc;
    }
    if (check_ends && r + 1 == n && b - off0 != len) rc.bad = true;
    const uint64_t L = b - a;
    if (L >= k) {
        rc.windows = L - k + 2;
        rc.kmers = L - k + 1;
    }
    return rc;
}

// Per-read windows, block-local exclusive prefix and block totals; also the
// k-mers and windows of each instance.  A single instance's totals are summed
// from per-block partials (kpart) by k_scan_partials: an atomic per block on
// one address would serialise about a thousand times.  In a batch, a block
// whose reads all belong to one instance, as they almost always do, adds its
// totals with one atomic.
__global__ __launch_bounds__(kScanBlock) void k_scan_local(
    const PassArgs *__restrict__ args, const Instance *__restrict__ inst, InstStatus *st,
    uint64_t *__restrict__ ws, uint64_t *__restrict__ partials, uint64_t *__restrict__ kpart) {
    __shared__ uint32_t s_t0, s_t1;
    const uint64_t *__restrict__ off = args->off;
    const uint64_t n = args->n_reads, len = args->reads_len;
    const uint32_t m = args->m, check_ends = args->check_ends;
    const uint64_t rb = (uint64_t)blockIdx.x * kScanReads;
    if (rb >= n) {  // grid sized for the capacity: blocks past the reads add nothing
        if (threadIdx.x == 0) partials[blockIdx.x] = kpart[blockIdx.x] = 0;
        return;
    }
    const uint64_t off0 = off[0];
    const uint64_t r0 = rb + (uint64_t)threadIdx.x * kScanPerThread;
    if (threadIdx.x == 0) {
        s_t0 = m == 1 ? 0u : instance_of_read(inst, m, rb);
        s_t1 = m == 1 ? 0u : instance_of_read(inst, m, min(rb + kScanReads, n) - 1);
    }
    __syncthreads();
    const bool uniform = s_t0 == s_t1;
    uint64_t w[kScanPerThread];
    uint64_t tw = 0, tk = 0;
    uint32_t t = (m == 1 || r0 >= n) ? 0u : instance_of_read(inst, m, r0);
    uint64_t run_w = 0, run_k = 0;  // this thread's sums for instance t (non-uniform blocks)
#pragma unroll
    for (uint32_t i = 0; i < kScanPerThread; ++i) {
        const uint64_t r = r0 + i;
        w[i] = 0;
        if (r < n) {
            while (t + 1 < m && inst[t + 1].read_begin <= r) {
                if (!uniform && (run_w | run_k)) {
                    atomic_add_u64(&st[t].windows, run_w);
                    atomic_add_u64(&st[t].inserts, run_k);
                }
                run_w = run_k = 0;
                ++t;
            }
            const ReadCount rc = count_read(off, off0, r, n, len, check_ends != 0, inst[t].k);
            if (rc.bad) atomic_or_u32(&st[t].err, kErrInval);
            w[i] = rc.windows;
            tw += rc.windows;
            tk += rc.kmers;
            run_w += rc.windows;
            run_k += rc.kmers;
        }
    }
    if (!uniform && (run_w | run_k)) {
        atomic_add_u64(&st[t].windows, run_w);
        atomic_add_u64(&st[t].inserts, run_k);
    }
    uint64_t total;
    uint64_t pre = block_exclusive_scan(tw, &total);
#pragma unroll
    for (uint32_t i = 0; i < kScanPerThread; ++i) {
        const uint64_t r = r0 + i;
        if (r < n) ws[r] = pre;
        pre += w[i];
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
    uint64_t ktotal = 0;
    if (uniform) block_exclusive_scan(tk, &ktotal);
    if (threadIdx.x == 0) {
        kpart[blockIdx.x] = m == 1 ? ktotal : 0;
        if (m > 1 && uniform && (total | ktotal)) {
            atomic_add_u64(&st[s_t0].inserts, ktotal);
            atomic_add_u64(&st[s_t0].windows, total);
        }
    }
}

// Exclusive scan of the block totals.  Valid offsets give at most one window
// per byte, which is what the tile map is sized for; overlapping (malformed)
// offsets can exceed that, and then every instance is flagged invalid and no
// window is processed.
__global__ __launch_bounds__(1024) void k_scan_partials(const PassArgs *__restrict__ args,
                                                       uint64_t *partials, const uint64_t *kpart, uint64_t nb,
                                                       CallState *cs, InstStatus *st) {
    const uint64_t max_windows = args->max_windows;
    const uint32_t m = args->m;
    uint64_t carry = 0, kcarry = 0;
    for (uint64_t base = 0; base < nb; base += blockDim.x) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? partials[i] : 0;
        uint64_t total, ktotal = 0;
        const uint64_t ex = block_exclusive_scan(v, &total);
        if (i < nb) partials[i] = carry + ex;
        carry += total;
        if (m == 1) {
            block_exclusive_scan(i < nb ? kpart[i] : 0, &ktotal);
            kcarry += ktotal;
        }
    }
    if (m == 1 && threadIdx.x == 0) {  // the single instance's totals
        st[0].windows = carry;
        st[0].inserts = kcarry;
    }
    if (carry > max_windows) {
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) atomic_or_u32(&st[i].err, kErrInval);
        carry = 0;
    }
    if (threadIdx.x == 0) cs->windows = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(
    const PassArgs *__restrict__ args, const Instance *__restrict__ inst, uint64_t *__restrict__ ws,
    const uint64_t *__restrict__ partials, uint64_t *__restrict__ tile_read) {
    const uint64_t *__restrict__ off = args->off;
    const uint64_t n = args->n_reads, len = args->reads_len, tile_cap = args->tile_cap;
    const uint32_t m = args->m, check_ends = args->check_ends, tile = args->tile;
    if ((uint64_t)blockIdx.x * kScanReads >= n) return;
    const uint64_t r0 = (uint64_t)blockIdx.x * kScanReads + (uint64_t)threadIdx.x * kScanPerThread;
    const uint64_t add = partials[blockIdx.x];
    const uint64_t off0 = off[0];
    uint32_t t = (m == 1 || r0 >= n) ? 0u : instance_of_read(inst, m, r0);
#pragma unroll
    for (uint32_t i = 0; i < kScanPerThread; ++i) {
        const uint64_t r = r0 + i;
        if (r >= n) break;
        while (t + 1 < m && inst[t + 1].read_begin <= r) ++t;
        const ReadCount rc = count_read(off, off0, r, n, len, check_ends != 0, inst[t].k);
        const uint64_t s = ws[r] + add;
        ws[r] = s;
        if (r + 1 == n) ws[n] = s + rc.windows;
        // tiles whose first window falls inside this read start here
        if (tile_read)
            for (uint64_t tt = (s + tile - 1) / tile; tt * tile < s + rc.windows && tt < tile_cap; ++tt)
                tile_read[tt] = r;
    }
}

// ---------------------------------------------------------------- build

// Find the slot of `key` in the table, claiming an empty one if the key is
// absent (paper Algorithms 3 and 4 in open-addressing form).  A relaxed load
// first: a non-empty value is final, so most lookups of an existing vertex
// never issue an atomic.  An empty value (possibly stale) is resolved by the
// CAS, whose returned value says whether this lane claimed the slot, another
// lane claimed it for the same key, or another key took it.
//
// Returns kAllOnes when no empty slot lies within kMaxProbe slots of the home
// slot (or within the whole table when it is smaller), or when another lane
// has already reported this table full.  At the load factors the table is
// sized for (<= 0.9) linear-probing clusters stay orders of magnitude shorter
// than kMaxProbe, so this only fires on a table that is full in practice.
constexpr uint64_t kMaxProbe = 1ull << 16;

// Home slot of a key in the direct table: the mixed key's range reduction,
// or, with the test hash, the key's low 3 bits (cap >= 64), which sends
// every key of the table down the same probe chain.
__device__ __forceinline__ uint64_t direct_home(uint64_t key_bits, uint64_t h, uint64_t cap, uint32_t test_hash) {
    return test_hash ? (key_bits & 7u) : home_slot(h, cap);
}

template <bool STATS>
__device__ __forceinline__ uint64_t find_or_claim(uint64_t *table, uint32_t ew, uint64_t cap,
                                                  uint64_t key, uint64_t h, bool &claimed,
                                                  uint32_t *err, uint32_t test_hash, ProbeStats &ps) {
    const uint64_t tag = key | kOccupied;
    const uint64_t limit = cap < kMaxProbe ? cap : kMaxProbe;
    uint64_t s = direct_home(key, h, cap, test_hash);
    for (uint64_t probe = 0; probe < limit; ++probe) {
        uint64_t *kp = table + s * ew;
        const uint64_t cur = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == tag) {
            if (STATS) ps.lookup((uint32_t)min<uint64_t>(probe + 1, 0xffffffffu));
            return s;
        }
        if (cur == 0) {
            uint64_t expected = 0;
            const bool won = __hip_atomic_compare_exchange_strong(kp, &expected, tag, __ATOMIC_RELAXED,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (STATS) {
                ++ps.cas;
                ps.lost += won ? 0u : 1u;
            }
            if (won || expected == tag) {
                claimed = won;
                if (STATS) ps.lookup((uint32_t)min<uint64_t>(probe + 1, 0xffffffffu));
                return s;
            }
        }
        s = (s + 1 == cap) ? 0 : s + 1;
        if ((probe & 255) == 255 &&
            (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrFull))
            return kAllOnes;
    }
    return kAllOnes;
}

__device__ __forceinline__ void add_count(uint64_t *table, uint32_t ew, uint64_t s, uint32_t letter,
                                          uint32_t inc) {
    uint32_t *cnt = reinterpret_cast<uint32_t *>(table + s * ew + 1);
    __hip_atomic_fetch_add(cnt + letter, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr uint32_t kMergeSlots = 128;
constexpr uint32_t kMaxWaves = 16;

struct Window {
    uint64_t key;
    uint32_t letter;
    uint32_t inst;
    bool valid;  // a window of a read of an instance without errors
    bool sink;   // last window of its read: vertex only, no counter
};

// Instance of read r for a batched launch, with bit 31 set when its windows
// must be skipped: its input failed validation, its k-mer total would
// overflow a counter (every workgroup evaluates the same test, so the whole
// instance is skipped), or its table is already full.
__device__ __forceinline__ uint32_t instance_state(const Instance *inst, uint32_t m, InstStatus *st,
                                                   uint64_t r) {
    const uint32_t t = instance_of_read(inst, m, r);
    uint32_t e = __hip_atomic_load(&st[t].err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(e & kErrRange) && inst[t].prior_inserts + st[t].inserts > 0xffffffffull) {
        atomic_or_u32(&st[t].err, kErrRange);
        e |= kErrRange;
    }
    return (e & (kErrBase | kErrInval | kErrRange | kErrFull | kErrSkip)) ? (t | 0x80000000u) : t;
}

template <bool SINGLE, bool MERGE, bool STATS>
__global__ __launch_bounds__(1024) void k_build(const PassArgs *__restrict__ args,
                                               const Instance *__restrict__ inst,
                                               const uint64_t *__restrict__ packed,
                                               const uint64_t *__restrict__ ws,
                                               const uint64_t *__restrict__ tile_read,
                                               InstStatus *st, CallState *cs, uint32_t wpt) {
    const uint64_t *__restrict__ off = args->off;
    const uint64_t n = args->n_reads;
    const uint32_t m = args->m;
    __shared__ uint64_t s_ws[kMapReads + 1];
    __shared__ uint64_t s_delta[kMapReads];
    __shared__ uint32_t s_inst[kMapReads];  // instance index, bit 31 = skip
    __shared__ uint64_t s_tile;
    __shared__ uint64_t s_claims;
    __shared__ uint32_t s_slot[MERGE ? kMaxWaves * kMergeSlots : 1];
    __shared__ uint32_t s_cnt[MERGE ? kMaxWaves * 64 * 4 : 1];

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t W = cs->windows;
    const uint64_t off0 = n ? off[0] : 0;
    const uint64_t T = (uint64_t)blockDim.x * wpt;
    const uint64_t ntiles = (W + T - 1) / T;

    // Single-graph launch: the graph's parameters stay in registers, and the
    // whole launch stops at once if validation failed or the k-mer count
    // would overflow a counter (every workgroup evaluates the same test).
    uint64_t *tab0 = nullptr;
    uint64_t cap0 = 0;
    uint32_t ew0 = 3, km1_0 = 0;
    if (SINGLE) {
        tab0 = inst[0].table;
        cap0 = inst[0].cap;
        ew0 = inst[0].entry_words;
        km1_0 = inst[0].k - 1;
        if (inst[0].prior_inserts + st[0].inserts > 0xffffffffull) {
            if (tid == 0) atomic_or_u32(&st[0].err, kErrRange);
            return;
        }
        if (__hip_atomic_load(&st[0].err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
            (kErrBase | kErrInval | kErrRange | kErrSkip))
            return;
    }

    uint64_t my_claims = 0;  // SINGLE: flushed once at the end
    if (tid == 0) s_claims = 0;
    const uint32_t test_hash = args->test_hash;
    ProbeStats ps;

    for (;;) {
        if (tid == 0) {
            s_tile = __hip_atomic_fetch_add(&cs->cursor, 1ull, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            // a full single table stops the whole launch
            if (SINGLE && (__hip_atomic_load(&st[0].err, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) & kErrFull))
                s_tile = ntiles;
        }
        __syncthreads();
        const uint64_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint64_t w0 = tile * T;
        const uint64_t w1 = min(w0 + T, W);
        const uint64_t r0 = tile_read[tile];
        const uint32_t R = (uint32_t)min((uint64_t)kMapReads, n - r0);

        // Stage the tile's reads: window prefix, base offset, instance.
        for (uint32_t i = tid; i <= R; i += blockDim.x) {
            const uint64_t r = r0 + i;
            const uint64_t wr = ws[r];
            s_ws[i] = wr;
            if (i < R) {
                s_delta[i] = off[r] - off0 - wr;
                s_inst[i] = SINGLE ? 0u : instance_state(inst, m, st, r);
            }
        }
        __syncthreads();

        uint32_t tile_inst0 = s_inst[0] & 0x7fffffffu;
        uint64_t tile_claims = 0;

        for (uint32_t it = 0; it < wpt; ++it) {
            const uint64_t w = w0 + (uint64_t)it * blockDim.x + tid;
            Window win{0, 0, 0, false, false};
            if (w < w1) {
                uint64_t wr, wr1, delta;
                uint32_t tinfo;
                if (w < s_ws[R]) {
                    uint32_t lo = 0, hi = R;  // s_ws[lo] <= w < s_ws[hi]
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (s_ws[mid] <= w) lo = mid; else hi = mid;
                    }
                    wr = s_ws[lo];
                    wr1 = s_ws[lo + 1];
                    delta = s_delta[lo];
                    tinfo = s_inst[lo];
                } else {
                    // The tile spans more reads than were staged.
                    uint64_t lo = r0 + R, hi = n;  // ws[lo] <= w < ws[hi]
                    while (hi - lo > 1) {
                        const uint64_t mid = (lo + hi) >> 1;
                        if (ws[mid] <= w) lo = mid; else hi = mid;
                    }
                    wr = ws[lo];
                    wr1 = ws[lo + 1];
                    delta = off[lo] - off0 - wr;
                    tinfo = SINGLE ? 0u : instance_state(inst, m, st, lo);
                }
                (void)wr;
                win.valid = (tinfo & 0x80000000u) == 0;
                win.inst = tinfo & 0x7fffffffu;
                win.sink = (w + 1 == wr1);
                if (win.valid) {
                    const uint32_t km1 = SINGLE ? km1_0 : inst[win.inst].k - 1;
                    const uint64_t b = bases_at(packed, w + delta);
                    win.key = b >> (64 - 2 * km1);
                    win.letter = (uint32_t)(b >> (62 - 2 * km1)) & 3u;
                }
            }
            uint64_t *tab = tab0;
            uint64_t cap = cap0;
            uint32_t ew = ew0;
            if (!SINGLE && win.valid) {
                tab = inst[win.inst].table;
                cap = inst[win.inst].cap;
                ew = inst[win.inst].entry_words;
            }
            const uint64_t h = mix64(win.key);

            uint32_t inc[4] = {0, 0, 0, 0};
            bool leader = win.valid;
            if (MERGE) {
                // Merge equal vertices of this wavefront: every lane writes
                // its lane id into a slot chosen by the key; the lane whose
                // id survives leads all lanes with the same key, which add
                // their letters into the leader's LDS counters.  A key whose
                // slot another key won simply stays on its own.
                uint32_t *slot = s_slot + wave * kMergeSlots;
                uint32_t *cnt = s_cnt + wave * 256;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    __hip_atomic_store(cnt + lane * 4 + c, 0u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
                const uint32_t sl = (uint32_t)h & (kMergeSlots - 1);
                if (win.valid)
                    __hip_atomic_store(slot + sl, lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                uint32_t winner = lane;
                if (win.valid)
                    winner = __hip_atomic_load(slot + sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                const uint64_t wkey = __shfl(win.key, (int)winner, 64);
                const uint32_t winst = __shfl(win.inst, (int)winner, 64);
                const uint32_t lead = (win.valid && wkey == win.key && winst == win.inst) ? winner : lane;
                if (win.valid && !win.sink)
                    __hip_atomic_fetch_add(cnt + lead * 4 + win.letter, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                leader = win.valid && lead == lane;
                if (leader) {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        inc[c] = __hip_atomic_load(cnt + lane * 4 + c, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            } else if (win.valid && !win.sink) {
                inc[win.letter] = 1;
            }

            if (leader) {
                bool claimed = false;
                const uint64_t s =
                    find_or_claim<STATS>(tab, ew, cap, win.key, h, claimed, &st[win.inst].err, test_hash, ps);
                if (s == kAllOnes) {
                    atomic_or_u32(&st[win.inst].err, kErrFull);
                } else {
                    if (MERGE) {
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (inc[c]) add_count(tab, ew, s, (uint32_t)c, inc[c]);
                    } else if (!win.sink) {
                        add_count(tab, ew, s, win.letter, 1u);
                    }
                    if (claimed) {
                        if (SINGLE) {
                            ++my_claims;
                        } else {
                            ++tile_claims;
                            if (win.inst != tile_inst0) {
                                // rare: tile crosses into another graph
                                atomic_add_u64(&st[win.inst].claimed, 1);
                                --tile_claims;
                            }
                        }
                    }
                }
            }
        }
        if (!SINGLE) {
            // claims of the tile's first graph: one atomic per workgroup
            for (int d = 32; d >= 1; d >>= 1) tile_claims += __shfl_xor(tile_claims, d, 64);
            if (lane == 0 && tile_claims)
                __hip_atomic_fetch_add(&s_claims, tile_claims, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            __syncthreads();
            if (tid == 0 && s_claims) {
                atomic_add_u64(&st[tile_inst0].claimed, s_claims);
                s_claims = 0;
            }
        }
        __syncthreads();
    }
    if (STATS) ps.flush(args->stats);
    if (SINGLE) {
        for (int d = 32; d >= 1; d >>= 1) my_claims += __shfl_xor(my_claims, d, 64);
        if (lane == 0 && my_claims)
            __hip_atomic_fetch_add(&s_claims, my_claims, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        if (tid == 0 && s_claims) atomic_add_u64(&st[0].claimed, s_claims);
    }
}

// ---------------------------------------------------------------- build, long k

// For 32 < k <= 64 the (k-1)-mer K has 64 to 126 bits and takes two words of
// a 32-byte entry: word 0 = kOccupied | K >> 63, word 1 = kWritten | (K mod
// 2^63), then the four counters.  A slot is claimed by the CAS of word 0
// alone; the claimer then stores word 1 once.  A lane that finds word 0
// equal to its own but word 1 still zero has met a claim in flight and reads
// the slot again (the claimer waits for nothing between its CAS and that
// store, so the wait ends); a word 1 of another key sends it on to the next
// slot.  Words are written once each, so no ordering between the two words
// is needed beyond each word's own atomicity.
constexpr uint64_t kWritten = 1ull << 63;
constexpr uint64_t kLow63 = kWritten - 1;
constexpr uint32_t kMaxInFlight = 1u << 20;  // re-reads of one claim in flight

template <bool STATS>
__device__ __forceinline__ uint64_t find_or_claim_wide(uint64_t *table, uint64_t cap, uint64_t tag0,
                                                       uint64_t tag1, uint64_t h, bool &claimed,
                                                       uint32_t *err, uint32_t test_hash, ProbeStats &ps) {
    const uint64_t limit = cap < kMaxProbe ? cap : kMaxProbe;
    uint64_t s = direct_home(tag1, h, cap, test_hash);
    uint64_t probes = 0;
    uint32_t waits = 0;
    for (;;) {
        uint64_t *e = table + s * 4;
        uint64_t cur = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0) {
            uint64_t expected = 0;
            const bool won = __hip_atomic_compare_exchange_strong(e, &expected, tag0, __ATOMIC_RELAXED,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (STATS) {
                ++ps.cas;
                ps.lost += won ? 0u : 1u;
            }
            if (won) {
                __hip_atomic_store(e + 1, tag1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                claimed = true;
                if (STATS) ps.lookup((uint32_t)min<uint64_t>(probes + 1, 0xffffffffu));
                return s;
            }
            cur = expected;
        }
        if (cur == tag0) {
            const uint64_t w1 = __hip_atomic_load(e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (w1 == tag1) {
                if (STATS) ps.lookup((uint32_t)min<uint64_t>(probes + 1, 0xffffffffu));
                return s;
            }
            if (w1 == 0) {  // a claim in flight: read this slot again
                if (++waits > kMaxInFlight) return kAllOnes;
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
        }
        if (++probes >= limit) return kAllOnes;
        s = (s + 1 == cap) ? 0 : s + 1;
        if ((probes & 255) == 255 &&
            (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrFull))
            return kAllOnes;
    }
}

// Plain (one-graph) build for 32 < k <= 64; same tiles and window map as
// k_build, one window per thread per step, no merging.
template <bool STATS>
__global__ __launch_bounds__(1024) void k_build_wide(const PassArgs *__restrict__ args,
                                                    const Instance *__restrict__ inst,
                                                    const uint64_t *__restrict__ packed,
                                                    const uint64_t *__restrict__ ws,
                                                    const uint64_t *__restrict__ tile_read,
                                                    InstStatus *st, CallState *cs, uint32_t wpt) {
    const uint64_t *__restrict__ off = args->off;
    const uint64_t n = args->n_reads;
    __shared__ uint64_t s_ws[kMapReads + 1];
    __shared__ uint64_t s_delta[kMapReads];
    __shared__ uint64_t s_tile;
    __shared__ uint64_t s_claims;

    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint64_t W = cs->windows;
    const uint64_t off0 = n ? off[0] : 0;
    const uint64_t T = (uint64_t)blockDim.x * wpt;
    const uint64_t ntiles = (W + T - 1) / T;
    uint64_t *tab = inst[0].table;
    const uint64_t cap = inst[0].cap;
    const uint32_t km1 = inst[0].k - 1;
    if (inst[0].prior_inserts + st[0].inserts > 0xffffffffull) {
        if (tid == 0) atomic_or_u32(&st[0].err, kErrRange);
        return;
    }
    if (__hip_atomic_load(&st[0].err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
        (kErrBase | kErrInval | kErrRange | kErrSkip))
        return;

    uint64_t my_claims = 0;
    if (tid == 0) s_claims = 0;
    const uint32_t test_hash = args->test_hash;
    ProbeStats ps;
    for (;;) {
        if (tid == 0) {
            s_tile = __hip_atomic_fetch_add(&cs->cursor, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(&st[0].err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrFull)
                s_tile = ntiles;
        }
        __syncthreads();
        const uint64_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint64_t w0 = tile * T;
        const uint64_t w1 = min(w0 + T, W);
        const uint64_t r0 = tile_read[tile];
        const uint32_t R = (uint32_t)min((uint64_t)kMapReads, n - r0);
        for (uint32_t i = tid; i <= R; i += blockDim.x) {
            const uint64_t rr = r0 + i;
            const uint64_t wr = ws[rr];
            s_ws[i] = wr;
            if (i < R) s_delta[i] = off[rr] - off0 - wr;
        }
        __syncthreads();

        for (uint32_t it = 0; it < wpt; ++it) {
            const uint64_t w = w0 + (uint64_t)it * blockDim.x + tid;
            if (w >= w1) continue;
            uint64_t wr1, delta;
            if (w < s_ws[R]) {
                uint32_t lo = 0, hi = R;  // s_ws[lo] <= w < s_ws[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_ws[mid] <= w) lo = mid; else hi = mid;
                }
                wr1 = s_ws[lo + 1];
                delta = s_delta[lo];
            } else {
                uint64_t lo = r0 + R, hi = n;  // ws[lo] <= w < ws[hi]
                while (hi - lo > 1) {
                    const uint64_t mid = (lo + hi) >> 1;
                    if (ws[mid] <= w) lo = mid; else hi = mid;
                }
                wr1 = ws[lo + 1];
                delta = off[lo] - off0 - ws[lo];
            }
            const bool sink = (w + 1 == wr1);
            uint64_t x0, x1, khi, klo;
            uint32_t letter;
            bases128_at(packed, w + delta, x0, x1);
            wide_window(x0, x1, km1, khi, klo, letter);
            const uint64_t a = (khi << 1) | (klo >> 63);
            const uint64_t tag0 = a | kOccupied, tag1 = (klo & kLow63) | kWritten;
            const uint64_t h = mix64(tag1 ^ mix64(a));
            bool claimed = false;
            const uint64_t s = find_or_claim_wide<STATS>(tab, cap, tag0, tag1, h, claimed, &st[0].err, test_hash, ps);
            if (s == kAllOnes) {
                atomic_or_u32(&st[0].err, kErrFull);
                continue;
            }
            if (!sink)
                __hip_atomic_fetch_add(reinterpret_cast<uint32_t *>(tab + s * 4 + 2) + letter, 1u,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            my_claims += claimed ? 1u : 0u;
        }
        __syncthreads();
    }
    if (STATS) ps.flush(args->stats);
    for (int d = 32; d >= 1; d >>= 1) my_claims += __shfl_xor(my_claims, d, 64);
    if (lane == 0 && my_claims)
        __hip_atomic_fetch_add(&s_claims, my_claims, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (tid == 0 && s_claims) atomic_add_u64(&st[0].claimed, s_claims);
}

// ---------------------------------------------------------------- extract

constexpr uint32_t kExtractBlock = 256;
constexpr uint32_t kExtractPerThread = 4;

// Compact occupied slots into (key, counts) records; one atomic per block
// reserves the output range.  Record order is unspecified.
template <bool WRITE>
__global__ __launch_bounds__(kExtractBlock) void k_extract(const uint64_t *__restrict__ table,
                                                          uint32_t ew, uint64_t cap,
                                                          uint64_t *__restrict__ okeys,
                                                          uint32_t *__restrict__ ocnt,
                                                          uint64_t ocap, uint64_t *out_n) {
    __shared__ uint64_t s_base;
    const uint64_t chunk = (uint64_t)kExtractBlock * kExtractPerThread;
    for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < cap; base += (uint64_t)gridDim.x * chunk) {
        uint64_t tags[kExtractPerThread];
        uint32_t mine = 0;
#pragma unroll
        for (uint32_t i = 0; i < kExtractPerThread; ++i) {
            const uint64_t s = base + (uint64_t)i * kExtractBlock + threadIdx.x;
            tags[i] = s < cap ? table[s * ew] : 0;
            mine += tags[i] != 0;
        }
        uint64_t total;
        uint64_t pre = block_exclusive_scan(mine, &total);
        if (threadIdx.x == 0) s_base = total ? atomicAdd((unsigned long long *)out_n, (unsigned long long)total) : 0;
        __syncthreads();
        if (WRITE) {
            uint64_t idx = s_base + pre;
#pragma unroll
            for (uint32_t i = 0; i < kExtractPerThread; ++i) {
                if (!tags[i]) continue;
                const uint64_t s = base + (uint64_t)i * kExtractBlock + threadIdx.x;
                if (idx < ocap) {
                    okeys[idx] = tags[i] & ~kOccupied;
                    const uint32_t *c = reinterpret_cast<const uint32_t *>(table + s * ew + 1);
                    uint4 v = make_uint4(c[0], c[1], c[2], c[3]);
                    *reinterpret_cast<uint4 *>(ocnt + 4 * idx) = v;
                }
                ++idx;
            }
        }
        __syncthreads();
    }
}

// Long-k table: each record's key as two words (K >> 64, K mod 2^64).
__global__ __launch_bounds__(kExtractBlock) void k_extract_wide(const uint64_t *__restrict__ table,
                                                               uint64_t cap, uint64_t *__restrict__ okeys,
                                                               uint32_t *__restrict__ ocnt, uint64_t ocap,
                                                               uint64_t *out_n) {
    __shared__ uint64_t s_base;
    const uint64_t chunk = (uint64_t)kExtractBlock * kExtractPerThread;
    for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < cap; base += (uint64_t)gridDim.x * chunk) {
        uint64_t tags[kExtractPerThread];
        uint32_t mine = 0;
#pragma unroll
        for (uint32_t i = 0; i < kExtractPerThread; ++i) {
            const uint64_t s = base + (uint64_t)i * kExtractBlock + threadIdx.x;
            tags[i] = s < cap ? table[s * 4] : 0;
            mine += tags[i] != 0;
        }
        uint64_t total;
        uint64_t pre = block_exclusive_scan(mine, &total);
        if (threadIdx.x == 0) s_base = total ? atomicAdd((unsigned long long *)out_n, (unsigned long long)total) : 0;
        __syncthreads();
        uint64_t idx = s_base + pre;
#pragma unroll
        for (uint32_t i = 0; i < kExtractPerThread; ++i) {
            if (!tags[i]) continue;
            const uint64_t s = base + (uint64_t)i * kExtractBlock + threadIdx.x;
            if (idx < ocap) {
                const ulonglong2 e = *reinterpret_cast<const ulonglong2 *>(table + s * 4);
                const uint4 c = *reinterpret_cast<const uint4 *>(table + s * 4 + 2);
                const uint64_t a = e.x & ~kOccupied, b = e.y & kLow63;
                okeys[2 * idx] = a >> 1;
                okeys[2 * idx + 1] = (a << 63) | b;
                *reinterpret_cast<uint4 *>(ocnt + 4 * idx) = c;
            }
            ++idx;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- roofline

// Random-access microbenchmark over `words` uint64 words: indices come from
// mix64 of the operation number, so no index array is read.
__global__ __launch_bounds__(1024) void k_roofline(uint64_t *mem, uint64_t words, uint64_t n_ops,
                                                  uint32_t kind, uint64_t seed, uint64_t *sink) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    const uint64_t entries = words / 3;
    for (uint64_t op = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; op < n_ops; op += stride) {
        const uint64_t h = mix64(seed + op);
        if (kind == 0) {
            acc += __hip_atomic_load(mem + home_slot(h, words), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        } else if (kind == 1) {
            uint32_t *m32 = reinterpret_cast<uint32_t *>(mem);
            __hip_atomic_fetch_add(m32 + home_slot(h, words * 2), 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else if (kind == 2) {
            uint64_t expected = 0;
            __hip_atomic_compare_exchange_strong(mem + home_slot(h, words), &expected, h | 1,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            acc += expected;
        } else {
            uint64_t *e = mem + home_slot(h, entries) * 3;
            const uint64_t k = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t *c = reinterpret_cast<uint32_t *>(e + 1);
            __hip_atomic_fetch_add(c + (k & 3), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (acc == 0x5eed5eed5eed5eedull) sink[0] = acc;
}

// Streaming copy of the first half of mem onto the second, 16 bytes per
// load and store: a plain copy of known size for scaling traffic counters.
__global__ __launch_bounds__(1024) void k_stream_copy(uint64_t *mem, uint64_t words) {
    const uint64_t half = (words / 2) & ~1ull;
    const ulonglong2 *src = reinterpret_cast<const ulonglong2 *>(mem);
    ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(mem + half);
    const uint64_t n = half / 2, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename K>
uint32_t grid_for(K kernel, int device, uint32_t block) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)block, 0) != hipSuccess ||
        per <= 0)
        per = 1;
    return (uint32_t)(cus * per);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_prepare(const PassArgs *args, Instance *inst, InstStatus *st, CallState *cs,
                          uint32_t m_cap, hipStream_t s) {
    const uint32_t threads = 256;
    const uint32_t blocks = (m_cap + threads - 1) / threads;
    hipLaunchKernelGGL(k_prepare, dim3(blocks ? blocks : 1), dim3(threads), 0, s, args, inst, st, cs);
    return hipGetLastError();
}

hipError_t launch_gather_u64(const uint64_t *src, const uint64_t *idx, uint64_t n, uint64_t *out, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u64, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, src, idx, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(uint64_t *words, uint64_t n_words, hipStream_t s) {
    if (!n_words) return hipSuccess;
    const uint64_t pairs = (n_words + 1) / 2;
    const uint64_t want = (pairs + 255) / 256;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(want, 256 * 64);
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, words, n_words);
    return hipGetLastError();
}

hipError_t launch_pack(const PassArgs *args, uint64_t *packed, const Instance *inst, InstStatus *st,
                       uint64_t len_cap, hipStream_t s) {
    const uint64_t n_words = packed_words(len_cap);
    const uint64_t want = (n_words + 255) / 256;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, 256 * 64));
    hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(256), 0, s, args, packed, inst, st);
    return hipGetLastError();
}

hipError_t launch_scan(const PassArgs *args, const Instance *inst, InstStatus *st, uint64_t *ws,
                       uint64_t *partials, uint64_t *tile_read, CallState *cs, uint64_t n_cap,
                       hipStream_t s) {
    const uint64_t nb = std::max<uint64_t>(1, scan_blocks(n_cap));
    uint64_t *kpart = partials + nb;  // the partials buffer holds 2 * nb + 1 words
    hipLaunchKernelGGL(k_scan_local, dim3((uint32_t)nb), dim3(kScanBlock), 0, s, args, inst, st, ws,
                       partials, kpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, args, partials, kpart, nb, cs, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)nb), dim3(kScanBlock), 0, s, args, inst, ws, partials,
                       tile_read);
    return hipGetLastError();
}

hipError_t launch_build(const PassArgs *args, const Instance *inst, const uint64_t *packed,
                        const uint64_t *ws, const uint64_t *tile_read, InstStatus *st, CallState *cs,
                        BuildShape shape, bool single, bool stats, hipStream_t s) {
    const dim3 g(shape.grid), b(shape.block);
#define DBG_LAUNCH_BUILD(SINGLE, MERGE, STATS)                                                                    \
    hipLaunchKernelGGL((k_build<SINGLE, MERGE, STATS>), g, b, 0, s, args, inst, packed, ws, tile_read, st, cs, \
                       shape.wpt)
    if (stats) {
        if (single) {
            if (shape.merge) DBG_LAUNCH_BUILD(true, true, true); else DBG_LAUNCH_BUILD(true, false, true);
        } else {
            if (shape.merge) DBG_LAUNCH_BUILD(false, true, true); else DBG_LAUNCH_BUILD(false, false, true);
        }
    } else {
        if (single) {
            if (shape.merge) DBG_LAUNCH_BUILD(true, true, false); else DBG_LAUNCH_BUILD(true, false, false);
        } else {
            if (shape.merge) DBG_LAUNCH_BUILD(false, true, false); else DBG_LAUNCH_BUILD(false, false, false);
        }
    }
#undef DBG_LAUNCH_BUILD
    return hipGetLastError();
}

hipError_t launch_build_wide(const PassArgs *args, const Instance *inst, const uint64_t *packed,
                             const uint64_t *ws, const uint64_t *tile_read, InstStatus *st, CallState *cs,
                             BuildShape shape, bool stats, hipStream_t s) {
    if (stats)
        hipLaunchKernelGGL(k_build_wide<true>, dim3(shape.grid), dim3(shape.block), 0, s, args, inst, packed, ws,
                           tile_read, st, cs, shape.wpt);
    else
        hipLaunchKernelGGL(k_build_wide<false>, dim3(shape.grid), dim3(shape.block), 0, s, args, inst, packed, ws,
                           tile_read, st, cs, shape.wpt);
    return hipGetLastError();
}

namespace {

// round-half-up(c * genome / total) = floor((2 c genome + total) / (2 total)),
// exactly: the 128-bit numerator is divided 16 bits at a time (the divisor
// 2 total is below 2^34, so a partial remainder shifted by 16 stays below
// 2^50); saturated at 2^32 - 1.
__device__ __forceinline__ uint32_t normalized(uint32_t c, uint64_t genome, uint64_t total) {
    if (!genome || !total) return c;
    uint64_t lo = (uint64_t)c * genome;
    uint64_t hi = __umul64hi((uint64_t)c, genome);
    hi = (hi << 1) | (lo >> 63);
    lo <<= 1;
    const uint64_t lo2 = lo + total;
    hi += lo2 < lo ? 1u : 0u;
    lo = lo2;
    const uint64_t d = 2 * total;
    uint64_t q = 0, r = 0;
    for (int i = 7; i >= 0; --i) {
        const uint64_t limb = (i >= 4 ? hi >> (16 * (i - 4)) : lo >> (16 * i)) & 0xffffu;
        const uint64_t cur = (r << 16) | limb;
        const uint64_t qd = cur / d;
        r = cur - qd * d;
        if (q >> 48) return 0xffffffffu;
        q = (q << 16) | qd;
    }
    return q > 0xffffffffull ? 0xffffffffu : (uint32_t)q;
}

__global__ __launch_bounds__(256) void k_normalize(uint32_t *counts, uint64_t n, uint64_t genome, uint64_t total,
                                                   uint8_t *out8) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = normalized(counts[i], genome, total);
        if (out8) out8[i] = (uint8_t)(v > 255u ? 255u : v);
        else counts[i] = v;
    }
}

}  // namespace

hipError_t launch_normalize(uint32_t *counts, uint64_t n, uint64_t genome, uint64_t total, uint8_t *out8,
                            hipStream_t s) {
    if (!n) return hipSuccess;
    const uint32_t g = (uint32_t)std::min<uint64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_normalize, dim3(g), dim3(256), 0, s, counts, n, genome, total, out8);
    return hipGetLastError();
}

hipError_t launch_extract(const uint64_t *table, uint32_t ew, uint64_t cap, uint64_t *okeys,
                          uint32_t *ocnt, uint64_t ocap, uint64_t *out_n, hipStream_t s) {
    const uint64_t chunk = (uint64_t)kExtractBlock * kExtractPerThread;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((cap + chunk - 1) / chunk, 256 * 32));
    hipLaunchKernelGGL((k_extract<true>), dim3(blocks), dim3(kExtractBlock), 0, s, table, ew, cap,
                       okeys, ocnt, ocap, out_n);
    return hipGetLastError();
}

hipError_t launch_extract_wide(const uint64_t *table, uint64_t cap, uint64_t *okeys, uint32_t *ocnt,
                               uint64_t ocap, uint64_t *out_n, hipStream_t s) {
    const uint64_t chunk = (uint64_t)kExtractBlock * kExtractPerThread;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((cap + chunk - 1) / chunk, 256 * 32));
    hipLaunchKernelGGL(k_extract_wide, dim3(blocks), dim3(kExtractBlock), 0, s, table, cap, okeys, ocnt, ocap,
                       out_n);
    return hipGetLastError();
}

hipError_t launch_count(const uint64_t *table, uint32_t ew, uint64_t cap, uint64_t *out_n,
                        hipStream_t s) {
    const uint64_t chunk = (uint64_t)kExtractBlock * kExtractPerThread;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((cap + chunk - 1) / chunk, 256 * 32));
    hipLaunchKernelGGL((k_extract<false>), dim3(blocks), dim3(kExtractBlock), 0, s, table, ew, cap,
                       nullptr, nullptr, 0, out_n);
    return hipGetLastError();
}

hipError_t launch_roofline(uint64_t *mem, uint64_t words, uint64_t n_ops, uint32_t kind, uint64_t seed,
                           uint32_t block, uint64_t *sink, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (kind == 4) {
        const uint32_t grid = grid_for(k_stream_copy, dev, block);
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(block), 0, s, mem, words);
        return hipGetLastError();
    }
    const uint32_t grid = grid_for(k_roofline, dev, block);
    hipLaunchKernelGGL(k_roofline, dim3(grid), dim3(block), 0, s, mem, words, n_ops, kind, seed, sink);
    return hipGetLastError();
}

uint32_t build_grid_wide(int device, uint32_t block) { return grid_for(k_build_wide<false>, device, block); }

uint32_t build_grid(int device, uint32_t block) {
    // the instantiations share the same resource shape up to LDS; the
    // merging one uses the most LDS and registers, so size from it (the
    // statistics kernels may fit fewer workgroups: tiles come from a cursor,
    // so extra workgroups simply start later)
    return grid_for(k_build<false, true, false>, device, block);
}

}  // namespace dbgk
