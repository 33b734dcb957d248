// Contigs of a built graph (Methods, "Finding contigs", Algorithm 5).
//
// The paper keeps a `first` flag per vertex, cleared whenever the vertex is
// added as a right vertex, so it marks vertices no k-mer ends in (in-degree
// 0).  Contigs start at every vertex with `first` or with more than one
// out-edge, one per out-edge, and go on while the vertex reached has exactly
// one out-edge.  The passage leaves loops of one-edge vertices open (the walk
// would never end); here a walk also stops on the first vertex it has already
// passed.  The vertex a walk stops on is part of its contig.
//
// On the device: the graph's vertices go into a walk table (key, out-letter
// mask).  For a binned graph the walk table has the graph's own segments:
// each workgroup rehashes one packed segment in LDS and writes its slots out,
// so a key is found from its image's segment digits and home slot, with no
// extraction and no global atomics.  For a direct graph the vertices are
// extracted and inserted into a hash table.  Then a mark pass follows every
// edge once and flags its target as having an in-edge (so `first` = no
// flag); a start pass lists one walk per out-edge of every start vertex; a
// length pass follows every walk (Brent's cycle detection finds the loops,
// then the first revisit is located exactly); a scan lays the contigs out;
// a write pass spells them.  Every loop is bounded, so a
// walk that cannot end reports an error instead of running forever.
#include "dbg_runtime.h"
#include "dbg_device.h"

using namespace dbgrt;
using dbgk::block_exclusive_scan;
using dbgk::bucket_of;
using dbgk::child_of;
using dbgk::home_slot;
using dbgk::image_top;
using dbgk::key_image;
using dbgk::key_of_image;
using dbgk::kOccupied;
using dbgk::kSegSlots;
using dbgk::mix64;
using dbgk::seg_counts;
using dbgk::seg_home;

namespace {

constexpr uint32_t kWalkBlock = 256;

constexpr uint8_t kOutMask = 0x0f;  // bits 0-3: out-edges by letter code
constexpr uint8_t kHasIn = 0x10;    // some k-mer ends in the vertex

struct WalkTable {
    uint64_t *keys;   // key (segmented: key image) | kOccupied, 0 = empty
    uint8_t *masks;   // bit c: the vertex has an out-edge for letter code c; kHasIn
    uint64_t cap;     // slots: a power of two, or (segmented) segments * kSegSlots
    uint64_t kmask;   // (k-1)-mer key mask
    uint32_t km1;
    uint32_t seg;     // 1: segmented like the binned graph, d1 x fan segments
    uint32_t d1, fan;
};

// The key stored in an occupied slot.
__device__ __forceinline__ uint64_t slot_key(const WalkTable &T, uint64_t s) {
    const uint64_t w = T.keys[s] & ~kOccupied;
    return T.seg ? key_of_image(w) : w;
}

// Slot of `key`, or ~0 when absent (after at most a segment's or the
// table's slots); *mb receives the slot's mask byte, loaded beside each
// probed key so that a walk step waits on one load, not two in a row.
__device__ __forceinline__ uint64_t walk_find(const WalkTable &T, uint64_t key, uint32_t *mb = nullptr) {
    if (T.seg) {
        const uint64_t img = key_image(key), tagv = img | kOccupied;
        const uint32_t top = image_top(img);
        const uint64_t base = ((uint64_t)bucket_of(top, T.d1) * T.fan + child_of(top, T.d1, T.fan)) * kSegSlots;
        uint32_t s = seg_home(img);
        for (uint32_t q = 0; q < kSegSlots; ++q) {
            const uint64_t cur = T.keys[base + s];
            const uint32_t m = T.masks[base + s];
            if (cur == tagv) {
                if (mb) *mb = m;
                return base + s;
            }
            if (cur == 0) return ~0ull;
            s = (s + 1) & (kSegSlots - 1);
        }
        return ~0ull;
    }
    const uint64_t tagv = key | kOccupied;
    uint64_t s = home_slot(mix64(key), T.cap);
    for (uint64_t q = 0; q < T.cap; ++q) {
        const uint64_t cur = T.keys[s];
        const uint32_t m = T.masks[s];
        if (cur == tagv) {
            if (mb) *mb = m;
            return s;
        }
        if (cur == 0) return ~0ull;
        s = (s + 1) & (T.cap - 1);
    }
    return ~0ull;
}

__global__ __launch_bounds__(kWalkBlock) void k_walk_insert(WalkTable T, const uint64_t *__restrict__ keys,
                                                            const uint32_t *__restrict__ counts, uint64_t n,
                                                            uint32_t *err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t key = keys[i];
        const uint4 c = *reinterpret_cast<const uint4 *>(counts + 4 * i);
        const uint8_t m = (uint8_t)((c.x ? 1u : 0u) | (c.y ? 2u : 0u) | (c.z ? 4u : 0u) | (c.w ? 8u : 0u));
        uint64_t s = home_slot(mix64(key), T.cap);
        bool placed = false;
        for (uint64_t q = 0; q < T.cap && !placed; ++q) {
            unsigned long long expected = 0;
            if (__hip_atomic_compare_exchange_strong(reinterpret_cast<unsigned long long *>(&T.keys[s]), &expected,
                                                     (unsigned long long)(key | kOccupied), __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                T.masks[s] = m;
                placed = true;
            } else {
                s = (s + 1) & (T.cap - 1);
            }
        }
        if (!placed) atomicOr(err, 1u);
    }
}


// Flag the target of every edge.  Every writer of a mask byte writes the same
// value (its out-edges and kHasIn), so plain byte stores suffice.
__global__ __launch_bounds__(kWalkBlock) void k_walk_mark(WalkTable T, uint32_t *err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T.cap; i += stride) {
        if (!T.keys[i]) continue;
        const uint64_t key = slot_key(T, i);
        const uint32_t m = T.masks[i] & kOutMask;
#pragma unroll
        for (uint32_t x = 0; x < 4; ++x) {
            if (!((m >> x) & 1u)) continue;
            uint32_t mt = 0;
            const uint64_t s = walk_find(T, ((key << 2) | x) & T.kmask, &mt);
            if (s == ~0ull) {
                atomicOr(err, 16u);  // an edge without its target vertex
                continue;
            }
            if (!(mt & kHasIn)) T.masks[s] = (uint8_t)(mt | kHasIn);
        }
    }
}

// Walk table of a binned graph: segment gp of the graph (its vertices packed
// at [0, seg_count[gp])) is rehashed in LDS by its image's home slots and
// written to slots [gp * kSegSlots, (gp + 1) * kSegSlots), empty ones as 0.
template <uint32_t EW>
__global__ __launch_bounds__(kWalkBlock) void k_walk_seg(const uint64_t *__restrict__ table,
                                                         const uint32_t *__restrict__ seg_count, uint64_t parts,
                                                         WalkTable T, uint32_t *err) {
    __shared__ uint64_t s_key[kSegSlots];
    __shared__ uint8_t s_mask[kSegSlots];
    for (uint64_t gp = blockIdx.x; gp < parts; gp += gridDim.x) {
        for (uint32_t j = threadIdx.x; j < kSegSlots; j += blockDim.x) {
            s_key[j] = 0;
            s_mask[j] = 0;
        }
        __syncthreads();
        const uint64_t *seg = table + gp * kSegSlots * EW;
        const uint32_t n = min(seg_count[gp], kSegSlots);
        for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) {
            const uint64_t tagv = seg[e];
            const uint4 c = seg_counts(seg)[e];
            const uint8_t m = (uint8_t)((c.x ? 1u : 0u) | (c.y ? 2u : 0u) | (c.z ? 4u : 0u) | (c.w ? 8u : 0u));
            uint32_t s = seg_home(tagv);
            bool placed = false;
            for (uint32_t q = 0; q < kSegSlots && !placed; ++q) {  // keys are distinct
                uint64_t expected = 0;
                if (__hip_atomic_compare_exchange_strong(&s_key[s], &expected, tagv, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    s_mask[s] = m;
                    placed = true;
                } else {
                    s = (s + 1) & (kSegSlots - 1);
                }
            }
            if (!placed) atomicOr(err, 1u);
        }
        __syncthreads();
        uint64_t *ok = T.keys + gp * kSegSlots;
        uint8_t *om = T.masks + gp * kSegSlots;
        for (uint32_t j = threadIdx.x; j < kSegSlots; j += blockDim.x) {
            ok[j] = s_key[j];
            om[j] = s_mask[j];
        }
        __syncthreads();
    }
}

// Walks (slot << 2 | letter) of the start vertices, appended in any order.
// A workgroup takes kStartChunk consecutive slots and reserves its output
// range with one atomic (an atomic per wavefront on one counter serialises
// millions of times at this table size).
constexpr uint32_t kStartEach = 16, kStartChunk = kWalkBlock * kStartEach;

__global__ __launch_bounds__(kWalkBlock) void k_walk_starts(WalkTable T, uint64_t *__restrict__ items,
                                                            uint64_t items_cap, unsigned long long *n_items,
                                                            uint32_t *err) {
    __shared__ unsigned long long s_base;
    const uint64_t chunks = (T.cap + kStartChunk - 1) / kStartChunk;
    for (uint64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const uint64_t s0 = ch * kStartChunk + threadIdx.x;
        uint32_t outs[kStartEach];
        uint32_t mine = 0;
#pragma unroll
        for (uint32_t j = 0; j < kStartEach; ++j) {
            const uint64_t s = s0 + (uint64_t)j * kWalkBlock;
            uint32_t mb = 0;
            if (s < T.cap && T.keys[s]) mb = T.masks[s];
            const uint32_t m = mb & kOutMask;
            const uint32_t deg = __popc(m);
            const bool start = deg >= 2 || (deg == 1 && !(mb & kHasIn));
            outs[j] = start ? m : 0u;
            mine += start ? deg : 0u;
        }
        uint64_t total;
        const uint64_t pre = block_exclusive_scan(mine, &total);
        if (threadIdx.x == 0) s_base = total ? atomicAdd(n_items, (unsigned long long)total) : 0ull;
        __syncthreads();
        uint64_t at = s_base + pre;
#pragma unroll
        for (uint32_t j = 0; j < kStartEach; ++j) {
            const uint64_t s = s0 + (uint64_t)j * kWalkBlock;
            for (uint32_t c = 0; c < 4; ++c) {
                if (!((outs[j] >> c) & 1u)) continue;
                if (at < items_cap) items[at] = (s << 2) | c;
                else atomicOr(err, 2u);
                ++at;
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ uint64_t succ(const WalkTable &T, uint64_t key, uint32_t m) {
    return ((key << 2) | (uint32_t)__builtin_ctz(m)) & T.kmask;
}

// Edges of every walk: x0 (the start) -> x1 -> ..., stopping on the first
// x_m with other than one out-edge or equal to an earlier x_j.  x0 is never
// passed again (it has no in-edge or several out-edges), so a revisit can
// only happen on a loop of one-edge vertices, which Brent's method finds;
// then the loop's length lam and entry mu give m = mu + lam exactly.
__global__ __launch_bounds__(kWalkBlock) void k_walk_length(WalkTable T, const uint64_t *__restrict__ items,
                                                            const unsigned long long *n_items,
                                                            uint64_t *__restrict__ edges, uint64_t limit,
                                                            uint32_t *err) {
    const uint64_t n = *n_items;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t it = items[i];
        const uint64_t key0 = slot_key(T, it >> 2);
        const uint64_t x1 = ((key0 << 2) | (it & 3)) & T.kmask;
        uint64_t hare = x1, tort = x1, power = 1, lam = 1, idx = 1;
        bool loop = false, bad = false;
        for (;;) {
            uint32_t mb = 0;
            const uint64_t s = walk_find(T, hare, &mb);
            if (s == ~0ull || idx > limit) { bad = true; break; }
            const uint32_t m = mb & kOutMask;
            if (__popc(m) != 1) break;  // stops on x_idx
            hare = succ(T, hare, m);
            ++idx;
            if (hare == tort) { loop = true; break; }
            if (power == lam) {
                tort = hare;
                power <<= 1;
                lam = 0;
            }
            ++lam;
        }
        if (loop) {
            // x_{mu} is the first vertex of the loop: walk a from x1 and b from
            // x_{1+lam} together until they meet
            uint64_t a = x1, b = x1;
            for (uint64_t q = 0; q < lam && !bad; ++q) {
                uint32_t mb = 0;
                const uint64_t s = walk_find(T, b, &mb);
                if (s == ~0ull) bad = true;
                else b = succ(T, b, mb & kOutMask);
            }
            uint64_t mu = 1;
            while (!bad && a != b) {
                uint32_t ma = 0, mbb = 0;
                const uint64_t sa = walk_find(T, a, &ma), sb = walk_find(T, b, &mbb);
                if (sa == ~0ull || sb == ~0ull || mu > limit) { bad = true; break; }
                a = succ(T, a, ma & kOutMask);
                b = succ(T, b, mbb & kOutMask);
                ++mu;
            }
            idx = mu + lam;
        }
        if (bad) {
            atomicOr(err, 4u);
            idx = 1;
        }
        edges[i] = idx;
    }
}

// Contig lengths in bases (k - 1 + edges), for the scan.
__global__ void k_walk_bases(const uint64_t *__restrict__ edges, const unsigned long long *n_items, uint32_t km1,
                             uint64_t *__restrict__ len) {
    const uint64_t n = *n_items;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) len[i] = km1 + edges[i];
}

// Exclusive scan of v[0, n) in place with v[n] = total, in three launches:
// per-block scans of kScanChunk values with the block sums in part[], one
// block scanning part[], and the carry added back.
constexpr uint32_t kScanThreads = 256, kScanEach = 8, kScanChunk = kScanThreads * kScanEach;

__global__ __launch_bounds__(kScanThreads) void k_walk_scan_local(uint64_t *v, uint64_t n, uint64_t *part) {
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanEach;
    uint64_t x[kScanEach], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanEach; ++j) {
        x[j] = b0 + j < n ? v[b0 + j] : 0;
        sum += x[j];
    }
    uint64_t total;
    uint64_t pre = block_exclusive_scan(sum, &total);
#pragma unroll
    for (uint32_t j = 0; j < kScanEach; ++j) {
        if (b0 + j < n) v[b0 + j] = pre;
        pre += x[j];
    }
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_walk_scan_part(uint64_t *part, uint64_t nb, uint64_t *v, uint64_t n) {
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += blockDim.x) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t x = i < nb ? part[i] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(x, &total);
        if (i < nb) part[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) v[n] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_walk_scan_add(uint64_t *v, uint64_t n, const uint64_t *part) {
    const uint64_t add = part[blockIdx.x];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk;
    for (uint32_t j = threadIdx.x; j < kScanChunk; j += kScanThreads)
        if (b0 + j < n) v[b0 + j] += add;
}

__global__ __launch_bounds__(kWalkBlock) void k_walk_write(WalkTable T, const uint64_t *__restrict__ items,
                                                           const unsigned long long *n_items,
                                                           const uint64_t *__restrict__ edges,
                                                           const uint64_t *__restrict__ off, uint8_t *__restrict__ seq,
                                                           uint32_t *err) {
    const uint8_t letters[4] = {'A', 'C', 'T', 'G'};
    const uint64_t n = *n_items;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t it = items[i];
        const uint64_t key0 = slot_key(T, it >> 2);
        uint8_t *o = seq + off[i];
        for (uint32_t b = 0; b < T.km1; ++b) *o++ = letters[(key0 >> (2 * (T.km1 - 1 - b))) & 3];
        *o++ = letters[it & 3];
        uint64_t cur = ((key0 << 2) | (it & 3)) & T.kmask;
        const uint64_t m = edges[i];
        for (uint64_t e = 1; e < m; ++e) {
            uint32_t mb = 0;
            const uint64_t s = walk_find(T, cur, &mb);
            if (s == ~0ull) {
                atomicOr(err, 8u);
                break;
            }
            const uint32_t c = (uint32_t)__builtin_ctz(mb & kOutMask);
            *o++ = letters[c];
            cur = ((cur << 2) | c) & T.kmask;
        }
    }
}

__global__ void k_walk_clear(uint64_t *keys, uint64_t cap) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) keys[i] = 0;
}

uint32_t grid_for(uint64_t n, uint32_t block) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + block - 1) / block, 65536));
}

}  // namespace

struct dbg_contig_state {
    DevBuf keys, masks, items, edges, off, part, seq, xkeys, xcnt, xn, scalars;
    uint64_t epoch = ~0ull;  // the graph's epoch the contigs were made for
    uint64_t n = 0, len = 0;
};

namespace {

// Compute (or reuse) the contigs of g on stream s: counts in cs->n / cs->len,
// contigs in cs->seq / cs->off on the device.
int compute_contigs(dbg_graph *g, dbg_contig_state *cs, hipStream_t s) {
    if (cs->epoch == g->epoch) return DBG_OK;
    const uint64_t V = g->vertices;
    cs->n = cs->len = 0;
    if (V == 0 || g->k == 0) {
        cs->epoch = g->epoch;
        return DBG_OK;
    }
    hipError_t e;
    // scalars: [0] walk count, [1] error bits
    if ((e = cs->scalars.reserve(32)) != hipSuccess) return hip_code(e);
    unsigned long long *n_items = cs->scalars.as<unsigned long long>();
    uint32_t *err = reinterpret_cast<uint32_t *>(cs->scalars.as<uint64_t>() + 1);
    e = dbgk::launch_fill_zero(cs->scalars.as<uint64_t>(), 2, s);
    const uint64_t kmask = (1ull << (2 * (g->k - 1))) - 1;
    WalkTable T{};
    if (g->binned) {
        // the graph's own segments, rehashed
        const uint64_t cap = (uint64_t)g->parts * kSegSlots;
        if (e == hipSuccess && ((e = cs->keys.reserve(cap * 8)) != hipSuccess || (e = cs->masks.reserve(cap)) != hipSuccess))
            return hip_code(e);
        T = WalkTable{cs->keys.as<uint64_t>(), cs->masks.as<uint8_t>(), cap, kmask, g->k - 1, 1u, g->d1, g->fan};
        if (e == hipSuccess) {
            const dim3 grid((uint32_t)std::min<uint64_t>(g->parts, 65536)), block(kWalkBlock);
            if (g->ew == 4)
                hipLaunchKernelGGL((k_walk_seg<4>), grid, block, 0, s, g->table.as<uint64_t>(),
                                   g->seg_count.as<uint32_t>(), (uint64_t)g->parts, T, err);
            else
                hipLaunchKernelGGL((k_walk_seg<3>), grid, block, 0, s, g->table.as<uint64_t>(),
                                   g->seg_count.as<uint32_t>(), (uint64_t)g->parts, T, err);
            e = hipGetLastError();
        }
    } else {
        // extracted vertices, inserted into a hash table
        uint64_t cap = 64;
        while (cap < 2 * V) cap <<= 1;
        if (e == hipSuccess &&
            ((e = cs->xkeys.reserve(V * 8)) != hipSuccess || (e = cs->xcnt.reserve(V * 16)) != hipSuccess ||
             (e = cs->xn.reserve(8)) != hipSuccess || (e = cs->keys.reserve(cap * 8)) != hipSuccess ||
             (e = cs->masks.reserve(cap)) != hipSuccess))
            return hip_code(e);
        T = WalkTable{cs->keys.as<uint64_t>(), cs->masks.as<uint8_t>(), cap, kmask, g->k - 1, 0u, 0u, 0u};
        uint64_t *xn = cs->xn.as<uint64_t>();
        if (e == hipSuccess) e = dbgk::launch_fill_zero(xn, 1, s);
        if (e == hipSuccess)
            e = dbgk::launch_extract(g->table.as<uint64_t>(), g->ew, g->cap, cs->xkeys.as<uint64_t>(),
                                     cs->xcnt.as<uint32_t>(), V, xn, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_walk_clear, dim3(grid_for(cap, 256)), dim3(256), 0, s, cs->keys.as<uint64_t>(), cap);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_walk_insert, dim3(grid_for(V, kWalkBlock)), dim3(kWalkBlock), 0, s, T,
                               cs->xkeys.as<uint64_t>(), cs->xcnt.as<uint32_t>(), V, err);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_walk_mark, dim3(grid_for(T.cap, kWalkBlock)), dim3(kWalkBlock), 0, s, T, err);
        e = hipGetLastError();
    }
    // walks are at most the edges, at most 4 per vertex
    const uint64_t items_cap = 4 * V;
    if (e == hipSuccess && (e = cs->items.reserve(items_cap * 8)) == hipSuccess) {
        hipLaunchKernelGGL(k_walk_starts, dim3(grid_for(T.cap, kStartChunk)), dim3(kWalkBlock), 0, s, T,
                           cs->items.as<uint64_t>(), items_cap, n_items, err);
        e = hipGetLastError();
    }
    uint64_t hs[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hs, cs->scalars.p, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_code(e);
    if ((uint32_t)hs[1]) return DBG_E_DEVICE;
    const uint64_t n = hs[0];
    const uint64_t nb = std::max<uint64_t>(1, (n + kScanChunk - 1) / kScanChunk);
    if ((e = cs->edges.reserve(std::max<uint64_t>(n, 1) * 8)) != hipSuccess ||
        (e = cs->off.reserve((n + 1) * 8)) != hipSuccess || (e = cs->part.reserve(nb * 8)) != hipSuccess)
        return hip_code(e);
    // a walk passes each vertex at most once before its loop closes, and
    // finding the loop takes at most twice its length more
    const uint64_t limit = 4 * V + 16;
    hipLaunchKernelGGL(k_walk_length, dim3(grid_for(n, kWalkBlock)), dim3(kWalkBlock), 0, s, T,
                       cs->items.as<uint64_t>(), n_items, cs->edges.as<uint64_t>(), limit, err);
    hipLaunchKernelGGL(k_walk_bases, dim3(grid_for(n, 256)), dim3(256), 0, s, cs->edges.as<uint64_t>(), n_items,
                       g->k - 1, cs->off.as<uint64_t>());
    hipLaunchKernelGGL(k_walk_scan_local, dim3((uint32_t)nb), dim3(kScanThreads), 0, s, cs->off.as<uint64_t>(), n,
                       cs->part.as<uint64_t>());
    hipLaunchKernelGGL(k_walk_scan_part, dim3(1), dim3(1024), 0, s, cs->part.as<uint64_t>(), nb,
                       cs->off.as<uint64_t>(), n);
    hipLaunchKernelGGL(k_walk_scan_add, dim3((uint32_t)nb), dim3(kScanThreads), 0, s, cs->off.as<uint64_t>(), n,
                       cs->part.as<uint64_t>());
    if ((e = hipGetLastError()) != hipSuccess) return hip_code(e);
    uint64_t total = 0;
    if ((e = hipMemcpyAsync(&total, cs->off.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_code(e);
    if ((e = cs->seq.reserve(std::max<uint64_t>(total, 1))) != hipSuccess) return hip_code(e);
    hipLaunchKernelGGL(k_walk_write, dim3(grid_for(n, kWalkBlock)), dim3(kWalkBlock), 0, s, T,
                       cs->items.as<uint64_t>(), n_items, cs->edges.as<uint64_t>(), cs->off.as<uint64_t>(),
                       cs->seq.as<uint8_t>(), err);
    if ((e = hipGetLastError()) != hipSuccess) return hip_code(e);
    uint32_t herr = 0;
    if ((e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_code(e);
    if (herr) return DBG_E_DEVICE;
    cs->n = n;
    cs->len = total;
    cs->epoch = g->epoch;
    return DBG_OK;
}

int contigs_common(dbg_graph *g, void *seq, uint64_t seq_cap, uint64_t *offsets, uint64_t offsets_cap,
                   uint64_t *n_contigs, uint64_t *seq_len, bool device_out, hipStream_t s) {
    if (!g || !n_contigs || !seq_len) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    if (g->pass.pending) {
        const int rc = harvest(g);
        if (rc != DBG_OK) g->unreported = rc;
    }
    if (g->poisoned) return DBG_E_STATE;
    if (g->k > 32) return DBG_E_K;  // walks use one-word keys
    if (!g->contigs) g->contigs = new dbg_contig_state();
    dbg_contig_state *cs = g->contigs;
    const int rc = compute_contigs(g, cs, s);
    if (rc != DBG_OK) {
        cs->epoch = ~0ull;
        return rc;
    }
    *n_contigs = cs->n;
    *seq_len = cs->len;
    if (!seq && !offsets) return DBG_OK;
    if (!seq || !offsets) return DBG_E_INVAL;
    if (seq_cap < cs->len || offsets_cap < cs->n + 1) return DBG_E_SPACE;
    const hipMemcpyKind kind = device_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipError_t e = hipSuccess;
    if (cs->len) e = hipMemcpyAsync(seq, cs->seq.p, cs->len, kind, s);
    if (e == hipSuccess) e = hipMemcpyAsync(offsets, cs->off.p, (cs->n + 1) * 8, kind, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? DBG_OK : DBG_E_DEVICE;
}

}  // namespace

void dbg_contigs_free(dbg_contig_state *cs) {
    if (!cs) return;
    DevBuf *b[] = {&cs->keys, &cs->masks, &cs->items, &cs->edges, &cs->off, &cs->part, &cs->seq, &cs->xkeys,
                   &cs->xcnt, &cs->xn, &cs->scalars};
    for (DevBuf *x : b) x->release();
    delete cs;
}

extern "C" {

int dbg_contigs(dbg_graph *g, char *seq, uint64_t seq_cap, uint64_t *offsets, uint64_t offsets_cap,
                uint64_t *n_contigs, uint64_t *seq_len) {
    return contigs_common(g, seq, seq_cap, offsets, offsets_cap, n_contigs, seq_len, false, g ? g->stream : nullptr);
}

int dbg_contigs_device(dbg_graph *g, uint8_t *d_seq, uint64_t seq_cap, uint64_t *d_offsets, uint64_t offsets_cap,
                       uint64_t *n_contigs, uint64_t *seq_len, void *stream) {
    return contigs_common(g, d_seq, seq_cap, d_offsets, offsets_cap, n_contigs, seq_len, true,
                          g ? g->pick(stream) : nullptr);
}

}  // extern "C"
