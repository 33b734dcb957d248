// Binned build for gfx950: the same graph as the direct build, with the
// per-k-mer claims and counts moved from device-scope atomics (which MI355X
// executes past the per-XCD L2, at most ~27 G/s) into LDS.
//
// Each instance's table is cut into segments of kSegSlots slots; a key's
// segment is chosen by the top bits of its image (a bijection of the key)
// and its home slot inside the segment by its low bits.  The windows of all
// reads become records (image << 3 | sink << 2 | letter: 8 bytes for
// k <= 31; 16 bytes for 33 <= k <= 63, whose image takes two words) that are
// partitioned by segment in two passes:
//
//   pass 1  windows -> records grouped by level-1 bucket (d1 buckets per
//           instance, each covering `fan` consecutive segments)
//   pass 2  records of each bucket -> records grouped by segment
//
// Every pass is count -> flat exclusive scan -> scatter, over chunks of
// consecutive tiles.  The count kernel writes one histogram per chunk, laid
// out bucket-major and chunk-minor, so one exclusive scan over the whole
// histogram array gives each (chunk, bucket) its output offset directly; the
// scatter kernel sorts each tile of its chunk by bucket in LDS and appends
// each bucket's run to the chunk's run of that bucket, so a chunk writes one
// contiguous run per bucket however many tiles it spans.
//
// Finally one workgroup owns each segment: it stages the segment in LDS,
// finds or claims each record's vertex with a 64-bit LDS compare-and-swap
// (the paper's CAS, Algorithm 1, on the segment's slots), raises its counter
// with a 32-bit LDS atomic add (Algorithm 3's increment), and writes the
// segment back.  No global atomic is issued per k-mer; a segment is only ever
// touched by its owner, so plain loads and stores move it.
#include "dbg_device.h"

#include <algorithm>

namespace dbgk {
namespace {

constexpr uint32_t kSkipMask = kErrBase | kErrInval | kErrRange | kErrSkip;
static_assert((kSegSlots & (kSegSlots - 1)) == 0, "segment size must be a power of two");
static_assert(kBinTile <= 4096 && kRefTile <= 4096, "ranks are packed into 12 bits");
static_assert(kMaxD1 % kBinBlock == 0 && kMaxFan % kRefBlock == 0, "bucket scans");

__device__ __forceinline__ uint64_t lds_load64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_add32(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Long keys (33 <= k <= 63, so K < 2^124) as (kh = K >> 64 < 2^60, kl):
// two Feistel rounds give the image (ih < 2^60, il): il = kl ^ mix64(kh),
// then ih = kh ^ (il * kWideMul) >> 4.  ih takes the place of a short key's
// image (its top bits are the segment digits) and il's low bits are the
// home slot; each round undoes itself given the other half.
constexpr uint64_t kWideMul = 0xD1B54A32D192ED03ull;  // odd

__device__ __forceinline__ void wide_image(uint64_t kh, uint64_t kl, uint64_t &ih, uint64_t &il) {
    il = kl ^ mix64(kh);
    ih = kh ^ ((il * kWideMul) >> 4);
}

__device__ __forceinline__ void wide_key(uint64_t ih, uint64_t il, uint64_t &kh, uint64_t &kl) {
    kh = ih ^ ((il * kWideMul) >> 4);
    kl = il ^ mix64(kh);
}

// A window record: RW = 1, one word image << 3 | sink << 2 | letter; RW = 2
// (long keys), that word built from ih, then il.  Both start with the word
// that carries the segment digits and the flags.
template <uint32_t RW> struct RecOf;
template <> struct RecOf<1> {
    using T = uint64_t;
    static __device__ __forceinline__ uint64_t head(uint64_t r) { return r; }
    static __device__ __forceinline__ uint64_t none() { return ~0ull; }
};
template <> struct RecOf<2> {
    using T = ulonglong2;
    static __device__ __forceinline__ uint64_t head(ulonglong2 r) { return r.x; }
    static __device__ __forceinline__ ulonglong2 none() { return make_ulonglong2(~0ull, 0); }
};


// Last index i in [0, n) with base(i) <= x, for a non-decreasing base.
template <typename F>
__device__ __forceinline__ uint64_t last_le(uint64_t n, uint64_t x, F base) {
    uint64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (base(mid) <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// XCD-aware order of a persistent loop over n tiles.  Workgroups are
// dispatched to the 8 XCDs round-robin (workgroup b runs on XCD b % 8), and
// each XCD has its own L2.  Tile t's output runs sit next to tile t+1's, so
// giving every XCD one contiguous range of tiles lets its L2 merge the
// partial cache lines that neighbouring tiles write.  Only speed depends on
// the dispatch order; every tile is visited exactly once for any grid.
struct XcdTiles {
    uint64_t next, end, step;
    __device__ XcdTiles(uint64_t n) {
        const uint32_t G = gridDim.x, b = blockIdx.x;
        const uint32_t groups = G >= 8 ? 8 : 1;
        const uint32_t g = b % groups;
        const uint32_t per_group = (G + groups - 1 - g) / groups;  // workgroups in group g
        const uint64_t span = (n + groups - 1) / groups;
        const uint64_t lo = min((uint64_t)g * span, n);
        next = lo + b / groups;
        end = min(lo + span, n);
        step = per_group;
    }
    __device__ bool valid() const { return next < end; }
    __device__ void advance() { next += step; }
};

// ---------------------------------------------------------------- window decode

// Reads of one pass-1 tile staged in LDS (all windows of the tile belong to
// one instance).
struct ReadStage {
    uint64_t ws[kMapReads + 1];
    uint64_t delta[kMapReads];
    uint64_t r0;
    uint32_t R;
};

// Stage the reads from r0 (the read holding the tile's first window) on,
// up to re.  Contains barriers: call from the whole block.
__device__ void stage_reads(ReadStage &S, const uint64_t *ws, const uint64_t *off, uint64_t off0,
                            uint64_t r0, uint64_t re) {
    if (threadIdx.x == 0) {
        S.r0 = r0;
        S.R = (uint32_t)min<uint64_t>(kMapReads, re - r0);
    }
    __syncthreads();
    const uint32_t R = S.R;
    for (uint32_t i = threadIdx.x; i <= R; i += blockDim.x) {
        const uint64_t r = r0 + i;
        const uint64_t wr = ws[r];
        S.ws[i] = wr;
        if (i < R) S.delta[i] = off[r] - off0 - wr;
    }
    __syncthreads();
}

// Local index of the staged read holding window w, found by binary search;
// kMapReads + 1 if w lies past the staged reads.
__device__ __forceinline__ uint32_t staged_read(const ReadStage &S, uint64_t w) {
    const uint32_t R = S.R;
    if (w >= S.ws[R]) return kMapReads + 1;
    uint32_t lo = 0, hi = R;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (S.ws[mid] <= w) lo = mid; else hi = mid;
    }
    return lo;
}

// Window range end and base delta (position = window + delta) of a read.
struct ReadPos {
    uint64_t wr1;    // one past the read's last window
    uint64_t delta;  // off[r] - off[0] - ws[r]
};

__device__ __forceinline__ ReadPos locate_read(const ReadStage &S, const uint64_t *ws,
                                               const uint64_t *off, uint64_t off0, uint64_t re,
                                               uint64_t w) {
    const uint32_t lo = staged_read(S, w);
    if (lo <= kMapReads && lo < S.R) return ReadPos{S.ws[lo + 1], S.delta[lo]};
    uint64_t glo = S.r0 + S.R, ghi = re;  // ws[glo] <= w < ws[ghi]
    while (ghi - glo > 1) {
        const uint64_t mid = (glo + ghi) >> 1;
        if (ws[mid] <= w) glo = mid; else ghi = mid;
    }
    return ReadPos{ws[glo + 1], off[glo] - off0 - ws[glo]};
}

// A thread's position among the reads: the window range end and base delta
// of the read holding its current window, and that read's staged index
// (kMapReads + 1 when it lies past the staged reads).
struct ReadCursor {
    uint64_t wr1, delta;
    uint32_t ri;
};

__device__ __forceinline__ ReadCursor first_read(const ReadStage &S, const uint64_t *ws, const uint64_t *off,
                                                 uint64_t off0, uint64_t re, uint64_t w) {
    const uint32_t lo = staged_read(S, w);
    if (lo < S.R) return ReadCursor{S.ws[lo + 1], S.delta[lo], lo};
    const ReadPos rp = locate_read(S, ws, off, off0, re, w);
    return ReadCursor{rp.wr1, rp.delta, kMapReads + 1};
}

// Window w (>= c.wr1) lies in a later read: the staged reads that follow are
// stepped through (reads shorter than k have no window), so crossing into
// the next read costs one or two LDS loads instead of a search.
__device__ __forceinline__ void next_read(ReadCursor &c, const ReadStage &S, const uint64_t *ws,
                                          const uint64_t *off, uint64_t off0, uint64_t re, uint64_t w) {
    if (c.ri < S.R) {
        uint32_t i = c.ri + 1;
        while (i < S.R && S.ws[i + 1] <= w) ++i;
        if (i < S.R) {
            c = ReadCursor{S.ws[i + 1], S.delta[i], i};
            return;
        }
    }
    const ReadPos rp = locate_read(S, ws, off, off0, re, w);
    c = ReadCursor{rp.wr1, rp.delta, kMapReads + 1};
}

// 64 bits starting `o` bits into the 192-bit big-endian word triple (o < 128).
__device__ __forceinline__ uint64_t funnel3(uint64_t a, uint64_t b, uint64_t c, uint32_t o) {
    if (o >= 64) {
        a = b;
        b = c;
        o -= 64;
    }
    return o ? (a << o) | (b >> (64 - o)) : a;
}

// Rolling window state of one-word keys (k <= 31).  Consecutive windows of a
// read share all but one base: the key of the next window is the key shifted
// by one base, with the window's letter shifted in and its first base shifted
// out.  The image multiplies the key by kKeyMul modulo 2^60, so with
// x = key * kKeyMul mod 2^60 the next window's x is
//   4 x + letter * kKeyMul - first * (4^(k-1) * kKeyMul)  (mod 2^60),
// one shift-add of a table entry indexed by (first base, letter).  F holds
// the 32 bases from the window's first on, L the 32 from its letter on, so a
// thread rolls through up to 32 windows of one read without touching the
// packed reads again.
struct Roll {
    uint64_t F, L, x;
};

// The state of the window whose first base is at position p of the packed
// reads.  kshift = 64 - 2 (k - 1).
__device__ __forceinline__ Roll roll_at(const uint64_t *__restrict__ packed, uint64_t p, uint32_t k,
                                        uint32_t kshift) {
    const uint64_t wb = p >> 5;
    const uint64_t a = packed[wb], b = packed[wb + 1], c = packed[wb + 2];
    const uint32_t o = (uint32_t)(p & 31) * 2;  // o + 2 (k - 1) <= 122: inside the triple
    const uint64_t F = funnel3(a, b, c, o);
    return Roll{F, funnel3(a, b, c, o + 2 * (k - 1)), ((F >> kshift) * kKeyMul) & kKey60};
}

// Table entry (first << 2 | letter): letter * kKeyMul - first * 4^(k-1) * kKeyMul, mod 2^60.
__device__ __forceinline__ uint64_t roll_entry(uint32_t e, uint32_t k) {
    const uint64_t out = (kKeyMul << (2 * (k - 1))) & kKey60;
    return ((uint64_t)(e & 3u) * kKeyMul - (uint64_t)(e >> 2) * out) & kKey60;
}

__device__ __forceinline__ void roll_next(Roll &r, const uint64_t *s_roll) {
    const uint32_t e = (uint32_t)(r.F >> 62) << 2 | (uint32_t)(r.L >> 62);
    r.F <<= 2;
    r.L <<= 2;
    r.x = ((r.x << 2) + s_roll[e]) & kKey60;
}

// Scatter tiles count with tagged counters: s_cnt[j] starts at j << rb, so
// the value a record's fetch-add returns is its tag, bucket << rb | rank, and
// bucket j's count is s_cnt[j] - (j << rb) (rb = 12 for tiles of 4096
// records, 14 for 16384).  Records past the end of a tile add into one extra
// counter, so the adds of a thread's records issue without branches.
//
// Exclusive prefix of the counts of s_cnt[0..n) in place (whole block): the
// starts are left in s_cnt, and s_gbase[j] = gbase(j) - start.
template <typename G>
__device__ void bucket_starts(uint32_t *s_cnt, uint64_t *s_gbase, uint32_t n, uint32_t rb, G gbase) {
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t j0 = threadIdx.x * per;
    uint64_t sum = 0;
    for (uint32_t q = 0; q < per; ++q)
        if (j0 + q < n) sum += s_cnt[j0 + q] - ((j0 + q) << rb);
    uint64_t total;
    uint64_t pre = block_exclusive_scan(sum, &total);
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t j = j0 + q;
        if (j < n) {
            const uint32_t c = s_cnt[j] - (j << rb);
            s_cnt[j] = (uint32_t)pre;
            s_gbase[j] = gbase(j) - pre;
            pre += c;
        }
    }
}

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

// ---------------------------------------------------------------- line-staged scatters
//
// A scatter chunk writes each of its runs (one per bucket or segment) in
// order, a tile at a time, and a tile adds only a few records to each run
// when there are many runs (about 6 per run for 713 runs and 4096 records).
// Stored as they come, those pieces cover parts of 128-byte lines, and HBM
// takes pieces of lines far more slowly than whole ones: appending 6-record
// pieces to 713 runs moves 12.8 GB in 12 ms where whole aligned lines (or a
// plain copy) take 5.5 ms, and 64-byte pieces 7.2 ms.  A staged scatter
// keeps each run's records that do not yet fill their line in LDS (s_stg,
// one line per run) and stores only whole lines, each by one group of
// consecutive lanes in one instruction; the chunk's end stores what is left.
// Only the first and last line of a chunk's run can then be partial.
//
// Per run j between tiles: s_front[j] is the global position of the run's
// next record, f, and s_cc[j] the number of records waiting in s_stg, at
// global [f - cc, f), all inside the line holding f; a waiting record sits
// at s_stg[j * L + (position mod L)].
constexpr uint32_t kLineBytes = 128;

// Scatter shapes.  A plain scatter (512 threads, tiles of 4096 records)
// stores each tile's runs as it sorts them; a staged one (1024 threads, one
// workgroup per CU when it stages 713 runs) stores whole lines only; a big
// one stores runs as they come from tiles two to four times larger.  Big
// tiles hold 128 KB of records (16384 one-word or 8192 two-word records;
// 1024 threads, one workgroup per CU), except in the first scatter of
// one-word records: 64 KB there (8192 records, 512 threads, 16 windows
// each, two workgroups per CU), where a second workgroup's waves help the
// window decode more than longer runs help the stores, up to a few hundred
// buckets.  kShapeBigWide is the 128 KB form of the first scatter's big
// tiles for one-word records (16384 records, 1024 threads, one workgroup
// per CU): it writes runs twice as long, which pays where the first pass
// has many buckets.  The shape codes of dbg_config and dbg_stats are these
// plus one.
enum : uint32_t { kShapeTile = 0, kShapeStaged = 1, kShapeBig = 2, kShapeBigWide = 3 };

__host__ __device__ constexpr bool is_big(uint32_t shape) { return shape == kShapeBig || shape == kShapeBigWide; }

__host__ __device__ constexpr uint32_t big_tile_bytes(uint32_t shape, bool first, uint32_t rw) {
    return first && rw == 1 && shape != kShapeBigWide ? 64u * 1024u : 128u * 1024u;
}

__host__ __device__ constexpr uint32_t scatter_block(uint32_t shape, bool first, uint32_t rw) {
    return shape == kShapeStaged || (is_big(shape) && big_tile_bytes(shape, first, rw) == 128u * 1024u) ? 1024u : 512u;
}

template <uint32_t SHAPE, uint32_t RW, bool FIRST>
struct ScatterShape {
    static constexpr uint32_t block = scatter_block(SHAPE, FIRST, RW);
    static constexpr uint32_t tile = is_big(SHAPE) ? big_tile_bytes(SHAPE, FIRST, RW) / (8u * RW) : 4096u;
    static constexpr uint32_t per = tile / block;  // records per thread
    static constexpr uint32_t rb = tile == 16384u ? 14u : tile == 8192u ? 13u : 12u;  // rank bits of a tag
    static_assert((1u << rb) == tile, "a tag's rank holds a tile");
};
constexpr uint32_t kStageBlock = scatter_block(kShapeStaged, false, 1);

// Windows per thread of a first-pass count of one-word keys: a count holds
// no records, so its threads roll through more windows than a scatter's, and
// the tile's fixed costs (staging its reads, locating each thread's first
// window) spread over more of them.  The longer form needs chunks of four
// planning tiles or more to fill its tiles; chunks are that long where the
// first scatter runs big tiles.
constexpr uint32_t kCountWindows = 16;
constexpr uint32_t kCountWindowsLong = 32;

template <typename R>
struct Lines {
    static constexpr uint32_t L = kLineBytes / (uint32_t)sizeof(R);  // records per line
    static constexpr uint32_t kShift = L == 16 ? 4 : 3;
    static_assert((1u << kShift) == L, "records per line");
};

// Dynamic LDS of a staged scatter with n runs and tiles of `tile` records:
// s_cnt[n + 1], s_front[n], s_rec[tile], s_stg[n lines], s_pack[n], s_cc[n]
// and the line-to-run table s_lrun (the lines a tile completes: at most
// tile / L + n, one per run beyond the tile's own records).
struct StageLayout {
    uint32_t front, rec, stg, pack, cc, lrun, bytes;
};

template <typename R>
__host__ __device__ inline StageLayout stage_layout(uint32_t n, uint32_t tile) {
    StageLayout o;
    o.front = align16(4 * (n + 1));
    o.rec = o.front + align16(8 * n);
    o.stg = o.rec + (uint32_t)sizeof(R) * tile;
    o.pack = o.stg + kLineBytes * n;
    o.cc = o.pack + align16(4 * n);
    o.lrun = o.cc + align16(n);
    o.bytes = o.lrun + align16(2 * (tile / Lines<R>::L + n + 1));
    return o;
}

// After a tile's tagged counts: s_cnt[j] becomes run j's start in the sorted
// tile; the lines the tile completes are numbered run by run (run j's from
// lp on: its line holding f, if the tile fills it, and every whole line
// after), s_lrun maps a line number to its run, and s_pack[j] packs start |
// lp << 13 | cc << 24.  *s_nlines receives the tile's line count.  Whole block.
template <typename R>
__device__ void stage_starts(uint32_t *s_cnt, const uint64_t *s_front, const uint8_t *s_cc, uint32_t *s_pack,
                             uint16_t *s_lrun, uint32_t *s_nlines, uint32_t n) {
    constexpr uint32_t S = Lines<R>::kShift;
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t j0 = threadIdx.x * per;
    uint64_t sum = 0;  // records in the low half, lines in the high half
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t j = j0 + q;
        if (j < n) {
            const uint32_t c = s_cnt[j] - (j << 12);  // staged tiles: 4096 records
            const uint64_t f = s_front[j];
            sum += c | ((((f + c) >> S) - (f >> S)) << 32);
        }
    }
    uint64_t total;
    uint64_t pre = block_exclusive_scan(sum, &total);
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t j = j0 + q;
        if (j >= n) break;
        const uint32_t c = s_cnt[j] - (j << 12);
        const uint64_t f = s_front[j];
        const uint32_t nl = (uint32_t)(((f + c) >> S) - (f >> S));
        const uint32_t start = (uint32_t)pre, lp = (uint32_t)(pre >> 32);
        s_cnt[j] = start;
        s_pack[j] = start | lp << 13 | (uint32_t)s_cc[j] << 24;
        for (uint32_t i = 0; i < nl; ++i) s_lrun[lp + i] = (uint16_t)j;
        pre += c | (uint64_t)nl << 32;
    }
    if (threadIdx.x == 0) *s_nlines = (uint32_t)(total >> 32);
}

// Store the tile's completed lines: L consecutive lanes per line, each
// record from the waiting ones (below f) or the sorted tile.  Positions of
// the run's first line below its start (another chunk's) are skipped.
template <typename R>
__device__ void stage_write(const uint16_t *s_lrun, const uint32_t *s_pack, const uint64_t *s_front, const R *s_stg,
                            const R *s_rec, uint32_t nlines, R *__restrict__ out) {
    constexpr uint32_t L = Lines<R>::L, S = Lines<R>::kShift;
    for (uint32_t idx = threadIdx.x; idx < nlines * L; idx += blockDim.x) {
        const uint32_t k = idx >> S, e = idx & (L - 1);
        const uint32_t j = s_lrun[k];
        const uint32_t pk = s_pack[j];
        const uint32_t start = pk & 0x1fffu, lp = (pk >> 13) & 0x7ffu, cc = pk >> 24;
        const uint64_t f = s_front[j];
        const uint64_t pos = (((f >> S) + (k - lp)) << S) | e;
        if (pos + cc >= f) out[pos] = pos < f ? s_stg[j * L + e] : s_rec[start + (uint32_t)(pos - f)];
    }
}

// After the lines are stored: the tile's records past its last whole line
// wait in s_stg, and each run's frontier moves to its end.  tile_n is the
// tile's record count.  Whole block, no barrier.
template <typename R>
__device__ void stage_tail(const uint32_t *s_cnt, uint64_t *s_front, uint8_t *s_cc, R *s_stg, const R *s_rec,
                           uint32_t n, uint32_t tile_n) {
    constexpr uint32_t L = Lines<R>::L;
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
        const uint32_t start = s_cnt[j], c = (j + 1 < n ? s_cnt[j + 1] : tile_n) - start;
        const uint64_t f = s_front[j], F = f + c, line = F & ~(uint64_t)(L - 1);
        for (uint64_t pos = line > f ? line : f; pos < F; ++pos)
            s_stg[j * L + (uint32_t)(pos & (L - 1))] = s_rec[start + (uint32_t)(pos - f)];
        const uint64_t first = f - s_cc[j];  // the first waiting record before the tile
        s_cc[j] = (uint8_t)(F - (line > first ? line : first));
        s_front[j] = F;
    }
}

// The chunk's end: every run's waiting records are stored (the run's last
// line, partial), L lanes per run.  Whole block, no barrier.
template <typename R>
__device__ void stage_flush(const uint64_t *s_front, const uint8_t *s_cc, const R *s_stg, uint32_t n,
                            R *__restrict__ out) {
    constexpr uint32_t L = Lines<R>::L, S = Lines<R>::kShift;
    for (uint32_t idx = threadIdx.x; idx < n * L; idx += blockDim.x) {
        const uint32_t j = idx >> S, e = idx & (L - 1);
        const uint64_t f = s_front[j], pos = (f & ~(uint64_t)(L - 1)) | e;
        if (pos < f && pos + s_cc[j] >= f) out[pos] = s_stg[j * L + e];
    }
}

// ---------------------------------------------------------------- plan

// Per instance: its window range, pass-1 tiles and chunks, histogram and
// bucket bases.  The chunk length (tiles) is max(min_chunk, floor(tiles / target))
// over the whole launch; chunks never span instances.  An instance that
// failed validation (or whose k-mer total would overflow a counter) gets no
// tiles, so it produces no records.
__global__ void k_bin_plan(const PassArgs *__restrict__ args, const Instance *inst, const uint64_t *ws,
                           InstStatus *st, BinPlan *plan, BinTotals *tot, uint32_t target, uint32_t min_chunk) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t m = args->m;
    uint64_t all_tiles = 0;
    for (uint32_t i = 0; i < m; ++i) {
        const Instance &in = inst[i];
        uint32_t e = st[i].err;
        if (!(e & kErrRange) && in.prior_inserts + st[i].inserts > 0xffffffffull) {
            atomic_or_u32(&st[i].err, kErrRange);
            e |= kErrRange;
        }
        const uint64_t wb = ws[in.read_begin], we = ws[in.read_end];
        if (!(e & kSkipMask) && we > wb) all_tiles += (we - wb + kBinTile - 1) / kBinTile;
    }
    const uint64_t chunk = max<uint64_t>(min_chunk, all_tiles / max(target, 1u));
    uint64_t tiles = 0, chunks = 0, hist = 0, buckets = 0;
    for (uint32_t i = 0; i < m; ++i) {
        const Instance &in = inst[i];
        const uint32_t e = st[i].err;
        BinPlan pl;
        pl.w_begin = ws[in.read_begin];
        pl.w_end = ws[in.read_end];
        const bool run = !(e & kSkipMask) && pl.w_end > pl.w_begin;
        pl.tiles = run ? (pl.w_end - pl.w_begin + kBinTile - 1) / kBinTile : 0;
        pl.chunks = (pl.tiles + chunk - 1) / chunk;
        pl.tile_base = tiles;
        pl.chunk_base = chunks;
        pl.hist_base = hist;
        pl.bucket_base = buckets;
        tiles += pl.tiles;
        chunks += pl.chunks;
        hist += (uint64_t)in.d1 * pl.chunks;
        buckets += in.d1;
        plan[i] = pl;
    }
    tot->tiles1 = tiles;
    tot->chunk1 = chunk;
    tot->chunks1 = chunks;
    tot->hist1_len = hist;
    tot->buckets = buckets;
    tot->chunk2 = 1;
    tot->chunks2 = 0;
    tot->hist2_len = 0;
    tot->records = 0;
}

// First read of every pass-1 tile: read r writes the tiles whose first
// window falls among its windows.
__global__ void k_tile_reads(const PassArgs *__restrict__ args, const Instance *__restrict__ inst,
                             const uint64_t *__restrict__ ws, const BinPlan *__restrict__ plan,
                             uint64_t *__restrict__ tile_read1, uint64_t tiles_cap) {
    const uint32_t m = args->m;
    const uint64_t n = args->n_reads;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const uint64_t a = ws[r], z = ws[r + 1];
        if (z == a) continue;
        const uint32_t i = m == 1 ? 0u : instance_of_read(inst, m, r);
        const BinPlan pl = plan[i];
        if (!pl.tiles) continue;  // instance not built in this launch
        uint64_t tl = (a - pl.w_begin + kBinTile - 1) / kBinTile;
        for (; pl.w_begin + tl * kBinTile < z; ++tl)
            if (pl.tile_base + tl < tiles_cap) tile_read1[pl.tile_base + tl] = r;
    }
}

// ---------------------------------------------------------------- pass 1

// Dynamic LDS of the pass-1 kernels: s_cnt[d1_max + 1] (+ s_gbase[d1_max]
// and s_rec[kBinTile] when scattering; the write-out recomputes each
// record's bucket rather than keep it in LDS beside the record).
__host__ __device__ inline uint32_t bin_lds_bytes(uint32_t d1_max, bool scatter, uint32_t rw = 1,
                                                 uint32_t shape = kShapeTile) {
    uint32_t b = align16(4 * (d1_max + 1));
    if (scatter) b += align16(8 * d1_max) + (is_big(shape) ? big_tile_bytes(shape, true, rw) : 8 * rw * kBinTile);
    return b;
}

// Pass 1, per chunk of tiles.  A thread takes WPT consecutive windows of a
// tile (kBinPerThread in plain tiles, 4 in the staged scatter's 1024-thread
// workgroups, 16 in big tiles, CW in a count): it finds their read once.
// One-word keys then roll from window to window (Roll above), with the
// thread's first read boundary prepared before the loop; a thread whose
// windows cross two boundaries, and plain scatter tiles, load three packed
// words and slide through them, a funnel shift per window.  The next
// read's bases follow the current read's in the packed array, so a window
// that starts another read (k - 2 bases further on) is found in the staged
// reads and mostly stays inside the three words.  Long keys (RW = 2) take
// each window's 128 bits from the packed array directly.
//
// Counting, a chunk's histogram accumulates in LDS over its tiles and is
// written once.  Scattering, s_gbase[j] holds the global position where the
// chunk's run of bucket j continues: each tile sorts its records by bucket
// in LDS, writes bucket j's records at s_gbase[j] on, and advances s_gbase[j]
// by their number; staged, it stores whole lines only (line-staged scatters
// above) and s_gbase[j] is the run's frontier throughout.  A big tile (and
// a count tile of CW windows a thread) is two or four consecutive planning
// tiles of the chunk (fewer at its end).
template <bool SCATTER, uint32_t RW, uint32_t SHAPE = kShapeTile, uint32_t CW = kCountWindows>
__global__ __launch_bounds__(scatter_block(SHAPE, true, RW)) __attribute__((amdgpu_waves_per_eu(SHAPE != kShapeTile ? 4 : RW == 2 ? 4 : SCATTER ? 6 : 8))) void k_bin(const PassArgs *__restrict__ args,
                                                  const Instance *__restrict__ inst,
                                                  const uint64_t *__restrict__ packed,
                                                  const uint64_t *__restrict__ ws,
                                                  const BinPlan *__restrict__ plan,
                                                  const BinTotals *__restrict__ tot,
                                                  uint32_t *__restrict__ hist1,
                                                  const uint64_t *__restrict__ scan1,
                                                  uint64_t *__restrict__ rec1w,
                                                  const uint64_t *__restrict__ tile_read1,
                                                  uint32_t d1_max) {
    using R = typename RecOf<RW>::T;
    using Sh = ScatterShape<SHAPE, RW, true>;
    constexpr bool STAGED = SHAPE == kShapeStaged;
    // rolling window decode (one-word keys), except in plain scatter tiles,
    // whose records and tags leave no registers for its state
    constexpr bool ROLL = RW == 1 && !(SCATTER && SHAPE == kShapeTile);
    // a count holds no records, so its threads roll through more windows
    constexpr uint32_t WPT = SCATTER || !ROLL ? Sh::per : CW;
    constexpr uint32_t TILE = WPT * Sh::block, RB = Sh::rb, TPS = TILE / kBinTile;
    static_assert(WPT * Sh::block == TILE && TILE % kBinTile == 0, "a tile is one window per thread slot");
    static_assert(SHAPE == kShapeTile || SCATTER, "counting uses plain tiles");
    __shared__ ReadStage S;
    __shared__ uint32_t s_nlines;
    __shared__ uint64_t s_roll[16];  // one-word keys: the rolling table of the tile's k
    extern __shared__ __align__(16) unsigned char s_dyn[];
    const StageLayout lay = stage_layout<R>(d1_max, kBinTile);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(s_dyn);
    uint64_t *s_gbase = reinterpret_cast<uint64_t *>(s_dyn + align16(4 * (d1_max + 1)));
    R *s_rec = reinterpret_cast<R *>(s_dyn + align16(4 * (d1_max + 1)) + align16(8 * d1_max));  // 16-byte aligned
    R *s_stg = reinterpret_cast<R *>(s_dyn + lay.stg);  // STAGED only, from here on
    uint32_t *s_pack = reinterpret_cast<uint32_t *>(s_dyn + lay.pack);
    uint8_t *s_cc = reinterpret_cast<uint8_t *>(s_dyn + lay.cc);
    uint16_t *s_lrun = reinterpret_cast<uint16_t *>(s_dyn + lay.lrun);
    R *rec1 = reinterpret_cast<R *>(rec1w);
    const uint32_t tid = threadIdx.x;
    const uint32_t m = args->m;
    const uint64_t *__restrict__ off = args->off;
    const uint64_t chunks = tot->chunks1, chunk = tot->chunk1;
    const uint64_t off0 = off[0];
    // One flat loop over the tiles of this workgroup's chunks: only the chunk
    // cursor and the tile index t carry from one tile to the next (a nested
    // chunk/tile loop keeps the chunk's values live across the decode, which
    // then spills).  Each tile looks its chunk up again.
    XcdTiles it(chunks);
    for (uint32_t t = 0; it.valid();) {
        const uint64_t gc = it.next;
        const uint32_t i = (uint32_t)last_le(m, gc, [&](uint64_t j) { return plan[j].chunk_base; });
        const Instance &in = inst[i];
        const uint32_t d1 = in.d1;
        const uint32_t kshift = 64 - 2 * (in.k - 1), lshift = 62 - 2 * (in.k - 1);
        const uint64_t read_end = in.read_end;
        const uint64_t c = gc - plan[i].chunk_base;
        const uint64_t tbeg = c * chunk;
        const uint32_t nt = (uint32_t)(min(tbeg + chunk, plan[i].tiles) - tbeg);
        if (t == 0) {  // the chunk starts
            if (!SCATTER) {
                for (uint32_t j = tid; j < d1; j += blockDim.x) s_cnt[j] = 0u;
            } else {
                const uint64_t *col = scan1 + plan[i].hist_base + c;
                const uint64_t stride = plan[i].chunks;
                for (uint32_t j = tid; j < d1; j += blockDim.x) {
                    s_gbase[j] = col[(uint64_t)j * stride];
                    if (STAGED) s_cc[j] = 0;
                }
            }
        }
        {
            const uint64_t w0 = plan[i].w_begin + (tbeg + t) * kBinTile;
            const uint64_t w_end = min(plan[i].w_begin + (tbeg + nt) * kBinTile, plan[i].w_end);  // the chunk's
            const uint32_t n_in = (uint32_t)(min(w0 + TILE, w_end) - w0);
            if (SCATTER)
                for (uint32_t j = tid; j <= d1; j += blockDim.x) s_cnt[j] = j << RB;
            if (ROLL && tid < 16) s_roll[tid] = roll_entry(tid, in.k);
            stage_reads(S, ws, off, off0, tile_read1[plan[i].tile_base + tbeg + t], read_end);

            R rec[WPT];
            uint32_t tag[WPT];  // scatter: bucket << RB | rank (bucket d1: past the end)
            const uint32_t j0 = tid * WPT;
#pragma unroll
            for (uint32_t q = 0; q < WPT; ++q) tag[q] = d1 << RB;
            if (j0 < n_in) {
                uint64_t w = w0 + j0;
                ReadCursor rp = first_read(S, ws, off, off0, read_end, w);
                bool rolled = false;
                if constexpr (ROLL) {
                    static_assert(WPT <= 32, "F and L hold the bases of 32 windows");
                    const uint32_t k = in.k, jend = min(j0 + WPT, n_in);
                    // read ends relative to w0, capped past the tile: 32-bit compares
                    auto rel_end = [&](uint64_t wr1) { return (uint32_t)min<uint64_t>(wr1 - w0, n_in + 1u); };
                    Roll st = roll_at(packed, w + rp.delta, k, kshift);
                    Roll st2 = st;  // the next read's first window, if one starts among this thread's
                    const uint32_t e1 = rel_end(rp.wr1);
                    uint32_t e2 = e1;
                    if (e1 < jend) {
                        ReadCursor c = rp;
                        next_read(c, S, ws, off, off0, read_end, rp.wr1);
                        st2 = roll_at(packed, rp.wr1 + c.delta, k, kshift);
                        e2 = rel_end(c.wr1);
                    }
                    if (e2 >= jend) {  // at most one read boundary: every window rolls
                        rolled = true;
#pragma unroll
                        for (uint32_t q = 0; q < WPT; ++q) {
                            const uint32_t j = j0 + q;
                            if (j >= n_in) break;
                            if (j == e1) st = st2;
                            const uint64_t sink = j + 1 == e1 || j + 1 == e2 ? 4u : 0u;
                            const uint64_t img = st.x ^ (st.x >> 30);  // the key's image
                            const uint64_t head = (img << 3) | sink | (uint32_t)(st.L >> 62);
                            rec[q] = head;
                            const uint32_t bk = bucket_of(image_top(img), d1);
                            if (SCATTER) {
                                tag[q] = lds_add32(&s_cnt[bk], 1u);  // the tag itself: no use until placement
                            } else {
                                __hip_atomic_fetch_add(&s_cnt[bk], 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                            }
                            roll_next(st, s_roll);
                        }
                    }
                }
                if (!rolled) {  // reads shorter than a thread's windows, long keys, plain scatter tiles
                    uint64_t p = w + rp.delta;
                    uint64_t wbase = p >> 5;
                    uint64_t a = 0, b = 0, cc = 0;
                    if (RW == 1) {
                        a = packed[wbase];
                        b = packed[wbase + 1];
                        cc = packed[wbase + 2];
                    }
                    // beside the rolling decode this loop may stay rolled (records
                    // then go through indexed registers, in a path long reads never take)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
#pragma unroll
                    for (uint32_t q = 0; q < WPT; ++q) {
                        if (j0 + q >= n_in) break;
                        if (w >= rp.wr1) {  // the next window starts another read
                            next_read(rp, S, ws, off, off0, read_end, w);
                            p = w + rp.delta;
                            // the words must hold this and the remaining windows' first
                            // bases at offsets below 64 (without a crossing a thread's
                            // offsets stay below 32 + WPT)
                            if (RW == 1 && p - 32 * wbase + (WPT - 1 - q) > 63) {
                                wbase = p >> 5;
                                a = packed[wbase];
                                b = packed[wbase + 1];
                                cc = packed[wbase + 2];
                            }
                        }
                        const uint64_t sink = w + 1 == rp.wr1 ? 4u : 0u;
                        uint64_t head;
                        if constexpr (RW == 1) {
                            const uint64_t v = funnel3(a, b, cc, (uint32_t)(p - 32 * wbase) * 2);
                            head = (key_image(v >> kshift) << 3) | sink | ((uint32_t)(v >> lshift) & 3u);
                            rec[q] = head;
                        } else {
                            uint64_t x0, x1, kh, kl, ih, il;
                            uint32_t letter;
                            bases128_at(packed, p, x0, x1);
                            wide_window(x0, x1, in.k - 1, kh, kl, letter);
                            wide_image(kh, kl, ih, il);
                            head = (ih << 3) | sink | letter;
                            rec[q] = make_ulonglong2(head, il);
                        }
                        const uint32_t bk = bucket_of(image_top(head >> 3), d1);
                        if (SCATTER) {
                            tag[q] = lds_add32(&s_cnt[bk], 1u);  // the tag itself: no use until placement
                        } else {
                            __hip_atomic_fetch_add(&s_cnt[bk], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        ++w;
                        ++p;
                    }
#pragma clang diagnostic pop
                }
            }
            __syncthreads();  // the next tile's staging waits on this barrier
            if (SCATTER && STAGED) {
                stage_starts<R>(s_cnt, s_gbase, s_cc, s_pack, s_lrun, &s_nlines, d1);
                __syncthreads();
#pragma unroll
                for (uint32_t q = 0; q < WPT; ++q) {
                    const uint32_t bk = tag[q] >> RB;
                    if (bk == d1) continue;  // past the tile's end
                    s_rec[s_cnt[bk] + (tag[q] & ((1u << RB) - 1))] = rec[q];
                }
                __syncthreads();
                stage_write<R>(s_lrun, s_pack, s_gbase, s_stg, s_rec, s_nlines, rec1);
                __syncthreads();
                stage_tail<R>(s_cnt, s_gbase, s_cc, s_stg, s_rec, d1, n_in);
                __syncthreads();
            } else if (SCATTER) {
            // s_gbase[j] becomes the global position of the tile's first record
            // of bucket j minus its position in the sorted tile
            bucket_starts(s_cnt, s_gbase, d1, RB, [&](uint32_t j) { return s_gbase[j]; });
            __syncthreads();
#pragma unroll
            for (uint32_t q = 0; q < WPT; ++q) {
                const uint32_t bk = tag[q] >> RB;
                if (bk == d1) continue;  // past the tile's end
                const uint32_t pos = s_cnt[bk] + (tag[q] & ((1u << RB) - 1));
                s_rec[pos] = rec[q];
            }
            __syncthreads();
            for (uint32_t j = tid; j < n_in; j += blockDim.x) {
                const R r = s_rec[j];
                const uint32_t bk = bucket_of(image_top(RecOf<RW>::head(r) >> 3), d1);
                rec1[s_gbase[bk] + j] = r;
            }
            __syncthreads();
            // the runs continue after this tile's records: start of bucket j + 1
            for (uint32_t j = tid; j < d1; j += blockDim.x) s_gbase[j] += j + 1 < d1 ? s_cnt[j + 1] : n_in;
            __syncthreads();
            }
        }
        t += TPS;
        if (t < nt) continue;
        // the chunk ends
        if (!SCATTER) {
            uint32_t *col = hist1 + plan[i].hist_base + c;
            const uint64_t stride = plan[i].chunks;
            for (uint32_t j = tid; j < d1; j += blockDim.x) col[(uint64_t)j * stride] = s_cnt[j];
            __syncthreads();
        } else if (STAGED) {
            stage_flush<R>(s_gbase, s_cc, s_stg, d1, rec1);
            __syncthreads();
        }
        t = 0;
        it.advance();
    }
}

// ---------------------------------------------------------------- flat scan

// Exclusive scan of `*len` uint32 values into uint64 (out[len] = total).
constexpr uint32_t kFlatBlock = 256;
constexpr uint32_t kFlatPer = 4;
constexpr uint32_t kFlatChunk = kFlatBlock * kFlatPer;

__global__ __launch_bounds__(kFlatBlock) void k_flat_local(const uint32_t *__restrict__ in,
                                                          const uint64_t *len_ptr,
                                                          uint64_t *__restrict__ out,
                                                          uint64_t *__restrict__ partials) {
    const uint64_t n = *len_ptr;
    const uint64_t base = (uint64_t)blockIdx.x * kFlatChunk;
    if (base >= n) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0;
        return;
    }
    const uint64_t i0 = base + (uint64_t)threadIdx.x * kFlatPer;
    uint32_t v[kFlatPer];
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kFlatPer; ++j) {
        v[j] = i0 + j < n ? in[i0 + j] : 0u;
        sum += v[j];
    }
    uint64_t total;
    uint64_t pre = block_exclusive_scan(sum, &total);
#pragma unroll
    for (uint32_t j = 0; j < kFlatPer; ++j) {
        if (i0 + j < n) out[i0 + j] = pre;
        pre += v[j];
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_flat_partials(uint64_t *partials, uint64_t nb,
                                                       const uint64_t *len_ptr, uint64_t *out) {
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += blockDim.x) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? partials[i] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(v, &total);
        if (i < nb) partials[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) out[*len_ptr] = carry;
}

__global__ __launch_bounds__(kFlatBlock) void k_flat_add(const uint64_t *len_ptr, uint64_t *out,
                                                        const uint64_t *partials) {
    const uint64_t n = *len_ptr;
    const uint64_t base = (uint64_t)blockIdx.x * kFlatChunk;
    if (base >= n) return;
    const uint64_t add = partials[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < kFlatChunk; j += blockDim.x)
        if (base + j < n) out[base + j] += add;
}

// ---------------------------------------------------------------- pass 2

// Per level-1 bucket: its record range, pass-2 chunks and histogram base.
// The chunk length (tiles of kRefTile records) is max(min_chunk, floor(tiles /
// target)) over the launch; chunks never span buckets.
__device__ __forceinline__ Bucket bucket_range(const PassArgs *__restrict__ args, const Instance *__restrict__ inst,
                                               const BinPlan *__restrict__ plan, const uint64_t *__restrict__ scan1,
                                               uint64_t g) {
    const uint32_t i = (uint32_t)last_le(args->m, g, [&](uint64_t j) { return plan[j].bucket_base; });
    const Instance &in = inst[i];
    const BinPlan pl = plan[i];
    const uint32_t b = (uint32_t)(g - pl.bucket_base);
    Bucket B{0, 0, 0, 0, 0, 0, 0, 0, 0};
    B.start = scan1[pl.hist_base + (uint64_t)b * pl.chunks];
    B.size = scan1[pl.hist_base + (uint64_t)(b + 1) * pl.chunks] - B.start;
    B.inst = i;
    B.b = b;
    B.fan = min(in.fan, in.parts - b * in.fan);
    return B;
}

__global__ __launch_bounds__(1024) void k_refine_plan(const PassArgs *__restrict__ args,
                                                     const Instance *__restrict__ inst,
                                                     const BinPlan *__restrict__ plan,
                                                     const uint64_t *__restrict__ scan1,
                                                     BinTotals *tot, Bucket *__restrict__ buckets, uint32_t target,
                                                     uint32_t min_chunk) {
    const uint64_t G = tot->buckets;
    // tiles over all buckets, for the chunk length
    uint64_t my_tiles = 0;
    for (uint64_t g = threadIdx.x; g < G; g += blockDim.x)
        my_tiles += (bucket_range(args, inst, plan, scan1, g).size + kRefTile - 1) / kRefTile;
    uint64_t all_tiles;
    (void)block_exclusive_scan(my_tiles, &all_tiles);
    const uint64_t chunk = max<uint64_t>(min_chunk, all_tiles / max(target, 1u));
    uint64_t carry_c = 0, carry_h = 0;
    for (uint64_t base = 0; base < G; base += blockDim.x) {
        const uint64_t g = base + threadIdx.x;
        Bucket B{0, 0, 0, 0, 0, 0, 0, 0, 0};
        uint64_t nc = 0, nh = 0;
        if (g < G) {
            B = bucket_range(args, inst, plan, scan1, g);
            const uint64_t nt = (B.size + kRefTile - 1) / kRefTile;
            nc = (nt + chunk - 1) / chunk;
            nh = nc * B.fan;
        }
        uint64_t tc, th;
        const uint64_t pc = block_exclusive_scan(nc, &tc);
        const uint64_t ph = block_exclusive_scan(nh, &th);
        if (g < G) {
            B.chunks = nc;
            B.chunk_base = carry_c + pc;
            B.hist_base = carry_h + ph;
            buckets[g] = B;
        }
        carry_c += tc;
        carry_h += th;
    }
    if (threadIdx.x == 0) {
        tot->chunk2 = chunk;
        tot->chunks2 = carry_c;
        tot->hist2_len = carry_h;
        tot->records = scan1[tot->hist1_len];
    }
}

// Dynamic LDS of the pass-2 kernels: s_cnt[fan_max] (+ s_gbase[fan_max],
// s_rec[tile] and, for one-word records in plain tiles, s_child[kRefTile]
// when scattering).
__host__ __device__ inline uint32_t ref_lds_bytes(uint32_t fan_max, bool scatter, uint32_t rw = 1,
                                                 uint32_t shape = kShapeTile) {
    uint32_t b = align16(4 * (fan_max + 1));
    if (scatter) b += align16(8 * fan_max) + (is_big(shape) ? big_tile_bytes(shape, false, rw) : 8 * rw * kRefTile + (rw == 1 ? 2 * kRefTile : 0));
    return b;
}


// Load the records of one pass-2 tile: [r0, r0 + n) with n <= kRefTile, PT
// per thread (the order of records over threads is free: counts and ranks
// only need each record once).  One-word records go two per load.
template <typename R, uint32_t PT>
__device__ __forceinline__ void refine_load(uint64_t r0, uint32_t n, const R *__restrict__ rec1, R (&rec)[PT]) {
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (uint32_t it = 0; it < PT / 2; ++it) {
            const uint32_t j = 2 * (it * blockDim.x + threadIdx.x);
            if (j + 1 < n) {
                const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(rec1 + r0 + j);
                rec[2 * it] = v.x;
                rec[2 * it + 1] = v.y;
            } else {
                rec[2 * it] = j < n ? rec1[r0 + j] : R{};
                rec[2 * it + 1] = R{};
            }
        }
    } else {
#pragma unroll
        for (uint32_t it = 0; it < PT; ++it) {
            const uint32_t j = it * blockDim.x + threadIdx.x;
            rec[it] = j < n ? rec1[r0 + j] : R{};
        }
    }
}

// Whether slot it of a thread's records holds one (matches refine_load).
template <typename R>
__device__ __forceinline__ bool refine_has(uint32_t n, uint32_t it) {
    if constexpr (sizeof(R) == 8)
        return 2 * ((it / 2) * blockDim.x + threadIdx.x) + (it & 1) < n;
    else
        return it * blockDim.x + threadIdx.x < n;
}

// Pass 2, per chunk of tiles of one level-1 bucket's records: count (or,
// with SCATTER, place) each record by its segment inside the bucket.  The
// next tile's records (in this chunk or the next one) are loaded while this
// tile is written.  Counting, a chunk's histogram accumulates in LDS over its
// tiles; scattering, s_gbase[j] holds where the chunk's run of segment j
// continues, as in pass 1 (staged: whole lines only; big: tiles of 16384
// records).
template <bool SCATTER, uint32_t RW, uint32_t SHAPE = kShapeTile>
__global__ __launch_bounds__(scatter_block(SHAPE, false, RW)) void k_refine(const BinTotals *__restrict__ tot,
                                                     const RefChunk *__restrict__ chunk2,
                                                     const uint64_t *__restrict__ rec1w,
                                                     uint32_t *__restrict__ hist2,
                                                     const uint64_t *__restrict__ scan2,
                                                     uint64_t *__restrict__ rec2w, uint32_t fan_max) {
    using R = typename RecOf<RW>::T;
    using Sh = ScatterShape<SHAPE, RW, false>;
    constexpr bool STAGED = SHAPE == kShapeStaged;
    constexpr bool CHILD = RW == 1 && SHAPE == kShapeTile;  // segments kept in s_child
    constexpr uint32_t PT = Sh::per, TILE = Sh::tile, RB = Sh::rb;
    static_assert(PT * Sh::block == TILE && PT % 2 == 0, "tile shape");
    static_assert(SHAPE == kShapeTile || SCATTER, "counting uses plain tiles");
    __shared__ uint32_t s_nlines;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    const StageLayout lay = stage_layout<R>(fan_max, kRefTile);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(s_dyn);
    uint64_t *s_gbase = reinterpret_cast<uint64_t *>(s_dyn + align16(4 * (fan_max + 1)));
    R *s_rec = reinterpret_cast<R *>(s_dyn + align16(4 * (fan_max + 1)) + align16(8 * fan_max));  // 16-byte aligned
    uint16_t *s_child = reinterpret_cast<uint16_t *>(s_rec + kRefTile);  // CHILD only
    R *s_stg = reinterpret_cast<R *>(s_dyn + lay.stg);  // STAGED only, from here on
    uint32_t *s_pack = reinterpret_cast<uint32_t *>(s_dyn + lay.pack);
    uint8_t *s_cc = reinterpret_cast<uint8_t *>(s_dyn + lay.cc);
    uint16_t *s_lrun = reinterpret_cast<uint16_t *>(s_dyn + lay.lrun);
    const R *rec1 = reinterpret_cast<const R *>(rec1w);
    R *rec2 = reinterpret_cast<R *>(rec2w);
    const uint32_t tid = threadIdx.x;
    XcdTiles xt(tot->chunks2);
    if (!xt.valid()) return;
    RefChunk C = chunk2[xt.next];
    R rec[PT];
    refine_load(C.r0, (uint32_t)min<uint64_t>(C.n, TILE), rec1, rec);
    for (;;) {
        xt.advance();
        const bool more = xt.valid();
        RefChunk N{};
        if (more) N = chunk2[xt.next];
        const uint32_t fan = C.fan, d1 = C.d1;
        if (!SCATTER) {
            for (uint32_t j = tid; j < fan; j += blockDim.x) s_cnt[j] = 0u;
        } else {
            for (uint32_t j = tid; j < fan; j += blockDim.x) {
                s_gbase[j] = scan2[C.hcol + (uint64_t)j * C.stride];
                if (STAGED) s_cc[j] = 0;
            }
        }
        for (uint64_t t0 = 0; t0 < C.n; t0 += TILE) {
            const uint32_t n = (uint32_t)min<uint64_t>(TILE, C.n - t0);
            // the tile after this one: in this chunk, else the next chunk's first
            const bool next_here = t0 + TILE < C.n;
            const uint64_t nr0 = next_here ? C.r0 + t0 + TILE : N.r0;
            const uint32_t nn = next_here ? (uint32_t)min<uint64_t>(TILE, C.n - t0 - TILE)
                                          : (more ? (uint32_t)min<uint64_t>(TILE, N.n) : 0u);
            if (SCATTER)
                for (uint32_t j = tid; j <= fan; j += blockDim.x) s_cnt[j] = j << RB;
            __syncthreads();
            uint32_t tag[PT];  // scatter: segment << RB | rank (segment fan: past the end)
#pragma unroll
            for (uint32_t it = 0; it < PT; ++it) {
                const uint32_t c =
                    refine_has<R>(n, it) ? child_of(image_top(RecOf<RW>::head(rec[it]) >> 3), d1, fan) : fan;
                if (SCATTER)
                    tag[it] = lds_add32(&s_cnt[c], 1u);
                else
                    __hip_atomic_fetch_add(&s_cnt[c], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (!SCATTER) {
                if (nn) refine_load(nr0, nn, rec1, rec);
                continue;  // the next tile's adds go to the same counters
            }
            __syncthreads();
            if (STAGED) {
                stage_starts<R>(s_cnt, s_gbase, s_cc, s_pack, s_lrun, &s_nlines, fan);
                __syncthreads();
#pragma unroll
                for (uint32_t it = 0; it < PT; ++it) {
                    const uint32_t c = tag[it] >> RB;
                    if (c == fan) continue;  // past the tile's end
                    s_rec[s_cnt[c] + (tag[it] & ((1u << RB) - 1))] = rec[it];
                }
                if (nn) refine_load(nr0, nn, rec1, rec);
                __syncthreads();
                stage_write<R>(s_lrun, s_pack, s_gbase, s_stg, s_rec, s_nlines, rec2);
                __syncthreads();
                stage_tail<R>(s_cnt, s_gbase, s_cc, s_stg, s_rec, fan, n);
                __syncthreads();  // before the next tile resets the counters
                continue;
            }
            bucket_starts(s_cnt, s_gbase, fan, RB, [&](uint32_t j) { return s_gbase[j]; });
            __syncthreads();
#pragma unroll
            for (uint32_t it = 0; it < PT; ++it) {
                const uint32_t c = tag[it] >> RB;
                if (c == fan) continue;  // past the tile's end
                const uint32_t pos = s_cnt[c] + (tag[it] & ((1u << RB) - 1));
                s_rec[pos] = rec[it];
                if (CHILD) s_child[pos] = (uint16_t)c;
            }
            if (nn) refine_load(nr0, nn, rec1, rec);
            __syncthreads();
            for (uint32_t j = tid; j < n; j += blockDim.x) {
                const R r = s_rec[j];
                const uint32_t c = CHILD ? s_child[j] : child_of(image_top(RecOf<RW>::head(r) >> 3), d1, fan);
                rec2[s_gbase[c] + j] = r;
            }
            __syncthreads();
            for (uint32_t j = tid; j < fan; j += blockDim.x) s_gbase[j] += j + 1 < fan ? s_cnt[j + 1] : n;
            __syncthreads();  // before the next tile resets the counters
        }
        __syncthreads();
        if (!SCATTER) {
            for (uint32_t j = tid; j < fan; j += blockDim.x) hist2[C.hcol + (uint64_t)j * C.stride] = s_cnt[j];
            __syncthreads();
        } else if (STAGED) {
            stage_flush<R>(s_gbase, s_cc, s_stg, fan, rec2);
            __syncthreads();
        }
        if (!more) break;
        C = N;
    }
}

// Descriptor of every pass-2 chunk: a block per level-1 bucket, a thread per chunk.
__global__ void k_chunk_descs(const Instance *__restrict__ inst, const Bucket *__restrict__ buckets,
                              const BinTotals *__restrict__ tot, RefChunk *__restrict__ chunk2,
                              uint64_t chunks_cap) {
    const uint64_t G = tot->buckets;
    const uint64_t span = tot->chunk2 * (uint64_t)kRefTile;  // records per chunk
    for (uint64_t g = blockIdx.x; g < G; g += gridDim.x) {
        const Bucket B = buckets[g];
        const uint32_t d1 = inst[B.inst].d1;
        for (uint64_t c = threadIdx.x; c < B.chunks && B.chunk_base + c < chunks_cap; c += blockDim.x) {
            RefChunk C;
            C.r0 = B.start + c * span;
            C.n = min<uint64_t>(span, B.size - c * span);
            C.hcol = B.hist_base + c;
            C.stride = B.chunks;
            C.fan = B.fan;
            C.d1 = d1;
            chunk2[B.chunk_base + c] = C;
        }
    }
}

// First record of every segment (and the total after the last).
__global__ void k_part_starts(const PassArgs *__restrict__ args, const Instance *__restrict__ inst,
                              const BinPlan *__restrict__ plan, const Bucket *__restrict__ buckets,
                              const uint64_t *__restrict__ scan2, const BinTotals *__restrict__ tot,
                              uint64_t *__restrict__ pstart) {
    const uint32_t m = args->m;
    const uint64_t parts_total = args->parts_total;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t gp = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gp < parts_total; gp += stride) {
        const uint32_t i = (uint32_t)last_le(m, gp, [&](uint64_t j) { return inst[j].part_base; });
        const Instance &in = inst[i];
        const uint32_t p = (uint32_t)(gp - in.part_base);
        const uint32_t b = p / in.fan, c = p - b * in.fan;
        const Bucket &B = buckets[plan[i].bucket_base + b];
        pstart[gp] = scan2[B.hist_base + (uint64_t)c * B.chunks];
        if (gp + 1 == parts_total) pstart[parts_total] = scan2[tot->hist2_len];
    }
}

// ---------------------------------------------------------------- reduce

// Sum of v over the block; thread 0 adds it to *dst.  Whole block.
__device__ void flush_block_sum(uint64_t v, uint64_t *dst, uint64_t *s_sum) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (threadIdx.x == 0) *s_sum = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && v)
        __hip_atomic_fetch_add(s_sum, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (threadIdx.x == 0 && *s_sum) atomic_add_u64(dst, *s_sum);
    __syncthreads();
}

constexpr uint32_t kReducePrefetch = 8;  // records a thread loads before using them
constexpr uint64_t kNoRecord = ~0ull;     // no record: a record's first word stays below 2^63

// Find-or-claim one record's vertex in the LDS segment and count its letter.
// Returns false when the segment has no free slot for it.
// home_mask: kSegSlots - 1, or 7 with the test hash (every key of a segment
// then starts at one of its first eight slots).
template <bool STATS>
__device__ __forceinline__ bool reduce_record(uint64_t rec, uint64_t *s_key, uint32_t *s_cnt,
                                              uint64_t &claims, uint32_t home_mask, ProbeStats &ps) {
    const uint64_t img = rec >> 3;
    const uint64_t tagv = img | kOccupied;
    uint32_t s = seg_home(img) & home_mask;
    uint32_t q = 0;
    if constexpr (!STATS) {
        // Each probe is one compare-and-swap of an empty slot to this key: it
        // claims the slot if empty and otherwise returns the key it holds, so
        // the loop has one exit test and no nested branch (10 % less reduce
        // time than a load followed by a CAS on empty slots).  The statistics
        // build below keeps the load, so that a CAS it issues is one that
        // expected an empty slot and a failed one is a lost race.
        uint64_t old;
        for (;;) {
            old = 0;
            __hip_atomic_compare_exchange_strong(&s_key[s], &old, tagv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0 || old == tagv) break;
            if (++q == kSegSlots) return false;
            s = (s + 1) & (kSegSlots - 1);
        }
        claims += old == 0 ? 1u : 0u;
        if (!(rec & 4)) lds_add32(&s_cnt[4 * s + (uint32_t)(rec & 3)], 1u);
        return true;
    }
    uint64_t cur = lds_load64(&s_key[s]);
    // probe until the slot holds this key (found, or claimed here); the count
    // is added once, after the loop
    for (;;) {
        if (cur == 0) {
            uint64_t expected = 0;
            __hip_atomic_compare_exchange_strong(&s_key[s], &expected, tagv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            if (STATS) {
                ++ps.cas;
                ps.lost += expected != 0 ? 1u : 0u;
            }
            if (expected == 0) {
                ++claims;
                break;
            }
            cur = expected;
        }
        if (cur == tagv) break;
        if (++q == kSegSlots) return false;
        s = (s + 1) & (kSegSlots - 1);
        cur = lds_load64(&s_key[s]);
    }
    if (STATS) ps.lookup(q + 1);
    if (!(rec & 4)) lds_add32(&s_cnt[4 * s + (uint32_t)(rec & 3)], 1u);
    return true;
}

// Long keys: a slot's key is two LDS words, hi (ih | kOccupied) and lo (il).
// A slot is claimed by the CAS of hi; the claimer then stores lo and sets
// kReady in hi.  A lane that finds its own hi without kReady has met a claim
// in flight and reads the slot again (the claimer waits on nothing between
// its CAS and those stores); with kReady set, lo decides whether the slot
// is this key's.  Returns the slot, or kSegSlots when none is found.
constexpr uint64_t kReady = 1ull << 62;
constexpr uint32_t kMaxInFlightReads = 1u << 20;

template <bool STATS>
__device__ __forceinline__ uint32_t wide_slot(uint64_t tag, uint64_t lo, uint64_t *s_hi, uint64_t *s_lo,
                                              bool &claimed, uint32_t home_mask, ProbeStats &ps) {
    uint32_t s = seg_home(lo) & home_mask, waits = 0;
    for (uint32_t q = 0;;) {
        uint64_t cur = __hip_atomic_load(&s_hi[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == 0) {
            uint64_t expected = 0;
            __hip_atomic_compare_exchange_strong(&s_hi[s], &expected, tag, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            if (STATS) {
                ++ps.cas;
                ps.lost += expected != 0 ? 1u : 0u;
            }
            if (expected == 0) {
                __hip_atomic_store(&s_lo[s], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_store(&s_hi[s], tag | kReady, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                claimed = true;
                if (STATS) ps.lookup(q + 1);
                return s;
            }
            cur = expected;
        }
        if ((cur & ~kReady) == tag) {
            if (!(cur & kReady)) {  // claim in flight: read the slot again
                if (++waits > kMaxInFlightReads) return kSegSlots;
                continue;
            }
            if (lds_load64(&s_lo[s]) == lo) {
                if (STATS) ps.lookup(q + 1);
                return s;
            }
        }
        if (++q == kSegSlots) return kSegSlots;
        s = (s + 1) & (kSegSlots - 1);
    }
}

template <bool STATS>
__device__ __forceinline__ bool reduce_record(ulonglong2 rec, uint64_t *s_key, uint32_t *s_cnt, uint64_t &claims,
                                              uint32_t home_mask, ProbeStats &ps) {
    bool claimed = false;
    const uint32_t s =
        wide_slot<STATS>((rec.x >> 3) | kOccupied, rec.y, s_key, s_key + kSegSlots, claimed, home_mask, ps);
    if (s == kSegSlots) return false;
    claims += claimed ? 1u : 0u;
    if (!(rec.x & 4)) lds_add32(&s_cnt[4 * s + (uint32_t)(rec.x & 3)], 1u);
    return true;
}

// One workgroup per segment.  The segment's hash slots live in LDS only: the
// vertices the table already holds (packed at entries [0, seg_count)) are
// re-inserted, every record of the segment is found-or-claimed and counted
// with LDS atomics, and the occupied slots are written back packed, with the
// new seg_count.  With a fused extraction (PassArgs.xkeys) they are also
// written, as keys and counters, to the caller's output arrays.  Each
// workgroup takes a contiguous run of segments, so it meets few instances
// and flushes its claim count once per instance.
//
// Nothing global sits on the path from one segment to the next: segment
// starts are read 256 at a time into LDS, the instance (and whether it is
// skipped) is kept until the run crosses an instance boundary, and the next
// segment's first records are loaded while this one is written back.
constexpr uint32_t kStartsChunk = 256;  // segment starts staged per LDS refill

template <uint32_t EW, uint32_t RW, bool STATS>
__global__ __launch_bounds__(kReduceBlock) void k_reduce(const PassArgs *__restrict__ args,
                                                        const Instance *__restrict__ inst,
                                                        const uint64_t *__restrict__ pstart,
                                                        const uint64_t *__restrict__ rec2w,
                                                        InstStatus *st) {
    using R = typename RecOf<RW>::T;
    const R *rec2 = reinterpret_cast<const R *>(rec2w);
    static_assert(RW == 1 || EW == 4, "long keys take 32-byte entries");
    const uint32_t m = args->m;
    const uint64_t parts_total = args->parts_total;
    // fused extraction (one instance): see the write-back
    uint64_t *__restrict__ xkeys = args->xkeys;
    uint4 *__restrict__ xcounts = reinterpret_cast<uint4 *>(args->xcounts);
    const uint64_t xcap = args->xcap;
    static_assert(kSegSlots % kReduceBlock == 0 && kReduceBlock % 64 == 0, "slot ranges per wavefront");
    constexpr uint32_t kWaves = kReduceBlock / 64;
    constexpr uint32_t kWaveSlots = kSegSlots / kWaves;  // slots compacted by one wavefront
    __shared__ uint64_t s_key[kSegSlots * RW];  // RW = 2: hi words, then lo words
    __shared__ __align__(16) uint32_t s_cnt[kSegSlots * 4];
    __shared__ uint64_t s_start[kStartsChunk + 2];
    __shared__ uint32_t s_wave_n[kWaves];
    __shared__ uint64_t s_sum, s_xbase;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t home_mask = args->test_hash ? 7u : kSegSlots - 1;
    ProbeStats ps, ps_old;  // ps_old: re-inserted vertices of earlier builds, not counted
    const uint64_t per_block = (parts_total + gridDim.x - 1) / gridDim.x;
    const uint64_t gp0 = min((uint64_t)blockIdx.x * per_block, parts_total);
    const uint64_t gp1 = min(gp0 + per_block, parts_total);
    if (gp0 >= gp1) return;
    // LDS starts zeroed and every write-back leaves it zeroed again
    for (uint32_t s = tid; s < kSegSlots; s += blockDim.x) {
        s_key[s] = 0;
        reinterpret_cast<uint4 *>(s_cnt)[s] = make_uint4(0, 0, 0, 0);
    }
    const R kNone = RecOf<RW>::none();
    // s_start[j] = pstart[c0 + j] for j <= kStartsChunk + 1 (within range)
    uint64_t c0 = gp0;
    auto stage_starts = [&]() {
        for (uint32_t j = tid; j < kStartsChunk + 2; j += blockDim.x)
            s_start[j] = c0 + j <= parts_total ? pstart[c0 + j] : 0;
        __syncthreads();
    };
    stage_starts();
    uint32_t cur_inst = (uint32_t)last_le(m, gp0, [&](uint64_t j) { return inst[j].part_base; });
    uint64_t next_base = cur_inst + 1 < m ? inst[cur_inst + 1].part_base : ~0ull;
    bool skip = __hip_atomic_load(&st[cur_inst].err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kSkipMask;
    uint64_t my_claims = 0;  // claims of cur_inst by this thread, not yet flushed

    R rv[kReducePrefetch];  // first records of the current segment
    {
        const uint64_t a = s_start[0], z = s_start[1];
#pragma unroll
        for (uint32_t c = 0; c < kReducePrefetch; ++c) {
            const uint64_t r = a + (uint64_t)c * blockDim.x + tid;
            rv[c] = r < z ? rec2[r] : kNone;
        }
    }
    for (uint64_t gp = gp0; gp < gp1; ++gp) {
        if (gp >= next_base) {  // uniform: the run enters the next instance
            flush_block_sum(my_claims, &st[cur_inst].claimed, &s_sum);
            my_claims = 0;
            while (gp >= next_base) {
                ++cur_inst;
                next_base = cur_inst + 1 < m ? inst[cur_inst + 1].part_base : ~0ull;
            }
            skip = __hip_atomic_load(&st[cur_inst].err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kSkipMask;
        }
        if (gp - c0 == kStartsChunk) {
            __syncthreads();  // every thread is done with the old starts
            c0 = gp;
            stage_starts();
        }
        const uint64_t a = s_start[gp - c0], z = s_start[gp - c0 + 1];
        const Instance &in = inst[cur_inst];
        const uint64_t seg_idx = gp - in.part_base;
        uint64_t *seg = in.table + seg_idx * (uint64_t)kSegSlots * EW;
        // a skipped (rejected) instance has no records and its table is left untouched
        const uint32_t n_old = (skip || in.fresh) ? 0u : min(in.seg_count[seg_idx], kSegSlots);
        for (uint32_t e = tid; e < n_old; e += blockDim.x) {
            // distinct keys: each claims its own slot, and nobody else touches
            // that slot's counters before the next barrier
            const uint64_t tagv = seg[e];
            const uint4 cv = seg_counts<RW>(seg)[e];
            if constexpr (RW == 2) {
                bool claimed = false;
                const uint32_t s =
                    wide_slot<false>(tagv, seg[kSegSlots + e], s_key, s_key + kSegSlots, claimed, home_mask, ps_old);
                if (s < kSegSlots) reinterpret_cast<uint4 *>(s_cnt)[s] = cv;
                continue;
            }
            uint32_t s = seg_home(tagv) & home_mask;
            for (uint32_t q = 0; q < kSegSlots; ++q) {
                uint64_t expected = 0;
                if (__hip_atomic_compare_exchange_strong(&s_key[s], &expected, tagv, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    reinterpret_cast<uint4 *>(s_cnt)[s] = cv;
                    break;
                }
                s = (s + 1) & (kSegSlots - 1);
            }
        }
        __syncthreads();
        bool full = false;
        for (uint64_t base = a;;) {
#pragma unroll
            for (uint32_t c = 0; c < kReducePrefetch; ++c)
                if (RecOf<RW>::head(rv[c]) != kNoRecord &&
                    !reduce_record<STATS>(rv[c], s_key, s_cnt, my_claims, home_mask, ps))
                    full = true;
            base += (uint64_t)blockDim.x * kReducePrefetch;
            if (base >= z) break;
#pragma unroll
            for (uint32_t c = 0; c < kReducePrefetch; ++c) {
                const uint64_t r = base + (uint64_t)c * blockDim.x + tid;
                rv[c] = r < z ? rec2[r] : kNone;
            }
        }
        // the next segment's first records load while this one is written back
        {
            const uint64_t na = z, nz = gp + 1 < gp1 ? s_start[gp - c0 + 2] : z;
#pragma unroll
            for (uint32_t c = 0; c < kReducePrefetch; ++c) {
                const uint64_t r = na + (uint64_t)c * blockDim.x + tid;
                rv[c] = r < nz ? rec2[r] : kNone;
            }
        }
        if (full) atomic_or_u32(&st[cur_inst].err, kErrFull);
        __syncthreads();
        if (skip) continue;  // uniform; LDS is still all zero
        // write the occupied slots back packed: each wavefront compacts its
        // own slot range with ballots, after one exchange of range totals
        const uint32_t s0 = wave * kWaveSlots;
        uint32_t mine = 0;
        for (uint32_t c0w = 0; c0w < kWaveSlots; c0w += 64)
            mine += (uint32_t)__popcll(__ballot(s_key[s0 + c0w + lane] != 0));
        if (lane == 0) s_wave_n[wave] = mine;
        __syncthreads();
        uint32_t out = 0, total = 0;
        for (uint32_t w2 = 0; w2 < kWaves; ++w2) {
            const uint32_t nw = s_wave_n[w2];
            out += w2 < wave ? nw : 0u;
            total += nw;
        }
        // Fused extraction: the segment's vertices also go to the caller's
        // arrays at [xbase, xbase + total), reserved with one device atomic
        // whose latency the table write-back below hides.  The order of
        // segments in the output is whatever order the reservations land in.
        uint64_t xbase = 0;
        if (xkeys && tid == 0)
            xbase = __hip_atomic_fetch_add(&st[cur_inst].emitted, (uint64_t)total, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t out0 = out;
        for (uint32_t c0w = 0; c0w < kWaveSlots; c0w += 64) {
            const uint32_t s = s0 + c0w + lane;
            const uint64_t tagv = s_key[s];
            const uint64_t mask = __ballot(tagv != 0);
            if (tagv) {
                const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1));
                seg[out + rank] = tagv & ~kReady;
                if (RW == 2) seg[kSegSlots + out + rank] = s_key[kSegSlots + s];
                seg_counts<RW>(seg)[out + rank] = reinterpret_cast<const uint4 *>(s_cnt)[s];
                if (!xkeys) {
                    s_key[s] = 0;
                    reinterpret_cast<uint4 *>(s_cnt)[s] = make_uint4(0, 0, 0, 0);
                }
            }
            out += (uint32_t)__popcll(mask);
        }
        if (xkeys) {  // uniform
            if (tid == 0) s_xbase = xbase;
            __syncthreads();
            const uint64_t xb = s_xbase;
            out = out0;
            for (uint32_t c0w = 0; c0w < kWaveSlots; c0w += 64) {
                const uint32_t s = s0 + c0w + lane;
                const uint64_t tagv = s_key[s];
                const uint64_t mask = __ballot(tagv != 0);
                if (tagv) {
                    const uint64_t o = xb + out + (uint32_t)__popcll(mask & ((1ull << lane) - 1));
                    if (o < xcap) {
                        if constexpr (RW == 1) {
                            xkeys[o] = key_of_image(tagv & ~kOccupied);
                        } else {  // two key words per record: K >> 64, K mod 2^64
                            uint64_t kh, kl;
                            wide_key(tagv & ~(kOccupied | kReady), s_key[kSegSlots + s], kh, kl);
                            xkeys[2 * o] = kh;
                            xkeys[2 * o + 1] = kl;
                        }
                        xcounts[o] = reinterpret_cast<const uint4 *>(s_cnt)[s];
                    }
                    s_key[s] = 0;
                    reinterpret_cast<uint4 *>(s_cnt)[s] = make_uint4(0, 0, 0, 0);
                }
                out += (uint32_t)__popcll(mask);
            }
        }
        if (tid == 0) in.seg_count[seg_idx] = total;
        __syncthreads();
    }
    flush_block_sum(my_claims, &st[cur_inst].claimed, &s_sum);
    if (STATS) ps.flush(args->stats);
}

// ---------------------------------------------------------------- extract

constexpr uint32_t kExtractSegBlock = 256;

// The vertices of segment gp (packed at its first entries) go to
// [seg_off[gp], seg_off[gp + 1]).
template <uint32_t EW, uint32_t RW>
__global__ __launch_bounds__(kExtractSegBlock) void k_extract_seg(const uint64_t *__restrict__ table,
                                                                 uint32_t parts,
                                                                 const uint64_t *__restrict__ seg_off,
                                                                 uint64_t *__restrict__ okeys,
                                                                 uint32_t *__restrict__ ocnt,
                                                                 uint64_t ocap, uint64_t *out_n) {
    for (uint32_t gp = blockIdx.x; gp < parts; gp += gridDim.x) {
        const uint64_t *seg = table + (uint64_t)gp * kSegSlots * EW;
        const uint64_t base = seg_off[gp];
        const uint32_t n = (uint32_t)min<uint64_t>(seg_off[gp + 1] - base, kSegSlots);
        for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) {
            const uint64_t idx = base + e;
            if (idx >= ocap) break;
            if constexpr (RW == 1) {
                okeys[idx] = key_of_image(seg[e] & ~kOccupied);
            } else {  // two key words per record: K >> 64, K mod 2^64
                uint64_t kh, kl;
                wide_key(seg[e] & ~kOccupied, seg[kSegSlots + e], kh, kl);
                okeys[2 * idx] = kh;
                okeys[2 * idx + 1] = kl;
            }
            *reinterpret_cast<uint4 *>(ocnt + 4 * idx) = seg_counts<RW>(seg)[e];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *out_n = seg_off[parts];
}

__global__ void k_set_len(uint64_t *len, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *len = v;
}

template <typename K>
uint32_t occupancy_grid(K kernel, int device, uint32_t block, uint64_t cap, uint32_t dyn_lds) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)block, dyn_lds) != hipSuccess ||
        per <= 0)
        per = 1;
    uint64_t g = std::min<uint64_t>((uint64_t)cus * per, cap);
    if (g >= 8) g &= ~7ull;  // whole rounds over the 8 XCDs
    return (uint32_t)std::max<uint64_t>(1, g);
}

// Dynamic LDS of a scatter of `shape` over n runs (pass 1: first, else pass 2).
template <typename R>
uint32_t scatter_lds_bytes(uint32_t shape, bool first, uint32_t n) {
    constexpr uint32_t rw = sizeof(R) / 8;
    if (shape == kShapeStaged) return stage_layout<R>(n, first ? kBinTile : kRefTile).bytes;
    return first ? bin_lds_bytes(n, true, rw, shape) : ref_lds_bytes(n, true, rw, shape);
}

// The binned pass for records of RW words (enqueue only).
template <uint32_t RW>
hipError_t launch_passes(const PassArgs *args, const Instance *inst, const uint64_t *packed, const uint64_t *ws,
                         InstStatus *st, const BinBuffers &bb, bool stats, hipStream_t s, hipEvent_t *marks) {
    hipError_t e;
    // pass 1
    using R = typename RecOf<RW>::T;
    const uint32_t lb0 = bin_lds_bytes(bb.d1_max, false, RW);
    const uint32_t lb1 = scatter_lds_bytes<R>(bb.shape1, true, bb.d1_max);
    const uint32_t g1c = bb.grid_bin_count, g1s = bb.grid_bin_scatter;
    constexpr uint32_t CWL = RW == 1 ? kCountWindowsLong : kCountWindows;  // long counts: one-word keys
    if (is_big(bb.shape1))
        hipLaunchKernelGGL((k_bin<false, RW, kShapeTile, CWL>), dim3(g1c), dim3(kBinBlock), lb0, s, args, inst, packed,
                           ws, bb.plan, bb.totals, bb.hist1, bb.scan1, bb.rec1, bb.tile_read1, bb.d1_max);
    else
        hipLaunchKernelGGL((k_bin<false, RW>), dim3(g1c), dim3(kBinBlock), lb0, s, args, inst, packed, ws, bb.plan,
                           bb.totals, bb.hist1, bb.scan1, bb.rec1, bb.tile_read1, bb.d1_max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (marks) (void)hipEventRecord(marks[1], s);
    const uint64_t nb1 = std::max<uint64_t>((bb.hist1_cap + kFlatChunk - 1) / kFlatChunk, 1);
    const uint64_t *len1 = &bb.totals->hist1_len;
    hipLaunchKernelGGL(k_flat_local, dim3((uint32_t)nb1), dim3(kFlatBlock), 0, s, bb.hist1, len1, bb.scan1,
                       bb.partials);
    hipLaunchKernelGGL(k_flat_partials, dim3(1), dim3(1024), 0, s, bb.partials, nb1, len1, bb.scan1);
    hipLaunchKernelGGL(k_flat_add, dim3((uint32_t)nb1), dim3(kFlatBlock), 0, s, len1, bb.scan1, bb.partials);
    if (marks) (void)hipEventRecord(marks[2], s);
#define DBG_LAUNCH_BIN(SH)                                                                                      \
    hipLaunchKernelGGL((k_bin<true, RW, SH>), dim3(g1s), dim3(scatter_block(SH, true, RW)), lb1, s, args, inst, packed, \
                       ws, bb.plan, bb.totals, bb.hist1, bb.scan1, bb.rec1, bb.tile_read1, bb.d1_max)
    bool launched = false;
    if (bb.shape1 == kShapeStaged) {
        DBG_LAUNCH_BIN(kShapeStaged);
        launched = true;
    }
    if (bb.shape1 == kShapeBig) {
        DBG_LAUNCH_BIN(kShapeBig);
        launched = true;
    }
    if constexpr (RW == 1) {
        if (bb.shape1 == kShapeBigWide) {
            DBG_LAUNCH_BIN(kShapeBigWide);
            launched = true;
        }
    }
    if (!launched) DBG_LAUNCH_BIN(kShapeTile);
#undef DBG_LAUNCH_BIN
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (marks) (void)hipEventRecord(marks[3], s);

    // pass 2
    hipLaunchKernelGGL(k_refine_plan, dim3(1), dim3(1024), 0, s, args, inst, bb.plan, bb.scan1, bb.totals,
                       bb.buckets, bb.target2,
                       bb.shape2 == kShapeBig ? ScatterShape<kShapeBig, RW, false>::tile / kRefTile : 1u);
    {
        const uint32_t g = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(bb.buckets_cap, 4096));
        hipLaunchKernelGGL(k_chunk_descs, dim3(g), dim3(256), 0, s, inst, bb.buckets, bb.totals, bb.chunk2,
                           bb.chunks2_cap);
    }
    if (marks) (void)hipEventRecord(marks[4], s);
    const uint32_t lr0 = ref_lds_bytes(bb.fan_max, false, RW);
    const uint32_t lr1 = scatter_lds_bytes<R>(bb.shape2, false, bb.fan_max);
    const uint32_t g2c = bb.grid_ref_count, g2s = bb.grid_ref_scatter;
    hipLaunchKernelGGL((k_refine<false, RW>), dim3(g2c), dim3(kRefBlock), lr0, s, bb.totals, bb.chunk2, bb.rec1,
                       bb.hist2, bb.scan2, bb.rec2, bb.fan_max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (marks) (void)hipEventRecord(marks[5], s);
    const uint64_t nb2 = std::max<uint64_t>((bb.hist2_cap + kFlatChunk - 1) / kFlatChunk, 1);
    const uint64_t *len2 = &bb.totals->hist2_len;
    hipLaunchKernelGGL(k_flat_local, dim3((uint32_t)nb2), dim3(kFlatBlock), 0, s, bb.hist2, len2, bb.scan2,
                       bb.partials);
    hipLaunchKernelGGL(k_flat_partials, dim3(1), dim3(1024), 0, s, bb.partials, nb2, len2, bb.scan2);
    hipLaunchKernelGGL(k_flat_add, dim3((uint32_t)nb2), dim3(kFlatBlock), 0, s, len2, bb.scan2, bb.partials);
    if (marks) (void)hipEventRecord(marks[6], s);
#define DBG_LAUNCH_REF(SH)                                                                                   \
    hipLaunchKernelGGL((k_refine<true, RW, SH>), dim3(g2s), dim3(scatter_block(SH, false, RW)), lr1, s, bb.totals, \
                       bb.chunk2, bb.rec1, bb.hist2, bb.scan2, bb.rec2, bb.fan_max)
    launched = false;
    if (bb.shape2 == kShapeStaged) {
        DBG_LAUNCH_REF(kShapeStaged);
        launched = true;
    }
    if (bb.shape2 == kShapeBig) {
        DBG_LAUNCH_REF(kShapeBig);
        launched = true;
    }
    if (!launched) DBG_LAUNCH_REF(kShapeTile);
#undef DBG_LAUNCH_REF
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (marks) (void)hipEventRecord(marks[7], s);

    // segment starts and the reduction
    const uint64_t P = bb.parts_cap;
    const uint32_t gs = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((P + 255) / 256, 4096));
    hipLaunchKernelGGL(k_part_starts, dim3(gs), dim3(256), 0, s, args, inst, bb.plan, bb.buckets, bb.scan2,
                       bb.totals, bb.pstart);
    if (marks) (void)hipEventRecord(marks[8], s);
    // every instance of a binned launch has the same entry width
    const uint32_t gr = bb.grid_reduce;
#define DBG_LAUNCH_REDUCE(EW, R2, STATS) \
    hipLaunchKernelGGL((k_reduce<EW, R2, STATS>), dim3(gr), dim3(kReduceBlock), 0, s, args, inst, bb.pstart, bb.rec2, st)
    if (RW == 2) {
        if (stats) DBG_LAUNCH_REDUCE(4, 2, true); else DBG_LAUNCH_REDUCE(4, 2, false);
    } else if (bb.entry_words == 4) {
        if (stats) DBG_LAUNCH_REDUCE(4, 1, true); else DBG_LAUNCH_REDUCE(4, 1, false);
    } else {
        if (stats) DBG_LAUNCH_REDUCE(3, 1, true); else DBG_LAUNCH_REDUCE(3, 1, false);
    }
#undef DBG_LAUNCH_REDUCE
    return hipGetLastError();
}


}  // namespace

hipError_t launch_binned(const PassArgs *args, const Instance *inst, const uint64_t *packed,
                         const uint64_t *ws, InstStatus *st, const BinBuffers &bb, uint64_t n_cap,
                         int device, bool stats, hipStream_t s, hipEvent_t *marks) {
    (void)device;
    hipError_t e;
    hipLaunchKernelGGL(k_bin_plan, dim3(1), dim3(64), 0, s, args, inst, ws, st, bb.plan, bb.totals, bb.target1,
                       is_big(bb.shape1) ? big_tile_bytes(bb.shape1, true, bb.rec_words) / (8u * bb.rec_words) / kBinTile
                                         : 1u);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        const uint32_t g = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n_cap + 255) / 256, 8192));
        hipLaunchKernelGGL(k_tile_reads, dim3(g), dim3(256), 0, s, args, inst, ws, bb.plan, bb.tile_read1,
                           bb.tiles1_cap);
    }
    if (marks) (void)hipEventRecord(marks[0], s);

    if (bb.rec_words == 2) return launch_passes<2>(args, inst, packed, ws, st, bb, stats, s, marks);
    return launch_passes<1>(args, inst, packed, ws, st, bb, stats, s, marks);
}

namespace {
constexpr uint32_t kScatterWide = 384;  // segments per bucket beyond which pass 2 scatters on half the grid

// Whether a staged scatter kernel with `dyn` bytes of dynamic LDS fits one
// workgroup (its static LDS included), with dynamic LDS allowed up to that.
template <typename K>
bool stage_fits(K kernel, int device, uint32_t dyn) {
    int max_lds = 0;
    hipFuncAttributes fa{};
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
        hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kernel)) != hipSuccess)
        return false;
    if ((uint64_t)dyn + fa.sharedSizeBytes > (uint64_t)max_lds) return false;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)dyn) == hipSuccess;
}

template <uint32_t RW>
void grids_for(int device, BinBuffers &bb) {
    using R = typename RecOf<RW>::T;
    // Scatter shapes (dbg_config bin_shape1/2: 0 automatic, 1 plain tiles,
    // 2 staged, 3 big tiles, 4 wide big tiles; a shape whose LDS does not
    // fit falls back to a smaller one).  Staging holds one LDS line per run, so with many runs
    // a staged scatter runs one 1024-thread workgroup per CU, and it
    // executes about twice the instructions of a plain one per record.  Big
    // tiles make a tile's runs four times longer (about 23 records at 713
    // runs), at one workgroup per CU as well.  Measured at 508 k segments
    // (713 runs a scatter): plain 11.1 and 11.9 ms, staged 15.5 and 9.1 ms,
    // big 9.5 and 8.1 ms for the first and second scatter; at 44.7 k
    // segments (212 runs) plain 0.52 and 0.61 ms, big 0.62 and 0.51 ms (the
    // first scatter also decodes windows, four planning tiles per thread
    // group at once).  With the rolling window decode and the first
    // scatter's 8192-record tiles of one-word keys, big tiles also win at
    // 35.7 k segments (189 runs): 0.43 against 0.50 ms, and the count
    // before it 0.13 against 0.17 ms.  At 713 runs the first scatter's
    // 16384-record tiles (kShapeBigWide) beat its 8192-record ones with the
    // rolling decode, 8.28 against 8.76 ms; at 189 runs they lose, 0.49
    // against 0.42 ms.  Automatic: the second scatter takes big tiles, and
    // so does the first for one-word keys (the wide form beyond kScatterWide
    // runs) or beyond kScatterWide runs.  Requested big tiles (3) take the
    // same size rule; 4 asks for the wide form (for two-word records and
    // the second scatter, plain big tiles, which are 128 KB already).  A big
    // tile needs chunks of at least as many planning tiles as it holds (the
    // plan kernels' min_chunk).  The line numbers of a staged tile must fit
    // s_pack's 11 bits.
    const auto pick = [&](uint32_t req, bool first, uint32_t n) -> uint32_t {
        uint32_t sh = req == 1 ? kShapeTile : req == 2 ? kShapeStaged : req >= 3 ? kShapeBig
                    : !first || RW == 1 || n > kScatterWide ? kShapeBig : kShapeTile;
        if (sh == kShapeBig && first && RW == 1 && (req == 4 || n > kScatterWide)) sh = kShapeBigWide;
        const uint32_t tile = first ? kBinTile : kRefTile;
        if (sh == kShapeStaged && !(tile / Lines<R>::L + n < 2048 &&
                                    (first ? stage_fits(k_bin<true, RW, kShapeStaged>, device,
                                                        scatter_lds_bytes<R>(sh, first, n))
                                           : stage_fits(k_refine<true, RW, kShapeStaged>, device,
                                                        scatter_lds_bytes<R>(sh, first, n)))))
            sh = kShapeTile;
        if constexpr (RW == 1) {
            if (sh == kShapeBigWide &&
                !stage_fits(k_bin<true, RW, kShapeBigWide>, device, scatter_lds_bytes<R>(sh, first, n)))
                sh = kShapeBig;
        }
        if (sh == kShapeBig &&
            !(first ? stage_fits(k_bin<true, RW, kShapeBig>, device, scatter_lds_bytes<R>(sh, first, n))
                    : stage_fits(k_refine<true, RW, kShapeBig>, device, scatter_lds_bytes<R>(sh, first, n))))
            sh = kShapeTile;
        return sh;
    };
    bb.shape1 = pick(bb.shape_req1, true, bb.d1_max);
    bb.shape2 = pick(bb.shape_req2, false, bb.fan_max);
    const uint32_t l1 = scatter_lds_bytes<R>(bb.shape1, true, bb.d1_max);
    const uint32_t l2 = scatter_lds_bytes<R>(bb.shape2, false, bb.fan_max);
    constexpr uint32_t CWL = RW == 1 ? kCountWindowsLong : kCountWindows;
    bb.grid_bin_count =
        is_big(bb.shape1)
            ? occupancy_grid(k_bin<false, RW, kShapeTile, CWL>, device, kBinBlock, bb.chunks1_cap,
                             bin_lds_bytes(bb.d1_max, false, RW))
            : occupancy_grid(k_bin<false, RW>, device, kBinBlock, bb.chunks1_cap, bin_lds_bytes(bb.d1_max, false, RW));
    bb.grid_bin_scatter = occupancy_grid(k_bin<true, RW>, device, kBinBlock, bb.chunks1_cap, l1);
    if (bb.shape1 == kShapeStaged)
        bb.grid_bin_scatter = occupancy_grid(k_bin<true, RW, kShapeStaged>, device, kStageBlock, bb.chunks1_cap, l1);
    if (bb.shape1 == kShapeBig)
        bb.grid_bin_scatter =
            occupancy_grid(k_bin<true, RW, kShapeBig>, device, scatter_block(kShapeBig, true, RW), bb.chunks1_cap, l1);
    if constexpr (RW == 1) {
        if (bb.shape1 == kShapeBigWide)
            bb.grid_bin_scatter = occupancy_grid(k_bin<true, RW, kShapeBigWide>, device,
                                                 scatter_block(kShapeBigWide, true, RW), bb.chunks1_cap, l1);
    }
    bb.grid_ref_count =
        occupancy_grid(k_refine<false, RW>, device, kRefBlock, bb.chunks2_cap, ref_lds_bytes(bb.fan_max, false, RW));
    // Plain tiles write one short run per segment when a bucket has many
    // segments; the partial lines of the workgroups in flight on an XCD then
    // outgrow its L2 before the next tiles complete them, and the pass-2
    // scatter writes faster on part of its resident grid.
    const uint32_t div = bb.scatter_div ? bb.scatter_div : (bb.fan_max > kScatterWide ? 2u : 1u);
    bb.grid_ref_scatter =
        std::max<uint32_t>(8, occupancy_grid(k_refine<true, RW>, device, kRefBlock, bb.chunks2_cap, l2) / div);
    if (bb.shape2 == kShapeStaged)
        bb.grid_ref_scatter = occupancy_grid(k_refine<true, RW, kShapeStaged>, device, kStageBlock, bb.chunks2_cap, l2);
    if (bb.shape2 == kShapeBig)
        bb.grid_ref_scatter =
            occupancy_grid(k_refine<true, RW, kShapeBig>, device, scatter_block(kShapeBig, false, RW), bb.chunks2_cap, l2);
    bb.grid_reduce = RW == 2 ? occupancy_grid(k_reduce<4, 2, false>, device, kReduceBlock, bb.parts_cap, 0)
                   : bb.entry_words == 4 ? occupancy_grid(k_reduce<4, 1, false>, device, kReduceBlock, bb.parts_cap, 0)
                                         : occupancy_grid(k_reduce<3, 1, false>, device, kReduceBlock, bb.parts_cap, 0);
    // about kChunksPerGroup chunks per resident scatter workgroup
    const uint32_t per = bb.chunks_per_group ? bb.chunks_per_group : kChunksPerGroup;
    bb.target1 = (uint32_t)std::min<uint64_t>(kMaxChunkTarget, (uint64_t)per * bb.grid_bin_scatter);
    bb.target2 = (uint32_t)std::min<uint64_t>(kMaxChunkTarget, (uint64_t)per * bb.grid_ref_scatter);
}
}  // namespace

void binned_grids(int device, BinBuffers &bb) {
    if (bb.rec_words == 2)
        grids_for<2>(device, bb);
    else
        grids_for<1>(device, bb);
}

hipError_t launch_extract_binned(const uint64_t *table, uint32_t entry_words, uint32_t key_words, uint32_t parts,
                                 const uint32_t *seg_count, uint64_t *seg_off, uint64_t *partials,
                                 uint64_t *len, uint64_t *out_keys, uint32_t *out_counts,
                                 uint64_t out_cap, uint64_t *out_n, int device, hipStream_t s) {
    const uint64_t nb = std::max<uint64_t>((parts + kFlatChunk - 1) / kFlatChunk, 1);
    hipLaunchKernelGGL(k_set_len, dim3(1), dim3(64), 0, s, len, (uint64_t)parts);
    hipLaunchKernelGGL(k_flat_local, dim3((uint32_t)nb), dim3(kFlatBlock), 0, s, seg_count, len, seg_off,
                       partials);
    hipLaunchKernelGGL(k_flat_partials, dim3(1), dim3(1024), 0, s, partials, nb, len, seg_off);
    hipLaunchKernelGGL(k_flat_add, dim3((uint32_t)nb), dim3(kFlatBlock), 0, s, len, seg_off, partials);
    if (key_words == 2) {
        if (entry_words != 4) return hipErrorInvalidValue;
        const uint32_t g = occupancy_grid(k_extract_seg<4, 2>, device, kExtractSegBlock, parts, 0);
        hipLaunchKernelGGL((k_extract_seg<4, 2>), dim3(g), dim3(kExtractSegBlock), 0, s, table, parts, seg_off,
                           out_keys, out_counts, out_cap, out_n);
    } else if (entry_words == 4) {
        const uint32_t g = occupancy_grid(k_extract_seg<4, 1>, device, kExtractSegBlock, parts, 0);
        hipLaunchKernelGGL((k_extract_seg<4, 1>), dim3(g), dim3(kExtractSegBlock), 0, s, table, parts, seg_off,
                           out_keys, out_counts, out_cap, out_n);
    } else {
        const uint32_t g = occupancy_grid(k_extract_seg<3, 1>, device, kExtractSegBlock, parts, 0);
        hipLaunchKernelGGL((k_extract_seg<3, 1>), dim3(g), dim3(kExtractSegBlock), 0, s, table, parts, seg_off,
                           out_keys, out_counts, out_cap, out_n);
    }
    return hipGetLastError();
}

}  // namespace dbgk
