// Internal interface between the HIP kernels and the host runtime of libdbg.
//
// One build pass over a batch of m graphs ("instances"; a plain build is the
// case m = 1) runs these kernels in stream order:
//
//   prepare    -- zero the per-call status words and the work cursor
//   pack       -- ASCII -> 2-bit letter codes, 32 bases per uint64, first
//                 base in the top bits; flags bytes outside ACGTacgt
//   scan_*     -- windows per read, exclusive prefix over reads, and the
//                 tile -> first-read map the build kernel starts from
//   build      -- persistent: workgroups pull tiles of windows from a
//                 cursor, extract each window's (k-1)-mer and next letter,
//                 optionally merge equal vertices within a wavefront, then
//                 find-or-claim the vertex slot (64-bit CAS) and raise its
//                 counter (32-bit atomic add)
//
// Table layout: an array of `cap` entries of `entry_words` uint64 words
// (3 = 24 bytes, 4 = 32 bytes).  Word 0 holds the vertex key with bit 63 set,
// the next 16 bytes four uint32 counters in letter-code order A, C, T, G.
// Long k (32 < k <= 64), direct build: 32-byte entries whose words 0 and 1
// hold the upper and lower 63 bits of the key, each with bit 63 set, and
// whose words 2-3 hold the counters (the binned build of 33 <= k <= 63 keeps
// its segments' key words and counters as arrays, as described below).
// Direct build: the entries are the open-addressing slots themselves (0 =
// empty, so a zero fill empties the table).  Binned build: the table is cut
// into segments of kSegSlots entries, and segment s holds its vertices packed
// at [0, seg_count[s]), stored as two arrays: kSegSlots key words, then
// kSegSlots groups of four counters (the hash slots live in LDS only while
// the segment is being built).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbgk {

constexpr uint64_t kOccupied = 1ull << 63;

// Status bits of one instance, reported back as DBG_E_* codes.
enum : uint32_t {
    kErrBase = 1u,   // a byte outside ACGTacgt in one of its reads
    kErrInval = 2u,  // inconsistent offsets
    kErrRange = 4u,  // cumulative k-mers would exceed 2^32 - 1
    kErrFull = 8u,   // no free slot left for some vertex
    kErrSkip = 16u,  // left out by the host (its status is decided there)
};

struct Instance {
    uint64_t *table;        // entry array of this graph
    uint64_t cap;           // slots
    uint64_t read_begin;    // first read (global index) of this instance
    uint64_t read_end;      // one past its last read
    uint64_t byte_begin;    // first byte of its reads, relative to the first read
    uint64_t byte_end;      // (both filled on the device from the offsets)
    uint64_t prior_inserts; // k-mers already counted into the table
    uint64_t part_base;     // binned: global index of its first table segment
    uint32_t *seg_count;    // binned: occupied slots per segment (written by the build)
    uint64_t reserved;
    uint32_t k;
    uint32_t entry_words;
    uint32_t skip;          // nonzero: the host left this instance out
    uint32_t parts;         // binned: table segments (cap / kSegSlots)
    uint32_t d1;            // binned: level-1 buckets
    uint32_t fan;           // binned: segments per level-1 bucket (the last may have fewer)
    uint32_t fresh;         // binned: the table is logically empty; segments are not read
    uint32_t pad;
};

// Per-call sizes and inputs, read by every kernel of a pass from device
// memory, so that one captured graph serves every call whose sizes fit the
// capacities the graph was captured for.  Stored at the start of the device
// instance buffer, followed (at kArgsBytes) by the Instance array.
struct PassArgs {
    const uint8_t *reads;   // ASCII bases; read i is reads[off[i]-off[0] .. off[i+1]-off[0])
    const uint64_t *off;    // n_reads + 1 offsets
    uint64_t n_reads;
    uint64_t reads_len;     // bytes (off[n] - off[0] when valid)
    uint64_t max_windows;   // more windows than this flags every instance invalid
    uint64_t tile_cap;      // direct build: tile map entries
    uint64_t parts_total;   // binned build: segments over all instances
    uint64_t *xkeys;        // binned build of one instance: when set, the reduce also writes
    uint32_t *xcounts;      // every vertex of the graph to these arrays (keys of one or two
    uint64_t xcap;          // words, four counters each; entries past xcap are dropped)
    uint64_t *stats;        // probe statistics of this pass (kStat* words), accumulated; null: not kept
    uint32_t m;             // instances
    uint32_t check_ends;    // require off[n] - off[0] == reads_len
    uint32_t tile;          // direct build: windows per tile
    uint32_t test_hash;     // nonzero: every key's home slot is its low 3 bits (tests only)
};
constexpr uint32_t kArgsBytes = 128;
static_assert(sizeof(PassArgs) <= kArgsBytes, "PassArgs grew");

struct InstStatus {
    uint32_t err;       // kErr* bits
    uint32_t pad;
    uint64_t claimed;   // slots claimed by this call
    uint64_t inserts;   // k-mers of this call
    uint64_t windows;   // windows of this call
    uint64_t emitted;   // vertices the reduce wrote to the PassArgs output arrays
};

// Probe statistics (kernels built with STATS): words of PassArgs::stats.
enum : uint32_t {
    kStatLookups = 0,   // vertex lookups that reached the table
    kStatProbes = 1,    // slots they examined
    kStatCas = 2,       // compare-and-swaps issued to claim a slot
    kStatCasLost = 3,   // of those, the ones another thread won first
    kStatHist = 4,      // 8 words: lookups by slots examined, 1, 2, 3-4, 5-8, 9-16, 17-32, 33-64, more
    kStatWords = 12,
};

// One thread's probe statistics, flushed once per wavefront.
struct ProbeStats {
    uint32_t lookups = 0, cas = 0, lost = 0;
    uint64_t probes = 0;
    uint32_t hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    __device__ void lookup(uint32_t n_probes) {
        ++lookups;
        probes += n_probes;
        const uint32_t bin = n_probes <= 1 ? 0u : min(7u, 32u - (uint32_t)__clz(n_probes - 1));
        ++hist[bin];
    }
    // Wavefront sums, added to stats[] by lane 0 (whole wavefront).
    __device__ void flush(uint64_t *stats) {
        uint64_t v[kStatWords] = {lookups, probes, cas, lost};
        for (int i = 0; i < 8; ++i) v[kStatHist + i] = hist[i];
        for (int i = 0; i < (int)kStatWords; ++i) {
            for (int d = 32; d >= 1; d >>= 1) v[i] += __shfl_xor(v[i], d, 64);
            if ((threadIdx.x & 63) == 0 && v[i])
                __hip_atomic_fetch_add(stats + i, v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
};

struct CallState {
    uint64_t cursor;    // next tile for the persistent build
    uint64_t windows;   // total windows over all instances
};

// Geometry of the build launch.
struct BuildShape {
    uint32_t block;     // threads per workgroup (multiple of 64, <= 1024)
    uint32_t wpt;       // windows per thread per tile
    uint32_t grid;      // persistent workgroups
    uint32_t merge;     // wavefront merge of equal vertices
};

// Binned build: the table of an instance is cut into segments of kSegSlots
// slots.  The records of all windows ((k-1)-mer << 3 | sink << 2 | letter)
// are partitioned by segment in two levels (d1 buckets, each split into at
// most `fan` segments), and one workgroup then owns each segment: it stages
// the segment in LDS, claims and counts there, and writes it back.
//
// Each partition pass works on chunks of consecutive tiles (a tile is what a
// workgroup sorts in LDS at once).  A chunk has one histogram, so a chunk's
// records of one bucket (or segment) form one contiguous output run that its
// workgroup extends tile after tile: runs stay long when there are many
// buckets, and the histograms stay small.  The chunk length is chosen on the
// device so that a pass has about `target` chunks.
constexpr uint32_t kSegSlots = 2048;
constexpr uint32_t kMaxD1 = 1024;     // level-1 buckets per instance, at most
constexpr uint32_t kMaxFan = 2048;    // segments per level-1 bucket, at most
constexpr uint32_t kBinBlock = 512;
constexpr uint32_t kBinPerThread = 8;
constexpr uint32_t kBinTile = kBinBlock * kBinPerThread;  // windows per pass-1 tile
constexpr uint32_t kRefBlock = 512;
constexpr uint32_t kRefPerThread = 8;
constexpr uint32_t kRefTile = kRefBlock * kRefPerThread;  // records per pass-2 tile
constexpr uint32_t kReduceBlock = 512;
constexpr uint32_t kMaxChunkTarget = 16384;  // chunks a pass aims for, at most
constexpr uint32_t kChunksPerGroup = 32;     // default target: chunks per resident workgroup

struct BinPlan {        // per instance
    uint64_t w_begin, w_end;  // its windows
    uint64_t tiles;           // pass-1 tiles
    uint64_t tile_base;       // first pass-1 tile
    uint64_t chunks;          // pass-1 chunks (of BinTotals::chunk1 tiles; the last may have fewer)
    uint64_t chunk_base;      // first pass-1 chunk
    uint64_t hist_base;       // first pass-1 histogram entry (d1 x chunks, bucket-major)
    uint64_t bucket_base;     // first level-1 bucket
};

struct Bucket {         // per level-1 bucket
    uint64_t start, size;     // record range in the level-1 output
    uint64_t chunks;          // pass-2 chunks (of BinTotals::chunk2 tiles; the last may have fewer)
    uint64_t chunk_base;      // first pass-2 chunk
    uint64_t hist_base;       // first pass-2 histogram entry (fan x chunks, segment-major)
    uint32_t inst;            // owning instance
    uint32_t b;               // bucket index within the instance
    uint32_t fan;             // segments in this bucket
    uint32_t pad;
};

struct RefChunk {       // per pass-2 chunk: everything its kernels need, in one load
    uint64_t r0;              // first record (level-1 output)
    uint64_t n;               // records
    uint64_t hcol;            // histogram entry of the bucket's first segment for this chunk
    uint64_t stride;          // histogram entries from one segment to the next (the bucket's chunks)
    uint32_t fan;             // segments in the bucket
    uint32_t d1;              // level-1 buckets of the instance (first digit's radix)
};

struct BinTotals {
    uint64_t tiles1, chunk1, chunks1, hist1_len, buckets, chunk2, chunks2, hist2_len, records;
};

struct BinBuffers {     // device scratch of one binned pass
    BinPlan *plan;            // m
    Bucket *buckets;          // sum of d1
    BinTotals *totals;
    uint32_t *hist1;          // hist1_cap
    uint64_t *scan1;          // hist1_cap + 1
    uint32_t *hist2;          // hist2_cap
    uint64_t *scan2;          // hist2_cap + 1
    uint64_t *partials;       // for the flat scans
    uint64_t *rec1, *rec2;    // records (rec_words words each), windows_cap each
    uint64_t *pstart;         // parts_total + 1
    uint64_t *tile_read1;     // first read of each pass-1 tile (tiles1_cap)
    RefChunk *chunk2;         // pass-2 chunks (chunks2_cap)
    uint64_t hist1_cap, hist2_cap, partials_cap;
    uint64_t tiles1_cap, chunks1_cap, tiles2_cap, chunks2_cap, buckets_cap, parts_cap;
    uint32_t d1_max, fan_max;  // largest d1 and fan over the launch (LDS sizing)
    uint32_t entry_words;      // of every instance in the launch
    uint32_t rec_words;        // record words: 1, or 2 for long keys (33 <= k <= 63)
    // persistent grids (binned_grids fills them; no query happens while a
    // launch is being captured)
    uint32_t grid_bin_count, grid_bin_scatter, grid_ref_count, grid_ref_scatter, grid_reduce;
    uint32_t target1, target2;  // chunks each partition pass aims for (<= kMaxChunkTarget)
    // launch shape (set before binned_grids): chunks per resident scatter
    // workgroup (0: kChunksPerGroup), the divisor of the pass-2 scatter's
    // resident grid when it stores runs as they come (0: automatic, 2 when a
    // bucket has more than 384 segments), and the requested scatter shapes
    // (dbg_config bin_shape1/2: 0 automatic, 1 plain tiles, 2 staged lines,
    // 3 big tiles, 4 big tiles of 128 KB)
    uint32_t chunks_per_group, scatter_div, shape_req1, shape_req2;
    // the scatter shapes in use (binned_grids decides: kShape* of
    // dbg_binned.hip, 0 plain tiles, 1 staged, 2 big tiles, 3 wide big tiles)
    uint32_t shape1, shape2;
};

// Fill the grid sizes of bb from occupancy and its capacities.
void binned_grids(int device, BinBuffers &bb);

constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kScanPerThread = 4;
constexpr uint32_t kScanReads = kScanBlock * kScanPerThread;  // reads per scan block
constexpr uint32_t kMapReads = 256;  // reads of one tile staged in LDS

__host__ __device__ inline uint64_t packed_words(uint64_t bytes) { return (bytes + 31) / 32 + 2; }
inline uint64_t scan_blocks(uint64_t n_reads) { return (n_reads + kScanReads - 1) / kScanReads; }
inline uint64_t max_tiles(uint64_t bytes, uint64_t tile) { return bytes / tile + 2; }

// Launchers (all stream-ordered; they only enqueue).  `args` and `inst` are
// device pointers; *_cap values are host upper bounds that size grids.
hipError_t launch_prepare(const PassArgs *args, Instance *inst, InstStatus *st, CallState *cs,
                          uint32_t m_cap, hipStream_t s);
hipError_t launch_fill_zero(uint64_t *words, uint64_t n_words, hipStream_t s);
// out[i] = src[idx[i]] for i < n (device arrays).
hipError_t launch_gather_u64(const uint64_t *src, const uint64_t *idx, uint64_t n, uint64_t *out, hipStream_t s);
hipError_t launch_pack(const PassArgs *args, uint64_t *packed, const Instance *inst, InstStatus *st,
                       uint64_t len_cap, hipStream_t s);
// tile_read may be null (no tile map).
hipError_t launch_scan(const PassArgs *args, const Instance *inst, InstStatus *st, uint64_t *ws,
                       uint64_t *partials, uint64_t *tile_read, CallState *cs, uint64_t n_cap,
                       hipStream_t s);
// stats: launch the kernels that keep probe statistics (PassArgs::stats set).
hipError_t launch_build(const PassArgs *args, const Instance *inst, const uint64_t *packed,
                        const uint64_t *ws, const uint64_t *tile_read, InstStatus *st, CallState *cs,
                        BuildShape shape, bool single, bool stats, hipStream_t s);
// Plain build for 32 < k <= 64 (one instance, direct table of 32-byte entries).
hipError_t launch_build_wide(const PassArgs *args, const Instance *inst, const uint64_t *packed,
                             const uint64_t *ws, const uint64_t *tile_read, InstStatus *st, CallState *cs,
                             BuildShape shape, bool stats, hipStream_t s);
// Records of a long-k table: two key words per record, (K >> 64, K mod 2^64).
hipError_t launch_extract_wide(const uint64_t *table, uint64_t cap, uint64_t *out_keys, uint32_t *out_counts,
                               uint64_t out_cap, uint64_t *out_n, hipStream_t s);
hipError_t launch_extract(const uint64_t *table, uint32_t entry_words, uint64_t cap,
                          uint64_t *out_keys, uint32_t *out_counts, uint64_t out_cap,
                          uint64_t *out_n, hipStream_t s);
// Normalized counters (Methods, "Normalization of graph"): counts[i] becomes
// round-half-up(counts[i] * genome / total), saturated at 2^32 - 1, in place,
// or into out8 saturated at 255 when out8 is not NULL (genome = 0: no
// division, saturation only).
hipError_t launch_normalize(uint32_t *counts, uint64_t n, uint64_t genome, uint64_t total, uint8_t *out8,
                            hipStream_t s);
hipError_t launch_count(const uint64_t *table, uint32_t entry_words, uint64_t cap,
                        uint64_t *out_n, hipStream_t s);
hipError_t launch_roofline(uint64_t *mem, uint64_t words, uint64_t n_ops, uint32_t kind,
                           uint64_t seed, uint32_t block, uint64_t *sink, hipStream_t s);

// marks, when not null, are kBinMarks events recorded between the kernels of
// the binned build, which times its phases (never under capture): after the
// plan, the pass-1 count, its scan, the pass-1 scatter, the pass-2 plan, the
// pass-2 count, its scan, the pass-2 scatter and the segment starts; the
// segment reduce follows the last.
constexpr uint32_t kBinMarks = 9;
hipError_t launch_binned(const PassArgs *args, const Instance *inst, const uint64_t *packed,
                         const uint64_t *ws, InstStatus *st, const BinBuffers &bb, uint64_t n_cap,
                         int device, bool stats, hipStream_t s, hipEvent_t *marks);

// Extraction of a binned table: seg_count (parts entries) is scanned into
// seg_off (parts + 1 entries, using `partials` of ceil(parts / 1024) + 1
// entries and a device word `len` that the call fills with parts), then each
// segment writes its vertices at its offset (segment order; unspecified
// order within a segment).  *out_n receives the total on the device.
// key_words = 2: long keys, written as two words per record.
hipError_t launch_extract_binned(const uint64_t *table, uint32_t entry_words, uint32_t key_words, uint32_t parts,
                                 const uint32_t *seg_count, uint64_t *seg_off, uint64_t *partials,
                                 uint64_t *len, uint64_t *out_keys, uint32_t *out_counts,
                                 uint64_t out_cap, uint64_t *out_n, int device, hipStream_t s);

// Occupancy-derived persistent grid for the build kernel (k <= 32) and for
// the long-k build.
uint32_t build_grid(int device, uint32_t block);
uint32_t build_grid_wide(int device, uint32_t block);

}  // namespace dbgk
