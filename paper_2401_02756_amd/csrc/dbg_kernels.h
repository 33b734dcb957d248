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
// (3 = 24 bytes, 4 = 32 bytes).  Word 0 holds the vertex key with bit 63 set
// (0 means the slot is empty, so a zero fill empties the table); the next
// 16 bytes hold four uint32 counters in letter-code order A, C, T, G.
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
    uint32_t k;
    uint32_t entry_words;
    uint32_t skip;          // nonzero: the host left this instance out
    uint32_t pad;
};

struct InstStatus {
    uint32_t err;       // kErr* bits
    uint32_t pad;
    uint64_t claimed;   // slots claimed by this call
    uint64_t inserts;   // k-mers of this call
    uint64_t windows;   // windows of this call
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

constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kScanPerThread = 4;
constexpr uint32_t kScanReads = kScanBlock * kScanPerThread;  // reads per scan block
constexpr uint32_t kMapReads = 256;  // reads of one tile staged in LDS

inline uint64_t packed_words(uint64_t bytes) { return (bytes + 31) / 32 + 2; }
inline uint64_t scan_blocks(uint64_t n_reads) { return (n_reads + kScanReads - 1) / kScanReads; }
inline uint64_t max_tiles(uint64_t bytes, uint64_t tile) { return bytes / tile + 2; }

// Launchers (all stream-ordered; they only enqueue).
hipError_t launch_prepare(Instance *inst, uint32_t m, InstStatus *st, CallState *cs,
                          const uint64_t *offsets, uint64_t n_reads, hipStream_t s);
hipError_t launch_fill_zero(uint64_t *words, uint64_t n_words, hipStream_t s);
hipError_t launch_pack(const uint8_t *ascii, uint64_t n_bytes, uint64_t *packed,
                       const Instance *inst, uint32_t m, InstStatus *st, hipStream_t s);
hipError_t launch_scan(const uint64_t *offsets, uint64_t n_reads, uint64_t reads_len,
                       bool check_ends, const Instance *inst, uint32_t m, InstStatus *st,
                       uint64_t *ws, uint64_t *partials, uint64_t *tile_read, uint64_t tile_cap,
                       uint32_t tile, CallState *cs, hipStream_t s);
hipError_t launch_build(const Instance *inst, uint32_t m, const uint64_t *packed,
                        const uint64_t *offsets, const uint64_t *ws, const uint64_t *tile_read,
                        uint64_t n_reads, InstStatus *st, CallState *cs, BuildShape shape,
                        hipStream_t s);
hipError_t launch_extract(const uint64_t *table, uint32_t entry_words, uint64_t cap,
                          uint64_t *out_keys, uint32_t *out_counts, uint64_t out_cap,
                          uint64_t *out_n, hipStream_t s);
hipError_t launch_count(const uint64_t *table, uint32_t entry_words, uint64_t cap,
                        uint64_t *out_n, hipStream_t s);
hipError_t launch_roofline(uint64_t *mem, uint64_t words, uint64_t n_ops, uint32_t kind,
                           uint64_t seed, uint32_t block, uint64_t *sink, hipStream_t s);

// Occupancy-derived persistent grid for the build kernel.
uint32_t build_grid(int device, uint32_t block);

}  // namespace dbgk
