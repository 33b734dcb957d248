// Host runtime internals of libdbg shared by the C ABI (dbg_api.hip) and the
// build server (dbg_server.hip): device and pinned buffers, the build pass
// (capacity classes, argument block, graph capture and replay), graph
// handles, table sizing, status folding and the batched pass.
#pragma once

#include "dbg.h"
#include "dbg_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

using dbgk::CallState;
using dbgk::Instance;
using dbgk::InstStatus;

namespace dbgrt {

constexpr uint64_t kCounterLimit = 0xffffffffull;

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
        }
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Grow-only pinned host buffer.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Makes `device` current for the scope of a call and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int device) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (device >= 0 && device != prev) ok = hipSetDevice(device) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline int err_code_of(uint32_t bits) {
    if (bits & dbgk::kErrInval) return DBG_E_INVAL;
    if (bits & dbgk::kErrBase) return DBG_E_BASE;
    if (bits & dbgk::kErrRange) return DBG_E_RANGE;
    if (bits & dbgk::kErrFull) return DBG_E_FULL;
    return DBG_OK;
}

inline bool validation_error(uint32_t bits) {
    return bits & (dbgk::kErrInval | dbgk::kErrBase | dbgk::kErrRange);
}

inline int hip_code(hipError_t e) {
    if (e == hipSuccess) return DBG_OK;
    return e == hipErrorOutOfMemory ? DBG_E_NOMEM : DBG_E_DEVICE;
}

// Windows and k-mers of host-resident offsets; false if offsets decrease.
inline bool host_counts(const uint64_t *off, uint64_t n, uint32_t k, uint64_t *windows, uint64_t *kmers) {
    uint64_t w = 0, e = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (off[i + 1] < off[i]) return false;
        const uint64_t L = off[i + 1] - off[i];
        if (L >= k) {
            w += L - k + 2;
            e += L - k + 1;
        }
    }
    *windows = w;
    *kmers = e;
    return true;
}

inline uint64_t capacity_for(uint64_t vertices, double lf) {
    const double c = std::ceil((double)vertices / lf);
    return std::max<uint64_t>(64, (uint64_t)c);
}

// Capacity of a buffer dimension: x rounded up to a multiple of an eighth of
// its power of two (at most 12.5 % slack), so that calls of similar size share
// buffers and captured graphs.
inline uint64_t size_class(uint64_t x, uint64_t floor) {
    x = std::max(x, floor);
    uint64_t p = 1;
    while (p < x) p <<= 1;
    const uint64_t g = std::max<uint64_t>(p / 8, 1);
    return (x + g - 1) / g * g;
}

// What a captured pass depends on besides its buffers.  Every buffer of a
// pass is sized from these capacities (pass_key, bin_caps, PassSizes).
struct PassKey {
    int binned = 0;
    int stats = 0;  // kernels that keep probe statistics
    uint32_t bin_chunks = 0, bin_div = 0, bin_shape1 = 0, bin_shape2 = 0;  // binned launch shape (dbg_config)
    int single = 0;
    int wide = 0;  // one instance with 32 < k <= 64, direct build
    uint32_t rw = 1;  // binned record words (2: long keys)
    uint32_t ew = 3;
    uint32_t m_cap = 0, d1_cap = 0, fan_cap = 0;
    uint64_t n_cap = 0, len_cap = 0, parts_cap = 0, buckets_cap = 0;
    dbgk::BuildShape shape{};
    bool operator==(const PassKey &o) const {
        return binned == o.binned && stats == o.stats && bin_chunks == o.bin_chunks && bin_div == o.bin_div &&
               bin_shape1 == o.bin_shape1 && bin_shape2 == o.bin_shape2 &&
               single == o.single && wide == o.wide && rw == o.rw && ew == o.ew &&
               m_cap == o.m_cap &&
               d1_cap == o.d1_cap && fan_cap == o.fan_cap && n_cap == o.n_cap && len_cap == o.len_cap &&
               parts_cap == o.parts_cap && buckets_cap == o.buckets_cap && shape.block == o.shape.block &&
               shape.wpt == o.shape.wpt && shape.grid == o.shape.grid && shape.merge == o.shape.merge;
    }
};

// Capacities of a pass over mm instances (host instances hi filled), n reads
// and len bytes.
inline PassKey pass_key(uint32_t mm, uint64_t n, uint64_t len, dbgk::BuildShape shape, bool binned,
                        const Instance *hi) {
    PassKey k;
    k.binned = binned ? 1 : 0;
    k.single = mm == 1 ? 1 : 0;
    k.shape = shape;
    k.wide = (mm == 1 && !binned && hi[0].k > 32) ? 1 : 0;
    k.rw = (mm == 1 && binned && hi[0].k > 32) ? 2 : 1;  // long keys: one graph at a time
    k.m_cap = (uint32_t)size_class(mm, 1);
    k.n_cap = size_class(n, 1024);
    k.len_cap = size_class(len, 4096);
    uint64_t P = 0, G1 = 0;
    uint32_t d1max = 1, fanmax = 1;
    for (uint32_t i = 0; i < mm; ++i) {
        P += hi[i].parts;
        G1 += hi[i].d1;
        d1max = std::max(d1max, hi[i].d1);
        fanmax = std::max(fanmax, hi[i].fan);
        if (hi[i].parts) k.ew = hi[i].entry_words;
    }
    if (binned) {
        k.parts_cap = size_class(P, 64);
        k.buckets_cap = size_class(G1, 64);
        k.d1_cap = (uint32_t)std::min<uint64_t>(size_class(d1max, 16), dbgk::kMaxD1);
        k.fan_cap = (uint32_t)std::min<uint64_t>(size_class(fanmax, 16), dbgk::kMaxFan);
    }
    return k;
}

// Capacities (not pointers) of the binned scratch of a key.
inline void bin_caps(const PassKey &k, dbgk::BinBuffers &bb) {
    // A pass with T tiles takes chunks of max(1, floor(T / target)) tiles
    // (target <= kMaxChunkTarget), so it has at most min(T, 2 target + one
    // partial chunk per instance or bucket) chunks.
    bb.tiles1_cap = k.len_cap / dbgk::kBinTile + k.m_cap + 1;
    bb.chunks1_cap = std::min<uint64_t>(bb.tiles1_cap, 2ull * dbgk::kMaxChunkTarget + k.m_cap) + 1;
    bb.hist1_cap = (uint64_t)k.d1_cap * bb.chunks1_cap;
    bb.tiles2_cap = k.len_cap / dbgk::kRefTile + k.buckets_cap + 1;
    bb.chunks2_cap = std::min<uint64_t>(bb.tiles2_cap, 2ull * dbgk::kMaxChunkTarget + k.buckets_cap) + 1;
    bb.hist2_cap = (uint64_t)k.fan_cap * bb.chunks2_cap;
    const uint64_t chunk = 1024;
    bb.partials_cap = std::max((bb.hist1_cap + chunk - 1) / chunk, (bb.hist2_cap + chunk - 1) / chunk) + 1;
    bb.buckets_cap = k.buckets_cap;
    bb.parts_cap = k.parts_cap;
    bb.d1_max = k.d1_cap;
    bb.fan_max = k.fan_cap;
    bb.entry_words = k.ew;
    bb.rec_words = k.rw;
}

// Byte sizes of every device buffer of a pass with key k (bb: bin_caps(k)).
struct PassSizes {
    // common: packed reads, window prefix, scan partials, arguments, status, tile map
    uint64_t packed, ws, partials, args, status, tiles;
    // binned
    uint64_t plan, buckets, totals, hist1, scan1, hist2, scan2, bpartials, rec1, rec2, pstart, tread1, tile2;
    uint64_t tile_cap;  // direct build: tile map entries
    PassSizes(const PassKey &k, const dbgk::BinBuffers &bb) {
        const uint64_t T = (uint64_t)k.shape.block * k.shape.wpt;
        tile_cap = dbgk::max_tiles(k.len_cap, T);
        packed = dbgk::packed_words(k.len_cap) * 8;
        ws = (k.n_cap + 1) * 8;
        partials = std::max<uint64_t>(1, dbgk::scan_blocks(k.n_cap)) * 16 + 8;
        args = dbgk::kArgsBytes + sizeof(Instance) * k.m_cap;
        status = sizeof(InstStatus) * k.m_cap + sizeof(CallState);
        tiles = k.binned ? 0 : tile_cap * 8;
        const bool b = k.binned != 0;
        plan = b ? sizeof(dbgk::BinPlan) * k.m_cap : 0;
        buckets = b ? sizeof(dbgk::Bucket) * std::max<uint64_t>(k.buckets_cap, 1) : 0;
        totals = b ? sizeof(dbgk::BinTotals) : 0;
        hist1 = b ? 4 * bb.hist1_cap : 0;
        scan1 = b ? 8 * (bb.hist1_cap + 1) : 0;
        hist2 = b ? 4 * bb.hist2_cap : 0;
        scan2 = b ? 8 * (bb.hist2_cap + 1) : 0;
        bpartials = b ? 8 * bb.partials_cap : 0;
        rec1 = b ? 8 * k.rw * k.len_cap : 0;
        rec2 = rec1;
        pstart = b ? 8 * (k.parts_cap + 1) : 0;
        tread1 = b ? 8 * bb.tiles1_cap : 0;
        tile2 = b ? sizeof(dbgk::RefChunk) * bb.chunks2_cap : 0;
    }
};

// Options of a pass besides its input: where its probe statistics go
// (DBG_F_STATS; null: none kept) and whether keys take the test hash.
struct PassOpts {
    uint64_t *stats = nullptr;
    uint32_t test_hash = 0;
    uint32_t bin_chunks = 0, bin_div = 0, bin_shape1 = 0, bin_shape2 = 0;  // binned launch shape (0: defaults)
};

inline PassOpts opts_of(const dbg_graph *g);

// The argument block of a pass (PassArgs) for key k.
inline void fill_args(dbgk::PassArgs &a, const PassKey &k, const PassSizes &z, uint32_t mm, const Instance *hi,
                      const uint8_t *d_reads, uint64_t len, const uint64_t *d_off, uint64_t n, bool check_ends,
                      uint64_t *xkeys, uint32_t *xcounts, uint64_t xcap, const PassOpts &o) {
    const uint64_t T = (uint64_t)k.shape.block * k.shape.wpt;
    uint64_t P = 0;
    for (uint32_t i = 0; i < mm; ++i) P += hi[i].parts;
    std::memset(&a, 0, sizeof a);
    a.reads = d_reads;
    a.off = d_off;
    a.n_reads = n;
    a.reads_len = len;
    a.max_windows = k.binned ? len : (z.tile_cap - 1) * T;
    a.tile_cap = z.tile_cap;
    a.parts_total = P;
    a.m = mm;
    a.check_ends = check_ends ? 1 : 0;
    a.tile = (uint32_t)T;
    a.stats = o.stats;
    a.test_hash = o.test_hash;
    if (k.binned && mm == 1 && xkeys) {
        a.xkeys = xkeys;
        a.xcounts = xcounts;
        a.xcap = xcap;
    }
}

// Buffers and launch sequence of one build pass over m instances.  With
// graphs enabled the pass is captured as two HIP graphs (setup: arguments,
// prepare, pack, scan; build: the build kernels and the status readback) on
// first use of a size class and replayed afterwards; every size and input
// pointer reaches the kernels through the PassArgs block in device memory,
// so a replay needs no kernel argument to change.
struct Pass {
    DevBuf packed, ws, partials, tiles, dargs, dstatus;
    // binned-mode scratch
    DevBuf bplan, bbuckets, btotals, hist1, scan1, hist2, scan2, bpartials, rec1, rec2, pstart;
    DevBuf tread1, tbucket2;
    HostBuf hargs, hstatus;  // pinned: PassArgs + Instance[m_cap]; InstStatus[m_cap] + CallState
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr;
    hipEvent_t marks[dbgk::kBinMarks] = {};  // binned phase boundaries (timed, uncaptured)
    bool marked = false;
    hipStream_t cap_stream = nullptr;
    uint32_t m = 0;
    hipStream_t stream = nullptr;
    bool pending = false;
    bool timing = false;
    bool use_graphs = false;
    uint64_t generation = 0;  // bumped whenever a buffer moves
    struct Cached {
        PassKey key;
        uint64_t generation;
        hipGraphExec_t setup, build;
    };
    std::vector<Cached> graphs;
    uint64_t captures = 0, replays = 0;
    uint32_t shapes = 0;  // scatter shapes of the last binned pass, as dbg_stats reports them (shape + 1)

    hipError_t init() {
        hipError_t e = hipEventCreate(&ev_a);
        if (e == hipSuccess) e = hipEventCreate(&ev_b);
        if (e == hipSuccess) e = hipEventCreate(&ev_c);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
        for (hipEvent_t &x : marks)
            if (e == hipSuccess) e = hipEventCreate(&x);
        return e;
    }
    void drop_graphs() {
        for (auto &c : graphs) {
            if (c.setup) (void)hipGraphExecDestroy(c.setup);
            if (c.build) (void)hipGraphExecDestroy(c.build);
        }
        graphs.clear();
    }
    void release() {
        drop_graphs();
        DevBuf *d[] = {&packed, &ws, &partials, &tiles, &dargs, &dstatus, &bplan, &bbuckets,
                       &btotals, &hist1, &scan1, &hist2, &scan2, &bpartials, &rec1, &rec2, &pstart,
                       &tread1, &tbucket2};
        for (DevBuf *b : d) b->release();
        hargs.release();
        hstatus.release();
        if (ev_a) (void)hipEventDestroy(ev_a);
        if (ev_b) (void)hipEventDestroy(ev_b);
        if (ev_c) (void)hipEventDestroy(ev_c);
        for (hipEvent_t &x : marks)
            if (x) (void)hipEventDestroy(x), x = nullptr;
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        ev_a = ev_b = ev_c = nullptr;
        cap_stream = nullptr;
    }
    // Grow a buffer; a move invalidates every captured graph.
    hipError_t grow(DevBuf &b, size_t bytes) {
        const void *old = b.p;
        const hipError_t e = b.reserve(bytes);
        if (b.p != old && old) ++generation;
        return e;
    }
    hipError_t reserve_instances(uint32_t mm) {
        const uint32_t m_cap = (uint32_t)size_class(mm, 1);
        const void *pa = hargs.p, *ps = hstatus.p;
        hipError_t e = hargs.reserve(dbgk::kArgsBytes + sizeof(Instance) * m_cap);
        if (e == hipSuccess) e = hstatus.reserve(sizeof(InstStatus) * m_cap + sizeof(CallState));
        if ((pa && hargs.p != pa) || (ps && hstatus.p != ps)) ++generation;  // graphs copy from these
        return e;
    }
    dbgk::PassArgs *host_args() const { return hargs.as<dbgk::PassArgs>(); }
    Instance *host_instances() const {
        return reinterpret_cast<Instance *>(hargs.as<unsigned char>() + dbgk::kArgsBytes);
    }
    const InstStatus *host_status() const { return hstatus.as<InstStatus>(); }

    // Reserve the binned-mode scratch for the key's capacities.
    hipError_t reserve_binned(const PassKey &k, dbgk::BinBuffers &bb) {
        bin_caps(k, bb);
        const PassSizes z(k, bb);
        hipError_t e;
        if ((e = grow(bplan, z.plan)) != hipSuccess || (e = grow(bbuckets, z.buckets)) != hipSuccess ||
            (e = grow(btotals, z.totals)) != hipSuccess || (e = grow(hist1, z.hist1)) != hipSuccess ||
            (e = grow(scan1, z.scan1)) != hipSuccess || (e = grow(hist2, z.hist2)) != hipSuccess ||
            (e = grow(scan2, z.scan2)) != hipSuccess || (e = grow(bpartials, z.bpartials)) != hipSuccess ||
            (e = grow(rec1, z.rec1)) != hipSuccess || (e = grow(rec2, z.rec2)) != hipSuccess ||
            (e = grow(pstart, z.pstart)) != hipSuccess || (e = grow(tread1, z.tread1)) != hipSuccess ||
            (e = grow(tbucket2, z.tile2)) != hipSuccess)
            return e;
        bb.plan = bplan.as<dbgk::BinPlan>();
        bb.buckets = bbuckets.as<dbgk::Bucket>();
        bb.totals = btotals.as<dbgk::BinTotals>();
        bb.hist1 = hist1.as<uint32_t>();
        bb.scan1 = scan1.as<uint64_t>();
        bb.hist2 = hist2.as<uint32_t>();
        bb.scan2 = scan2.as<uint64_t>();
        bb.partials = bpartials.as<uint64_t>();
        bb.rec1 = rec1.as<uint64_t>();
        bb.rec2 = rec2.as<uint64_t>();
        bb.pstart = pstart.as<uint64_t>();
        bb.tile_read1 = tread1.as<uint64_t>();
        bb.chunk2 = tbucket2.as<dbgk::RefChunk>();
        return hipSuccess;
    }
    // Grid sizes per binned key (queried once, outside any capture).
    std::vector<std::pair<PassKey, dbgk::BinBuffers>> grid_memo;
    void binned_grids(const PassKey &k, int device, dbgk::BinBuffers &bb) {
        for (auto &g : grid_memo)
            if (g.first == k) {
                bb.grid_bin_count = g.second.grid_bin_count;
                bb.grid_bin_scatter = g.second.grid_bin_scatter;
                bb.grid_ref_count = g.second.grid_ref_count;
                bb.grid_ref_scatter = g.second.grid_ref_scatter;
                bb.grid_reduce = g.second.grid_reduce;
                bb.target1 = g.second.target1;
                bb.target2 = g.second.target2;
                bb.shape1 = g.second.shape1;
                bb.shape2 = g.second.shape2;
                return;
            }
        bb.chunks_per_group = k.bin_chunks;
        bb.scatter_div = k.bin_div;
        bb.shape_req1 = k.bin_shape1;
        bb.shape_req2 = k.bin_shape2;
        dbgk::binned_grids(device, bb);
        if (grid_memo.size() > 16) grid_memo.clear();
        grid_memo.emplace_back(k, bb);
    }

    // The two halves of the pass, enqueued on `s` (directly or under capture).
    hipError_t enqueue_setup(const PassKey &k, hipStream_t s) {
        dbgk::PassArgs *da = dargs.as<dbgk::PassArgs>();
        Instance *di = reinterpret_cast<Instance *>(dargs.as<unsigned char>() + dbgk::kArgsBytes);
        InstStatus *dst = dstatus.as<InstStatus>();
        CallState *cs = reinterpret_cast<CallState *>(dst + k.m_cap);
        hipError_t e = hipMemcpyAsync(dargs.p, hargs.p, dbgk::kArgsBytes + sizeof(Instance) * k.m_cap,
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = dbgk::launch_prepare(da, di, dst, cs, k.m_cap, s);
        if (e == hipSuccess) e = dbgk::launch_pack(da, packed.as<uint64_t>(), di, dst, k.len_cap, s);
        if (e == hipSuccess)
            e = dbgk::launch_scan(da, di, dst, ws.as<uint64_t>(), partials.as<uint64_t>(),
                                  k.binned ? nullptr : tiles.as<uint64_t>(), cs, k.n_cap, s);
        return e;
    }
    hipError_t enqueue_build(const PassKey &k, const dbgk::BinBuffers &bb, int device, hipStream_t s,
                             bool mark = false) {
        dbgk::PassArgs *da = dargs.as<dbgk::PassArgs>();
        Instance *di = reinterpret_cast<Instance *>(dargs.as<unsigned char>() + dbgk::kArgsBytes);
        InstStatus *dst = dstatus.as<InstStatus>();
        CallState *cs = reinterpret_cast<CallState *>(dst + k.m_cap);
        hipError_t e;
        if (k.wide)
            e = dbgk::launch_build_wide(da, di, packed.as<uint64_t>(), ws.as<uint64_t>(), tiles.as<uint64_t>(), dst,
                                        cs, k.shape, k.stats != 0, s);
        else if (k.binned)
            e = dbgk::launch_binned(da, di, packed.as<uint64_t>(), ws.as<uint64_t>(), dst, bb, k.n_cap, device,
                                    k.stats != 0, s,
                                    mark ? marks : nullptr);
        else
            e = dbgk::launch_build(da, di, packed.as<uint64_t>(), ws.as<uint64_t>(), tiles.as<uint64_t>(), dst,
                                   cs, k.shape, k.single != 0, k.stats != 0, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hstatus.p, dstatus.p, sizeof(InstStatus) * k.m_cap + sizeof(CallState),
                               hipMemcpyDeviceToHost, s);
        return e;
    }

    hipError_t capture(const PassKey &k, const dbgk::BinBuffers &bb, int device, Cached &out) {
        out.key = k;
        out.generation = generation;
        out.setup = out.build = nullptr;
        for (int half = 0; half < 2; ++half) {
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            const hipError_t ee = half == 0 ? enqueue_setup(k, cap_stream) : enqueue_build(k, bb, device, cap_stream);
            e = hipStreamEndCapture(cap_stream, &g);
            if (ee != hipSuccess) e = ee;
            if (e == hipSuccess) e = hipGraphInstantiate(half == 0 ? &out.setup : &out.build, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
        }
        ++captures;
        return hipSuccess;
    }

    // Enqueue the pass.  hinst[0..mm) must be filled (tables, read ranges,
    // prior k-mers, k, entry words, and the segment geometry when binned).
    // Reads are device-resident: read i is d_reads[off[i] - off[0] ..
    // off[i+1] - off[0]).
    // xkeys / xcounts / xcap: the fused extraction of a one-instance binned
    // pass (PassArgs); null otherwise.
    hipError_t enqueue(uint32_t mm, const uint8_t *d_reads, uint64_t len, const uint64_t *d_off,
                       uint64_t n, dbgk::BuildShape shape, bool binned, int device, bool check_ends,
                       bool time_it, hipStream_t s, const PassOpts &o, uint64_t *xkeys = nullptr,
                       uint32_t *xcounts = nullptr, uint64_t xcap = 0) {
        const Instance *hi = host_instances();
        PassKey k = pass_key(mm, n, len, shape, binned, hi);
        k.stats = o.stats != nullptr;
        k.bin_chunks = o.bin_chunks;
        k.bin_div = o.bin_div;
        k.bin_shape1 = o.bin_shape1;
        k.bin_shape2 = o.bin_shape2;
        dbgk::BinBuffers bb{};
        if (binned) bin_caps(k, bb);
        const PassSizes z(k, bb);
        hipError_t e;
        if ((e = grow(packed, z.packed)) != hipSuccess || (e = grow(ws, z.ws)) != hipSuccess ||
            (e = grow(partials, z.partials)) != hipSuccess || (e = grow(dargs, z.args)) != hipSuccess ||
            (e = grow(dstatus, z.status)) != hipSuccess || (!binned && (e = grow(tiles, z.tiles)) != hipSuccess) ||
            (binned && (e = reserve_binned(k, bb)) != hipSuccess))
            return e;
        if (binned) {
            binned_grids(k, device, bb);
            shapes = (bb.shape1 + 1) | (bb.shape2 + 1) << 8;
        }
        fill_args(*host_args(), k, z, mm, hi, d_reads, len, d_off, n, check_ends, xkeys, xcounts, xcap, o);

        Cached *c = nullptr;
        if (use_graphs) {
            for (auto &x : graphs)
                if (x.key == k && x.generation == generation) c = &x;
            if (!c) {
                if (graphs.size() >= 8 || (!graphs.empty() && graphs[0].generation != generation)) drop_graphs();
                Cached fresh{};
                e = capture(k, bb, device, fresh);
                if (e != hipSuccess) {
                    if (fresh.setup) (void)hipGraphExecDestroy(fresh.setup);
                    if (fresh.build) (void)hipGraphExecDestroy(fresh.build);
                    return e;
                }
                graphs.push_back(fresh);
                c = &graphs.back();
            } else {
                ++replays;
            }
        }
        if (time_it) (void)hipEventRecord(ev_a, s);
        e = c ? hipGraphLaunch(c->setup, s) : enqueue_setup(k, s);
        if (time_it && e == hipSuccess) (void)hipEventRecord(ev_b, s);
        marked = !c && time_it && binned;
        if (e == hipSuccess) e = c ? hipGraphLaunch(c->build, s) : enqueue_build(k, bb, device, s, marked);
        if (time_it && e == hipSuccess) (void)hipEventRecord(ev_c, s);
        if (e != hipSuccess) return e;
        m = mm;
        stream = s;
        pending = true;
        timing = time_it;
        return hipSuccess;
    }

    // Phase times of the last timed pass, in ms: setup, then (binned,
    // uncaptured) the kBinMarks + 1 phases between the marks and the end of
    // the pass, or (otherwise) the whole build.
    double phase_ms[dbgk::kBinMarks + 2] = {};
    uint32_t n_phases = 0;

    // Wait for the enqueued pass; times in ms when it was timed.
    hipError_t wait(double *build_ms, double *total_ms) {
        if (!pending) return hipSuccess;
        pending = false;
        hipError_t e = hipStreamSynchronize(stream);
        if (e == hipSuccess && timing) {
            float a = 0, b = 0, x = 0;
            if (hipEventElapsedTime(&a, ev_b, ev_c) == hipSuccess && build_ms) *build_ms = a;
            if (hipEventElapsedTime(&b, ev_a, ev_c) == hipSuccess && total_ms) *total_ms = b;
            n_phases = 0;
            if (hipEventElapsedTime(&x, ev_a, ev_b) == hipSuccess) phase_ms[n_phases++] = x;
            if (marked) {
                hipEvent_t prev = ev_b;
                for (hipEvent_t m : marks) {
                    phase_ms[n_phases++] = hipEventElapsedTime(&x, prev, m) == hipSuccess ? x : 0.0;
                    prev = m;
                }
                phase_ms[n_phases++] = hipEventElapsedTime(&x, prev, ev_c) == hipSuccess ? x : 0.0;
            } else {
                phase_ms[n_phases++] = a;
            }
        }
        return e;
    }
};

}  // namespace dbgrt

// Contigs of a graph (dbg_contigs.hip): device buffers kept until the next
// build or reset.
struct dbg_contig_state;
void dbg_contigs_free(dbg_contig_state *cs);

struct dbg_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t flags = 0;
    double lf = 0.5;
    uint64_t expected = 0, cap_req = 0;
    dbgk::BuildShape shape{256, 4, 0, 0};
    uint32_t grid_wide = 0;  // persistent grid of the long-k build
    uint32_t bin_chunks = 0, bin_div = 0, bin_shape1 = 0, bin_shape2 = 0;  // binned launch shape (dbg_config)

    uint64_t cap = 0;
    uint32_t ew = 3;
    dbgrt::DevBuf table;
    bool binned = false;     // table cut into segments, built by the binned kernels
    bool fresh = true;       // binned: logically empty (contents need not be zero)
    uint32_t parts = 0, d1 = 0, fan = 0;
    dbgrt::DevBuf seg_count, seg_off, seg_partials, seg_len;  // binned: per-segment occupancy

    // A zero fill enqueued on `stream` (direct tables) that a build enqueued
    // on another stream must wait for.
    hipEvent_t zero_ev = nullptr;
    bool zero_wait = false;

    uint32_t k = 0;
    int32_t poisoned = DBG_OK;
    int32_t unreported = DBG_OK;

    dbgrt::Pass pass;
    uint32_t pending_k = 0;
    dbgrt::DevBuf reads, offsets;   // staging of host input
    dbgrt::DevBuf xkeys, xcnt, xn;  // extraction staging
    dbgrt::DevBuf pstats;           // probe statistics (DBG_F_STATS): dbgk::kStatWords words
    dbgrt::DevBuf nkeys, ncnt, n8;  // normalized extraction staging

    uint64_t vertices = 0, inserts = 0, windows = 0, builds = 0;
    uint64_t epoch = 0;  // advanced by every build and reset
    double last_build_ms = 0, last_total_ms = 0;
    dbg_contig_state *contigs = nullptr;

    hipStream_t pick(void *s) const { return s ? static_cast<hipStream_t>(s) : stream; }
    uint64_t table_words() const { return cap * ew; }
};

namespace dbgrt {

inline PassOpts opts_of(const dbg_graph *g) {
    PassOpts o;
    o.stats = (g->flags & DBG_F_STATS) ? g->pstats.as<uint64_t>() : nullptr;
    o.test_hash = (g->flags & DBG_F_TEST_HASH) ? 1u : 0u;
    o.bin_chunks = g->bin_chunks;
    o.bin_div = g->bin_div;
    o.bin_shape1 = g->bin_shape1;
    o.bin_shape2 = g->bin_shape2;
    return o;
}

// Segment geometry of a binned table of at least `cap` slots: d1 level-1
// buckets of `fan` segments each (about the square root, so both partition
// passes write runs of similar length), d1 * fan segments of kSegSlots slots
// in all (a segment is a pair of digits of the key image).  False if the
// table is too large for the two levels.
inline bool binned_geometry(uint64_t cap, uint32_t *d1, uint32_t *fan, uint64_t *parts) {
    const uint64_t want = std::max<uint64_t>(1, (cap + dbgk::kSegSlots - 1) / dbgk::kSegSlots);
    uint64_t target = (uint64_t)std::ceil(std::sqrt((double)want));
    target = std::max<uint64_t>(1, std::min<uint64_t>(target, dbgk::kMaxD1));
    const uint64_t f = (want + target - 1) / target;
    if (f > dbgk::kMaxFan) return false;
    *fan = (uint32_t)f;
    *d1 = (uint32_t)((want + f - 1) / f);
    *parts = (uint64_t)*d1 * f;
    return true;
}

// Zero the whole table on the graph's stream; builds on other streams are
// ordered after it by order_after_zero.
inline hipError_t zero_table(dbg_graph *g) {
    hipError_t e = dbgk::launch_fill_zero(g->table.as<uint64_t>(), g->table_words(), g->stream);
    if (e == hipSuccess && g->zero_ev) e = hipEventRecord(g->zero_ev, g->stream);
    if (e == hipSuccess) g->zero_wait = g->zero_ev != nullptr;
    return e;
}

// Zero the probe statistics (DBG_F_STATS) on the graph's stream, ordered
// before later builds on other streams like a table fill.
inline hipError_t zero_stats(dbg_graph *g) {
    hipError_t e = dbgk::launch_fill_zero(g->pstats.as<uint64_t>(), dbgk::kStatWords, g->stream);
    if (e == hipSuccess && g->zero_ev) e = hipEventRecord(g->zero_ev, g->stream);
    if (e == hipSuccess) g->zero_wait = g->zero_ev != nullptr;
    return e;
}

inline hipError_t order_after_zero(dbg_graph *g, hipStream_t s) {
    if (!g->zero_wait) return hipSuccess;
    g->zero_wait = false;
    return s == g->stream ? hipSuccess : hipStreamWaitEvent(s, g->zero_ev, 0);
}

inline hipError_t allocate_table(dbg_graph *g, uint64_t cap) {
    if (g->binned) {
        uint64_t parts = 0;
        if (!binned_geometry(cap, &g->d1, &g->fan, &parts)) return hipErrorInvalidValue;
        g->parts = (uint32_t)parts;
        cap = parts * dbgk::kSegSlots;
        hipError_t e;
        if ((e = g->seg_count.reserve(4 * parts)) != hipSuccess ||
            (e = g->seg_off.reserve(8 * (parts + 1))) != hipSuccess ||
            (e = g->seg_partials.reserve(8 * ((parts + 1023) / 1024 + 2))) != hipSuccess ||
            (e = g->seg_len.reserve(8)) != hipSuccess)
            return e;
    }
    g->cap = cap;
    hipError_t e = g->table.reserve(g->table_words() * sizeof(uint64_t));
    if (e != hipSuccess) {
        g->cap = 0;
        return e;
    }
    // a binned build rewrites every segment of a fresh table: no zeros needed
    return g->binned ? hipSuccess : zero_table(g);
}

inline int ensure_table(dbg_graph *g, uint64_t windows_bound) {
    if (g->cap) return DBG_OK;
    uint64_t cap = g->cap_req;
    if (!cap) cap = capacity_for(g->expected ? g->expected : std::max<uint64_t>(windows_bound, 1), g->lf);
    const hipError_t e = allocate_table(g, cap);
    if (e == hipErrorInvalidValue) return DBG_E_INVAL;
    g->fresh = true;
    return hip_code(e);
}

// Binned builds take k <= 31 (one-word records) and 33 <= k <= 63 (two-word
// records).  A binned graph whose first build has k = 32 or 64 becomes a
// direct one; its table must then hold zeros.  A build with k > 32 needs
// 32-byte entries (two key words): the graph's table is re-allocated for
// them before its first build.
inline bool binnable_k(uint32_t k) { return k <= 31 || (k >= 33 && k <= 63); }

inline int settle_mode(dbg_graph *g, uint32_t k) {
    const bool wide = k > 32 && g->ew != 4;
    if (!wide && (!g->binned || binnable_k(k))) return DBG_OK;
    if (g->k || g->vertices) return DBG_E_K;
    if (!binnable_k(k)) g->binned = false;
    if (wide) {
        g->ew = 4;
        if (g->cap) {
            g->table.release();
            const hipError_t e = g->table.reserve(g->table_words() * sizeof(uint64_t));
            if (e != hipSuccess) {
                g->cap = 0;
                return hip_code(e);
            }
        }
    }
    // a binned table is rewritten from scratch by its first build
    if (g->cap && !g->binned && zero_table(g) != hipSuccess) return DBG_E_DEVICE;
    return DBG_OK;
}

inline void fill_instance(Instance &in, dbg_graph *g, uint64_t read_begin, uint64_t read_end, uint32_t k) {
    in.table = g->table.as<uint64_t>();
    in.cap = g->cap;
    in.read_begin = read_begin;
    in.read_end = read_end;
    in.byte_begin = 0;
    in.byte_end = 0;
    in.prior_inserts = g->inserts;
    in.k = k;
    in.entry_words = g->ew;
    in.skip = 0;
    in.part_base = 0;
    in.parts = g->binned ? g->parts : 0;
    in.d1 = g->binned ? g->d1 : 0;
    in.fan = g->binned ? g->fan : 0;
    in.fresh = (g->binned && g->fresh) ? 1u : 0u;
    in.seg_count = g->binned ? g->seg_count.as<uint32_t>() : nullptr;
    in.reserved = 0;
    in.pad = 0;
}

// Fold one instance's status of a finished pass into its graph.
inline int fold_status(dbg_graph *g, const InstStatus &st, uint32_t k) {
    if (validation_error(st.err)) {  // nothing was modified
        // an empty graph whose table was sized from this rejected input is
        // sized again, from its input, by the next build
        if (g->builds == 0 && !g->cap_req && !g->expected) g->cap = 0;
        return err_code_of(st.err);
    }
    g->k = k;
    g->fresh = false;
    ++g->epoch;
    g->vertices += st.claimed;
    g->inserts += st.inserts;
    g->windows += st.windows;
    g->builds += 1;
    if (st.err & dbgk::kErrFull) {
        g->poisoned = DBG_E_FULL;
        return DBG_E_FULL;
    }
    return DBG_OK;
}

// Waits for the handle's own enqueued build and folds its status.
inline int harvest(dbg_graph *g) {
    if (!g->pass.pending) return DBG_OK;
    if (g->pass.wait(&g->last_build_ms, &g->last_total_ms) != hipSuccess) return DBG_E_DEVICE;
    return fold_status(g, g->pass.host_status()[0], g->pending_k);
}

// uint64 words per extracted key: two for a long-k graph.
inline uint64_t key_words(const dbg_graph *g) { return g->k > 32 ? 2 : 1; }

// Largest k of a plain build, and of every other path (batches, the
// server, contigs), whose keys must fit one word.
constexpr uint32_t kMaxK = 64;
constexpr uint32_t kMaxKWord = 32;

inline int check_common(dbg_graph *g, uint32_t k, uint32_t kmax = kMaxKWord) {
    if (!g) return DBG_E_INVAL;
    if (g->poisoned) return DBG_E_STATE;
    if (k < 2 || k > kmax) return DBG_E_K;
    if (g->k && g->k != k) return DBG_E_K;
    return DBG_OK;
}

inline int enqueue_single(dbg_graph *g, const uint8_t *d_reads, uint64_t len, const uint64_t *d_off,
                   uint64_t n, uint32_t k, hipStream_t s, uint64_t *xkeys = nullptr, uint32_t *xcounts = nullptr,
                   uint64_t xcap = 0) {
    hipError_t e = g->pass.reserve_instances(1);
    if (e != hipSuccess) return hip_code(e);
    fill_instance(g->pass.host_instances()[0], g, 0, n, k);
    if ((e = order_after_zero(g, s)) != hipSuccess) return hip_code(e);
    dbgk::BuildShape shape = g->shape;
    if (k > 32) {
        shape.grid = g->grid_wide;
        shape.merge = 0;
    }
    e = g->pass.enqueue(1, d_reads, len, d_off, n, shape, g->binned, g->device, true,
                        (g->flags & DBG_F_TIMING) != 0, s, opts_of(g), xkeys, xcounts, xcap);
    if (e != hipSuccess) return hip_code(e);
    g->pending_k = k;
    return DBG_OK;
}

// ---------------------------------------------------------------- batch context

// Per-device scratch of batched builds (one batched call at a time per
// device; calls are serialised by the mutex).
struct BatchCtx {
    std::mutex mu;
    hipStream_t stream = nullptr;
    Pass pass;
    DevBuf reads, offsets;
    DevBuf sizing;  // instance boundaries of a batch whose graphs are sized from their inputs
    std::vector<uint64_t> hoff;
    bool ready = false;
};

inline std::mutex g_ctx_mu;
inline std::map<int, std::unique_ptr<BatchCtx>> g_ctx;

inline BatchCtx *batch_ctx(int device) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto &p = g_ctx[device];
    if (!p) p.reset(new BatchCtx());
    return p.get();
}

}  // namespace dbgrt

namespace dbgrt {

// One batched pass between its enqueue and its finish.
struct BatchRun {
    std::vector<dbg_graph *> graphs;
    std::vector<uint32_t> ks;
    std::vector<uint8_t> run;  // graph i takes part in the launch
    bool launched = false;
    bool timing = false;
    hipError_t error = hipSuccess;
};

// Enqueue one batched pass (not waiting for it): graphs[i] takes reads
// [read_begin[i], read_begin[i+1]) of the device-resident concatenation.  A
// graph that fails a host-side check stays in the launch as a skipped
// instance, so its reads are attributed to it and never touched; its status
// is final here.  The others get their status from batch_finish.
// bounds[i] bounds instance i's windows (its byte count will do); a graph
// never sized is sized from its own bound, as dbg_build sizes it.
inline void batch_enqueue(dbg_graph *const *graphs, uint32_t m, const uint64_t *read_begin,
                          const uint32_t *ks, const uint8_t *d_reads, uint64_t reads_len,
                          const uint64_t *d_offsets, const uint64_t *bounds, int32_t *statuses,
                          hipStream_t stream, Pass &pass, bool check_ends, BatchRun &br) {
    br = BatchRun();
    br.graphs.assign(graphs, graphs + m);
    br.ks.assign(ks, ks + m);
    br.run.assign(m, 0);
    const int device = graphs[0]->device;
    uint32_t n_run = 0;
    int mode = -1;  // direct (0) or binned with 3/4-word entries: the first graph that runs decides
    for (uint32_t i = 0; i < m; ++i) {
        dbg_graph *g = graphs[i];
        int rc = check_common(g, ks[i]);
        if (rc == DBG_OK && g->device != device) rc = DBG_E_INVAL;
        if (rc == DBG_OK && read_begin[i + 1] < read_begin[i]) rc = DBG_E_INVAL;
        for (uint32_t j = 0; rc == DBG_OK && j < i; ++j)
            if (graphs[j] == g) rc = DBG_E_INVAL;  // one graph per instance
        if (rc == DBG_OK && g->pass.pending) rc = harvest(g);
        if (rc == DBG_OK && read_begin[i + 1] > read_begin[i]) {
            rc = ensure_table(g, std::max<uint64_t>(bounds[i], 1));
            if (rc == DBG_OK) rc = settle_mode(g, ks[i]);
            // binned launches share one entry width, and a launch one home-slot function
            const int gm = (g->binned ? (int)g->ew : 0) | ((g->flags & DBG_F_TEST_HASH) ? 16 : 0);
            if (rc == DBG_OK && mode < 0) mode = gm;
            if (rc == DBG_OK && gm != mode) rc = DBG_E_INVAL;  // one mode per launch
            if (rc == DBG_OK) {
                br.run[i] = 1;
                ++n_run;
            }
        }
        statuses[i] = rc;
    }
    if (!n_run) return;

    hipError_t e = pass.reserve_instances(m);
    if (e != hipSuccess) {
        for (uint32_t i = 0; i < m; ++i)
            if (br.run[i]) statuses[i] = hip_code(e);
        return;
    }
    Instance *hi = pass.host_instances();
    const dbg_graph *g0 = nullptr;
    uint64_t part_base = 0;
    for (uint32_t i = 0; i < m; ++i) {
        fill_instance(hi[i], graphs[i], read_begin[i], read_begin[i + 1], br.run[i] ? ks[i] : 31u);
        hi[i].skip = br.run[i] ? 0u : 1u;
        if ((mode & 15) == 0 || !br.run[i]) {
            // segments only for the graphs a binned launch builds
            hi[i].parts = hi[i].d1 = hi[i].fan = 0;
            hi[i].fresh = 0;
        }
        hi[i].part_base = part_base;
        part_base += hi[i].parts;
        if (br.run[i] && !g0) g0 = graphs[i];
    }
    for (uint32_t i = 0; i < m && e == hipSuccess; ++i)
        if (br.run[i]) e = order_after_zero(graphs[i], stream);
    if (e != hipSuccess) {
        for (uint32_t i = 0; i < m; ++i)
            if (br.run[i]) statuses[i] = hip_code(e);
        return;
    }
    br.timing = (g0->flags & DBG_F_TIMING) != 0;
    pass.use_graphs = (g0->flags & DBG_F_GRAPH) != 0;
    const uint64_t n = read_begin[m];
    PassOpts o = opts_of(g0);  // the first graph's launch shape; batched passes keep no probe statistics
    o.stats = nullptr;
    o.test_hash = (mode & 16) ? 1u : 0u;
    br.error = pass.enqueue(m, d_reads, reads_len, d_offsets, n, g0->shape, (mode & 15) != 0, device, check_ends,
                            br.timing, stream, o);
    br.launched = br.error == hipSuccess;
}

// Wait for an enqueued batched pass and fold each graph's status.
inline void batch_finish(BatchRun &br, Pass &pass, int32_t *statuses) {
    const uint32_t m = (uint32_t)br.graphs.size();
    double bms = 0, tms = 0;
    hipError_t e = br.error;
    if (br.launched) e = pass.wait(&bms, &tms);
    const InstStatus *st = pass.host_status();
    for (uint32_t i = 0; i < m; ++i) {
        if (!br.run[i]) continue;
        if (e != hipSuccess) {
            statuses[i] = DBG_E_DEVICE;
            continue;
        }
        statuses[i] = fold_status(br.graphs[i], st[i], br.ks[i]);
        if (br.timing) {
            br.graphs[i]->last_build_ms = bms;
            br.graphs[i]->last_total_ms = tms;
        }
    }
    br.launched = false;
}

// Both halves, synchronously.  bounds as for batch_enqueue; NULL: each
// instance's byte count, read from the device offsets when some graph of the
// batch still has to be sized.
inline void batch_device_impl(dbg_graph *const *graphs, uint32_t m, const uint64_t *read_begin,
                              const uint32_t *ks, const uint8_t *d_reads, uint64_t reads_len,
                              const uint64_t *d_offsets, const uint64_t *bounds, int32_t *statuses,
                              hipStream_t stream, BatchCtx *ctx, bool check_ends) {
    std::vector<uint64_t> own;
    if (!bounds) {
        own.assign(m, 0);
        bool unsized = false;
        for (uint32_t i = 0; i < m; ++i) unsized |= graphs[i] && !graphs[i]->cap;
        if (unsized) {
            // offsets at every instance boundary: a gather on the device, one copy back
            hipError_t e = ctx->sizing.reserve(16 * (uint64_t)(m + 1));
            uint64_t *d_idx = ctx->sizing.as<uint64_t>(), *d_at = d_idx + (m + 1);
            std::vector<uint64_t> at(m + 1, 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_idx, read_begin, 8 * (uint64_t)(m + 1), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = dbgk::launch_gather_u64(d_offsets, d_idx, m + 1, d_at, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(at.data(), d_at, 8 * (uint64_t)(m + 1), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                for (uint32_t i = 0; i < m; ++i) statuses[i] = hip_code(e);
                return;
            }
            // bytes of instance i (clamped: inconsistent offsets are the device checks' to report)
            for (uint32_t i = 0; i < m; ++i)
                own[i] = at[i + 1] >= at[i] ? std::min(at[i + 1] - at[i], reads_len) : reads_len;
        }
        bounds = own.data();
    }
    BatchRun br;
    batch_enqueue(graphs, m, read_begin, ks, d_reads, reads_len, d_offsets, bounds, statuses, stream, ctx->pass,
                  check_ends, br);
    batch_finish(br, ctx->pass, statuses);
}

inline int first_error(const int32_t *statuses, uint32_t m) {
    for (uint32_t i = 0; i < m; ++i)
        if (statuses[i] != DBG_OK) return statuses[i];
    return DBG_OK;
}


}  // namespace dbgrt
