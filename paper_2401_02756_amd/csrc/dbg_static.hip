// dbg_build_device_static: dbg_build_device for callers that cannot allocate
// device memory.  Every scratch buffer of the build pass (packed reads, window
// prefix, scan partials, argument block, status words, tile map and, for a
// binned graph, the partition records, histograms and segment starts) is
// carved out of one file-scope device array of kStaticScratchBytes, and the
// argument block reaches the device as kernel arguments, so the call makes no
// allocation of any kind: no hipMalloc/hipFree, no pinned host buffer, no
// library routine that allocates.  The graph's table must already exist.
//
// Each device that runs the call holds its own copy of the array (at its own
// address, looked up once per device with hipGetSymbolAddress) until the
// process ends.  Calls on one device share that copy: a per-device lock
// serialises them, and the call is synchronous, so two calls never overlap
// on the array within a process.  The array keeps the last call's contents;
// the pass writes every word it reads (the prepare kernel clears the status
// words and counters), so nothing needs to start at zero.
#include "dbg_runtime.h"

using namespace dbgrt;
using dbgk::CallState;
using dbgk::Instance;
using dbgk::InstStatus;

namespace {

constexpr uint64_t kStaticScratchBytes = 256ull << 20;  // per device
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Per device: the array's device address (never the host-side name of the
// array, which is no device address) and the lock that serialises calls.
struct StaticSlot {
    std::mutex mu;
    unsigned char *ptr = nullptr;
    bool looked_up = false;
};
StaticSlot g_slots[kStaticMaxDevices];

// The pass's argument block and its one instance, stored by a kernel from its
// arguments (no host staging buffer, no copy from host memory).
__global__ void k_put_args(dbgk::PassArgs a, Instance in, unsigned char *dargs) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *reinterpret_cast<dbgk::PassArgs *>(dargs) = a;
        *reinterpret_cast<Instance *>(dargs + dbgk::kArgsBytes) = in;
    }
}

// Bump allocation of sub-buffers of the scratch array, 256-byte aligned.
struct Carve {
    uint64_t used = 0;
    uint64_t take(uint64_t bytes) {
        const uint64_t at = (used + 255) & ~255ull;
        used = at + std::max<uint64_t>(bytes, 1);
        return at;
    }
};

}  // namespace

extern "C" int dbg_build_device_static(dbg_graph *g, const uint8_t *d_reads, uint64_t reads_len,
                                       const uint64_t *d_offsets, uint64_t n_reads, uint32_t k, void *stream) {
    int rc = check_common(g, k, kMaxKWord);
    if (rc != DBG_OK) return rc;
    if (n_reads == 0) return DBG_OK;
    if (!d_offsets || (!d_reads && reads_len)) return DBG_E_INVAL;
    if (g->device < 0 || g->device >= kStaticMaxDevices) return DBG_E_INVAL;
    if (!g->cap) return DBG_E_INVAL;  // sizing the table would allocate it
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    StaticSlot &slot = g_slots[g->device];
    std::lock_guard<std::mutex> lk(slot.mu);
    if (!slot.looked_up) {
        // once per device, with that device current
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DBG_E_DEVICE;
        slot.ptr = static_cast<unsigned char *>(p);
        slot.looked_up = true;
    }
    if (g->pass.pending) {
        rc = harvest(g);
        if (rc != DBG_OK) return rc;
    }
    hipStream_t s = g->pick(stream);

    // The pass this input needs, and whether its buffers fit the array:
    // checked before any device work.
    const bool binned = g->binned && binnable_k(k);  // the mode settle_mode leaves
    Instance hi[1];
    fill_instance(hi[0], g, 0, n_reads, k);
    if (!binned) hi[0].parts = hi[0].d1 = hi[0].fan = 0;
    const PassKey key = pass_key(1, n_reads, reads_len, g->shape, binned, hi);
    dbgk::BinBuffers bb{};
    if (binned) bin_caps(key, bb);
    const PassSizes z(key, bb);
    Carve c;
    const uint64_t o_packed = c.take(z.packed), o_ws = c.take(z.ws), o_partials = c.take(z.partials),
                   o_args = c.take(z.args), o_status = c.take(z.status), o_tiles = c.take(z.tiles);
    uint64_t o_plan = 0, o_buckets = 0, o_totals = 0, o_hist1 = 0, o_scan1 = 0, o_hist2 = 0, o_scan2 = 0,
             o_bpart = 0, o_rec1 = 0, o_rec2 = 0, o_pstart = 0, o_tread1 = 0, o_tile2 = 0;
    if (binned) {
        o_plan = c.take(z.plan);
        o_buckets = c.take(z.buckets);
        o_totals = c.take(z.totals);
        o_hist1 = c.take(z.hist1);
        o_scan1 = c.take(z.scan1);
        o_hist2 = c.take(z.hist2);
        o_scan2 = c.take(z.scan2);
        o_bpart = c.take(z.bpartials);
        o_rec1 = c.take(z.rec1);
        o_rec2 = c.take(z.rec2);
        o_pstart = c.take(z.pstart);
        o_tread1 = c.take(z.tread1);
        o_tile2 = c.take(z.tile2);
    }
    if (c.used > kStaticScratchBytes) return DBG_E_SCRATCH;

    rc = settle_mode(g, k);  // k <= 32 here: at most a switch to the direct build, no allocation
    if (rc != DBG_OK) return rc;
    fill_instance(hi[0], g, 0, n_reads, k);
    if ((rc = hip_code(order_after_zero(g, s))) != DBG_OK) return rc;

    unsigned char *base = slot.ptr;
    unsigned char *dargs = base + o_args;
    auto *da = reinterpret_cast<dbgk::PassArgs *>(dargs);
    auto *di = reinterpret_cast<Instance *>(dargs + dbgk::kArgsBytes);
    auto *dst = reinterpret_cast<InstStatus *>(base + o_status);
    auto *cs = reinterpret_cast<CallState *>(dst + key.m_cap);
    auto *packed = reinterpret_cast<uint64_t *>(base + o_packed);
    auto *ws = reinterpret_cast<uint64_t *>(base + o_ws);
    if (binned) {
        bb.plan = reinterpret_cast<dbgk::BinPlan *>(base + o_plan);
        bb.buckets = reinterpret_cast<dbgk::Bucket *>(base + o_buckets);
        bb.totals = reinterpret_cast<dbgk::BinTotals *>(base + o_totals);
        bb.hist1 = reinterpret_cast<uint32_t *>(base + o_hist1);
        bb.scan1 = reinterpret_cast<uint64_t *>(base + o_scan1);
        bb.hist2 = reinterpret_cast<uint32_t *>(base + o_hist2);
        bb.scan2 = reinterpret_cast<uint64_t *>(base + o_scan2);
        bb.partials = reinterpret_cast<uint64_t *>(base + o_bpart);
        bb.rec1 = reinterpret_cast<uint64_t *>(base + o_rec1);
        bb.rec2 = reinterpret_cast<uint64_t *>(base + o_rec2);
        bb.pstart = reinterpret_cast<uint64_t *>(base + o_pstart);
        bb.tile_read1 = reinterpret_cast<uint64_t *>(base + o_tread1);
        bb.chunk2 = reinterpret_cast<dbgk::RefChunk *>(base + o_tile2);
        bb.chunks_per_group = g->bin_chunks;
        bb.scatter_div = g->bin_div;
        bb.shape_req1 = g->bin_shape1;
        bb.shape_req2 = g->bin_shape2;
        dbgk::binned_grids(g->device, bb);
    }
    dbgk::PassArgs a;
    PassOpts o = opts_of(g);
    o.stats = nullptr;  // the statistics kernels are not part of this entry point
    fill_args(a, key, z, 1, hi, d_reads, reads_len, d_offsets, n_reads, true, nullptr, nullptr, 0, o);

    hipLaunchKernelGGL(k_put_args, dim3(1), dim3(64), 0, s, a, hi[0], dargs);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = dbgk::launch_prepare(da, di, dst, cs, key.m_cap, s);
    if (e == hipSuccess) e = dbgk::launch_pack(da, packed, di, dst, key.len_cap, s);
    if (e == hipSuccess)
        e = dbgk::launch_scan(da, di, dst, ws, reinterpret_cast<uint64_t *>(base + o_partials),
                              binned ? nullptr : reinterpret_cast<uint64_t *>(base + o_tiles), cs, key.n_cap, s);
    if (e == hipSuccess) {
        if (binned)
            e = dbgk::launch_binned(da, di, packed, ws, dst, bb, key.n_cap, g->device, false, s, nullptr);
        else
            e = dbgk::launch_build(da, di, packed, ws, reinterpret_cast<uint64_t *>(base + o_tiles), dst, cs,
                                   key.shape, true, false, s);
    }
    InstStatus st{};
    if (e == hipSuccess) e = hipMemcpyAsync(&st, dst, sizeof st, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return DBG_E_DEVICE;
    return fold_status(g, st, k);
}
