// C ABI of libdbg (the declarations and their contracts are in dbg.h).
//
// The paper's constructor takes k, the thread count, the hash table size and
// the genome size (Methods, "Code organization"); here a handle takes the
// table size (capacity, or expected vertices and a load factor) and the launch
// shape; k is fixed by the first build.
#include "dbg_runtime.h"

using namespace dbgrt;
using dbgk::CallState;
using dbgk::Instance;
using dbgk::InstStatus;

extern "C" {

void dbg_config_init(dbg_config *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->device = -1;
}

int dbg_create(const dbg_config *cfg_in, dbg_graph **out) {
    if (!out) return DBG_E_INVAL;
    *out = nullptr;
    dbg_config cfg;
    dbg_config_init(&cfg);
    if (cfg_in) cfg = *cfg_in;
    const double lf = cfg.load_factor == 0 ? 0.5 : cfg.load_factor;
    if (!(lf > 0 && lf < 1)) return DBG_E_INVAL;
    if ((cfg.flags & DBG_F_BINNED) && lf > DBG_BINNED_MAX_LOAD) return DBG_E_INVAL;  // segment overflow odds
    const uint32_t block = cfg.block_size ? cfg.block_size : 256;
    if (block % 64 || block > 1024) return DBG_E_INVAL;
    const uint32_t wpt = cfg.windows_per_thread ? cfg.windows_per_thread : 4;
    if (wpt > 64) return DBG_E_INVAL;
    if (cfg.bin_chunks > dbgk::kMaxChunkTarget || cfg.bin_scatter_div > 64 || cfg.bin_shape1 > 4 ||
        cfg.bin_shape2 > 4)
        return DBG_E_INVAL;

    int device = cfg.device;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return DBG_E_DEVICE;
    DeviceGuard guard(device);
    if (!guard.ok) return DBG_E_DEVICE;

    dbg_graph *g = new dbg_graph();
    g->device = device;
    g->flags = cfg.flags;
    g->lf = lf;
    g->expected = cfg.expected_vertices;
    g->cap_req = cfg.capacity;
    g->ew = (cfg.flags & DBG_F_ENTRY32) ? 4 : 3;
    g->binned = (cfg.flags & DBG_F_BINNED) != 0;
    g->pass.use_graphs = (cfg.flags & DBG_F_GRAPH) != 0;
    g->shape.block = block;
    g->shape.wpt = wpt;
    g->shape.merge = (cfg.flags & DBG_F_MERGE) ? 1 : 0;
    g->shape.grid = dbgk::build_grid(device, block);
    g->bin_chunks = cfg.bin_chunks;
    g->bin_div = cfg.bin_scatter_div;
    g->bin_shape1 = cfg.bin_shape1;
    g->bin_shape2 = cfg.bin_shape2;
    g->grid_wide = dbgk::build_grid_wide(device, block);

    int rc = DBG_OK;
    if (cfg.stream) {
        g->stream = static_cast<hipStream_t>(cfg.stream);
    } else if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) == hipSuccess) {
        g->own_stream = true;
    } else {
        rc = DBG_E_DEVICE;
    }
    if (rc == DBG_OK && g->pass.init() != hipSuccess) rc = DBG_E_DEVICE;
    if (rc == DBG_OK && hipEventCreateWithFlags(&g->zero_ev, hipEventDisableTiming) != hipSuccess)
        rc = DBG_E_DEVICE;
    if (rc == DBG_OK && (g->flags & DBG_F_STATS)) {
        hipError_t e = g->pstats.reserve(8 * dbgk::kStatWords);
        if (e == hipSuccess) e = zero_stats(g);
        if (e != hipSuccess) rc = hip_code(e);
    }
    if (rc == DBG_OK && (g->cap_req || g->expected)) rc = ensure_table(g, 0);
    if (rc != DBG_OK) {
        dbg_destroy(g);
        return rc;
    }
    *out = g;
    return DBG_OK;
}

int dbg_build_device(dbg_graph *g, const uint8_t *d_reads, uint64_t reads_len,
                     const uint64_t *d_offsets, uint64_t n_reads, uint32_t k, void *stream) {
    int rc = check_common(g, k, kMaxK);
    if (rc != DBG_OK) return rc;
    if (n_reads == 0) return DBG_OK;
    if (!d_offsets || (!d_reads && reads_len)) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    if (g->pass.pending) {
        rc = harvest(g);
        if (rc != DBG_OK) return rc;
    }
    rc = ensure_table(g, reads_len);
    if (rc == DBG_OK) rc = settle_mode(g, k);
    if (rc != DBG_OK) return rc;
    return enqueue_single(g, d_reads, reads_len, d_offsets, n_reads, k, g->pick(stream));
}

int dbg_sync(dbg_graph *g) {
    if (!g) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    int rc = harvest(g);
    if (rc == DBG_OK && g->unreported != DBG_OK) rc = g->unreported;
    g->unreported = DBG_OK;
    return rc;
}

int dbg_build(dbg_graph *g, const char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k) {
    int rc = check_common(g, k, kMaxK);
    if (rc != DBG_OK) return rc;
    if (n_reads == 0) return DBG_OK;
    if (!offsets) return DBG_E_INVAL;
    uint64_t windows = 0, kmers = 0;
    if (!host_counts(offsets, n_reads, k, &windows, &kmers)) return DBG_E_INVAL;
    const uint64_t base = offsets[0];
    const uint64_t len = offsets[n_reads] - base;
    if (len && !reads) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    if (g->pass.pending) {
        rc = harvest(g);
        if (rc != DBG_OK) return rc;
    }
    if (g->inserts + kmers > kCounterLimit) return DBG_E_RANGE;
    rc = ensure_table(g, windows);
    if (rc == DBG_OK) rc = settle_mode(g, k);
    if (rc != DBG_OK) return rc;

    hipError_t e;
    if ((e = g->reads.reserve(std::max<uint64_t>(len, 1))) != hipSuccess ||
        (e = g->offsets.reserve((n_reads + 1) * 8)) != hipSuccess)
        return hip_code(e);
    hipStream_t s = g->stream;
    if (len && hipMemcpyAsync(g->reads.p, reads + base, len, hipMemcpyHostToDevice, s) != hipSuccess)
        return DBG_E_DEVICE;
    if (hipMemcpyAsync(g->offsets.p, offsets, (n_reads + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return DBG_E_DEVICE;
    rc = enqueue_single(g, g->reads.as<uint8_t>(), len, g->offsets.as<uint64_t>(), n_reads, k, s);
    if (rc != DBG_OK) return rc;
    return harvest(g);
}

static int extract_impl(dbg_graph *g, uint64_t *keys, uint32_t *counts, uint64_t cap,
                        uint64_t *n_vertices, bool device_out, hipStream_t s) {
    if (!g || !n_vertices) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    if (g->pass.pending) {
        const int rc = harvest(g);
        if (rc != DBG_OK) g->unreported = rc;
    }
    const uint64_t V = g->vertices;
    *n_vertices = V;
    if (!keys) return DBG_OK;
    if (cap < V) return DBG_E_SPACE;
    if (!counts) return DBG_E_INVAL;
    if (V == 0) return DBG_OK;
    const uint64_t kw = key_words(g);

    uint64_t *okeys = keys;
    uint32_t *ocnt = counts;
    hipError_t e;
    if (!device_out) {
        if ((e = g->xkeys.reserve(V * 8 * kw)) != hipSuccess || (e = g->xcnt.reserve(V * 16)) != hipSuccess)
            return hip_code(e);
        okeys = g->xkeys.as<uint64_t>();
        ocnt = g->xcnt.as<uint32_t>();
    }
    if (g->xn.reserve(8) != hipSuccess) return DBG_E_DEVICE;
    uint64_t found = 0;
    e = dbgk::launch_fill_zero(g->xn.as<uint64_t>(), 1, s);
    if (e == hipSuccess && kw == 2 && !g->binned)
        e = dbgk::launch_extract_wide(g->table.as<uint64_t>(), g->cap, okeys, ocnt, V, g->xn.as<uint64_t>(), s);
    else if (e == hipSuccess && g->binned)
        e = dbgk::launch_extract_binned(g->table.as<uint64_t>(), g->ew, (uint32_t)kw, g->parts,
                                        g->seg_count.as<uint32_t>(), g->seg_off.as<uint64_t>(),
                                        g->seg_partials.as<uint64_t>(), g->seg_len.as<uint64_t>(), okeys,
                                        ocnt, V, g->xn.as<uint64_t>(), g->device, s);
    else if (e == hipSuccess)
        e = dbgk::launch_extract(g->table.as<uint64_t>(), g->ew, g->cap, okeys, ocnt, V,
                                 g->xn.as<uint64_t>(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&found, g->xn.p, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !device_out) {
        e = hipMemcpyAsync(keys, okeys, V * 8 * kw, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(counts, ocnt, V * 16, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return DBG_E_DEVICE;
    return found == V ? DBG_OK : DBG_E_DEVICE;
}

int dbg_build_extract_device(dbg_graph *g, const uint8_t *d_reads, uint64_t reads_len,
                             const uint64_t *d_offsets, uint64_t n_reads, uint32_t k, uint64_t *d_keys,
                             uint32_t *d_counts, uint64_t cap, uint64_t *n_vertices, void *stream) {
    int rc = check_common(g, k, kMaxK);
    if (rc != DBG_OK) return rc;
    if (!n_vertices || (n_reads && !d_offsets) || (!d_reads && reads_len) || (d_keys && cap && !d_counts))
        return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    if (g->pass.pending) {
        rc = harvest(g);
        if (rc != DBG_OK) return rc;
    }
    hipStream_t s = g->pick(stream);
    if (n_reads) {
        rc = ensure_table(g, reads_len);
        if (rc == DBG_OK) rc = settle_mode(g, k);
        if (rc != DBG_OK) return rc;
        // fused: a binned build (the mode settle_mode chose for k)
        const bool fuse = d_keys && g->binned;
        rc = enqueue_single(g, d_reads, reads_len, d_offsets, n_reads, k, s, fuse ? d_keys : nullptr,
                            fuse ? d_counts : nullptr, fuse ? cap : 0);
        if (rc != DBG_OK) return rc;
        rc = harvest(g);
        if (rc != DBG_OK) return rc;
        if (fuse) {
            const uint64_t V = g->vertices;
            *n_vertices = V;
            if (g->pass.host_status()[0].emitted != V) return DBG_E_DEVICE;
            return cap < V ? DBG_E_SPACE : DBG_OK;
        }
    }
    return extract_impl(g, d_keys, d_counts, cap, n_vertices, true, s);
}

int dbg_extract(dbg_graph *g, uint64_t *keys, uint32_t *counts, uint64_t cap, uint64_t *n_vertices) {
    return extract_impl(g, keys, counts, cap, n_vertices, false, g ? g->stream : nullptr);
}

int dbg_extract_device(dbg_graph *g, uint64_t *d_keys, uint32_t *d_counts, uint64_t cap,
                       uint64_t *n_vertices, void *stream) {
    return extract_impl(g, d_keys, d_counts, cap, n_vertices, true, g ? g->pick(stream) : nullptr);
}

int dbg_extract_normalized(dbg_graph *g, uint64_t genome_size, uint32_t flags, uint64_t *keys, void *counts,
                           uint64_t cap, uint64_t *n_vertices) {
    if (!g || !n_vertices || (flags & ~DBG_NORM_U8)) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (!guard.ok) return DBG_E_DEVICE;
    if (g->pass.pending) {
        const int rc = harvest(g);
        if (rc != DBG_OK) g->unreported = rc;
    }
    const uint64_t V = g->vertices;
    *n_vertices = V;
    if (!keys) return DBG_OK;
    if (cap < V) return DBG_E_SPACE;
    if (!counts) return DBG_E_INVAL;
    if (V == 0) return DBG_OK;
    const uint64_t kw = key_words(g);
    hipError_t e;
    if ((e = g->nkeys.reserve(V * 8 * kw)) != hipSuccess || (e = g->ncnt.reserve(V * 16)) != hipSuccess ||
        (e = g->n8.reserve(V * 4)) != hipSuccess)
        return hip_code(e);
    uint64_t n = 0;
    int rc = extract_impl(g, g->nkeys.as<uint64_t>(), g->ncnt.as<uint32_t>(), V, &n, true, g->stream);
    if (rc != DBG_OK) return rc;
    hipStream_t s = g->stream;
    const bool u8 = (flags & DBG_NORM_U8) != 0;
    e = dbgk::launch_normalize(g->ncnt.as<uint32_t>(), 4 * V, genome_size, g->inserts,
                               u8 ? g->n8.as<uint8_t>() : nullptr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(keys, g->nkeys.p, V * 8 * kw, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, u8 ? g->n8.p : g->ncnt.p, u8 ? V * 4 : V * 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? DBG_OK : DBG_E_DEVICE;
}

int dbg_reset(dbg_graph *g) {
    if (!g) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (g->pass.pending) (void)harvest(g);
    g->k = 0;
    g->poisoned = DBG_OK;
    g->unreported = DBG_OK;
    g->vertices = g->inserts = g->windows = g->builds = 0;
    ++g->epoch;
    g->fresh = true;
    if ((g->flags & DBG_F_STATS) && zero_stats(g) != hipSuccess) return DBG_E_DEVICE;
    // A binned build rewrites every slot of a fresh table, so its reset only
    // marks the table empty; the direct build needs the zeros.
    if (!g->cap || g->binned) return DBG_OK;
    return zero_table(g) == hipSuccess ? DBG_OK : DBG_E_DEVICE;
}

int dbg_get_stats(dbg_graph *g, dbg_stats *out) {
    if (!g || !out) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (g->pass.pending) {
        const int rc = harvest(g);
        if (rc != DBG_OK) g->unreported = rc;
    }
    std::memset(out, 0, sizeof *out);
    out->capacity = g->cap;
    out->table_bytes = g->table_words() * 8;
    out->vertices = g->vertices;
    out->inserts = g->inserts;
    out->windows = g->windows;
    out->builds = g->builds;
    out->k = g->k;
    out->status = g->poisoned;
    out->last_build_ms = g->last_build_ms;
    out->last_total_ms = g->last_total_ms;
    out->block_size = g->shape.block;
    out->windows_per_thread = g->shape.wpt;
    out->grid_size = g->shape.grid;
    out->entry_bytes = g->ew * 8;
    out->graph_captures = g->pass.captures;
    out->graph_replays = g->pass.replays;
    out->binned = g->binned ? 1u : 0u;
    out->bin_chunks = g->bin_chunks;
    out->bin_scatter_div = g->bin_div;
    out->bin_shape1 = g->pass.shapes & 0xffu;
    out->bin_shape2 = g->pass.shapes >> 8;
    return DBG_OK;
}

void dbg_destroy(dbg_graph *g) {
    if (!g) return;
    DeviceGuard guard(g->device);
    if (g->pass.pending) (void)g->pass.wait(nullptr, nullptr);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    DevBuf *bufs[] = {&g->table, &g->reads,     &g->offsets, &g->xkeys,        &g->xcnt,    &g->xn,
                      &g->nkeys, &g->ncnt,      &g->n8,      &g->seg_count,    &g->seg_off, &g->seg_partials,
                      &g->seg_len, &g->pstats};
    for (DevBuf *b : bufs) b->release();
    g->pass.release();
    dbg_contigs_free(g->contigs);
    if (g->zero_ev) (void)hipEventDestroy(g->zero_ev);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

int dbg_get_probe_stats(dbg_graph *g, dbg_probe_stats *out) {
    if (!g || !out) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (g->pass.pending) {
        const int rc = harvest(g);
        if (rc != DBG_OK) g->unreported = rc;
    }
    std::memset(out, 0, sizeof *out);
    if (!(g->flags & DBG_F_STATS)) return DBG_OK;
    uint64_t w[dbgk::kStatWords] = {};
    hipError_t e = hipMemcpyAsync(w, g->pstats.p, sizeof w, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return DBG_E_DEVICE;
    out->lookups = w[dbgk::kStatLookups];
    out->probes = w[dbgk::kStatProbes];
    out->cas_attempts = w[dbgk::kStatCas];
    out->cas_lost = w[dbgk::kStatCasLost];
    for (int i = 0; i < 8; ++i) out->probe_hist[i] = w[dbgk::kStatHist + i];
    return DBG_OK;
}

int dbg_get_phase_times(dbg_graph *g, double *ms, uint32_t cap, uint32_t *n_phases) {
    if (!g || !n_phases || (cap && !ms)) return DBG_E_INVAL;
    DeviceGuard guard(g->device);
    if (g->pass.pending) {
        const int rc = harvest(g);
        if (rc != DBG_OK) g->unreported = rc;
    }
    *n_phases = g->pass.n_phases;
    for (uint32_t i = 0; i < g->pass.n_phases && i < cap; ++i) ms[i] = g->pass.phase_ms[i];
    return DBG_OK;
}

const char *dbg_strerror(int code) {
    switch (code) {
    case DBG_OK: return "ok";
    case DBG_E_INVAL: return "invalid argument (NULL pointer, bad offsets or configuration)";
    case DBG_E_K: return "k outside [2, 64] (outside [2, 32] for batches, the server and contigs) or different from the graph's k";
    case DBG_E_BASE: return "read byte outside ACGTacgt";
    case DBG_E_NOMEM: return "device memory allocation refused";
    case DBG_E_FULL: return "table capacity exhausted; graph poisoned";
    case DBG_E_SPACE: return "output buffer smaller than the vertex count";
    case DBG_E_DEVICE: return "HIP runtime error";
    case DBG_E_RANGE: return "cumulative k-mers would exceed 2^32-1";
    case DBG_E_STATE: return "graph poisoned by an earlier capacity overflow";
    case DBG_E_SCRATCH: return "input needs more than the static scratch buffer of dbg_build_device_static";
    default: return "unknown error";
    }
}

int dbg_build_batch(dbg_graph *const *graphs, const dbg_input *inputs, uint32_t m,
                    int32_t *statuses, void *stream) {
    if (m == 0) return DBG_OK;
    if (!graphs || !inputs || !statuses) return DBG_E_INVAL;
    for (uint32_t i = 0; i < m; ++i)
        if (!graphs[i]) return DBG_E_INVAL;
    const int device = graphs[0]->device;
    DeviceGuard guard(device);
    if (!guard.ok) return DBG_E_DEVICE;
    BatchCtx *ctx = batch_ctx(device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->ready) {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
            ctx->pass.init() != hipSuccess)
            return DBG_E_DEVICE;
        ctx->ready = true;
    }
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;

    // Host-side validation and the concatenated layout.  Instances that fail
    // here keep zero reads in the launch, so nothing of theirs is touched.
    std::vector<uint64_t> read_begin(m + 1, 0);
    std::vector<uint32_t> ks(m);
    std::vector<int32_t> pre(m, DBG_OK);
    uint64_t total_bytes = 0, total_reads = 0;
    std::vector<uint64_t> bound(m, 0);  // each instance's windows: the size of an unsized graph
    for (uint32_t i = 0; i < m; ++i) {
        const dbg_input &in = inputs[i];
        ks[i] = in.k;
        read_begin[i] = total_reads;
        int rc = check_common(graphs[i], in.k);
        uint64_t w = 0, km = 0;
        if (rc == DBG_OK && in.n_reads && !in.offsets) rc = DBG_E_INVAL;
        if (rc == DBG_OK && in.n_reads && !host_counts(in.offsets, in.n_reads, in.k, &w, &km))
            rc = DBG_E_INVAL;
        if (rc == DBG_OK && in.n_reads && in.offsets[in.n_reads] > in.offsets[0] && !in.reads)
            rc = DBG_E_INVAL;
        if (rc == DBG_OK && graphs[i]->inserts + km > kCounterLimit) rc = DBG_E_RANGE;
        pre[i] = rc;
        bound[i] = w;
        if (rc == DBG_OK && in.n_reads) {
            total_reads += in.n_reads;
            total_bytes += in.offsets[in.n_reads] - in.offsets[0];
        }
    }
    read_begin[m] = total_reads;
    std::vector<uint64_t> &hoff = ctx->hoff;
    hoff.assign(total_reads + 1, 0);
    hipError_t e;
    if ((e = ctx->reads.reserve(std::max<uint64_t>(total_bytes, 1))) != hipSuccess ||
        (e = ctx->offsets.reserve((total_reads + 1) * 8)) != hipSuccess) {
        for (uint32_t i = 0; i < m; ++i) statuses[i] = hip_code(e);
        return hip_code(e);
    }
    uint64_t byte_at = 0;
    for (uint32_t i = 0; i < m; ++i) {
        const dbg_input &in = inputs[i];
        if (pre[i] != DBG_OK || !in.n_reads) continue;
        const uint64_t b0 = in.offsets[0], len = in.offsets[in.n_reads] - b0;
        for (uint64_t r = 0; r < in.n_reads; ++r) hoff[read_begin[i] + r] = byte_at + (in.offsets[r] - b0);
        if (len && hipMemcpyAsync(ctx->reads.as<uint8_t>() + byte_at, in.reads + b0, len,
                                  hipMemcpyHostToDevice, s) != hipSuccess)
            return DBG_E_DEVICE;
        byte_at += len;
    }
    hoff[total_reads] = byte_at;
    if (hipMemcpyAsync(ctx->offsets.p, hoff.data(), (total_reads + 1) * 8, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DBG_E_DEVICE;

    // graphs that failed host validation take part with no reads
    std::vector<dbg_graph *> gs(graphs, graphs + m);
    std::vector<uint32_t> kk(ks);
    std::vector<uint64_t> rb(read_begin);
    std::vector<dbg_graph *> run_g;
    std::vector<uint32_t> run_k;
    std::vector<uint64_t> run_rb, run_bound;
    std::vector<uint32_t> where;
    for (uint32_t i = 0; i < m; ++i) {
        if (pre[i] != DBG_OK) continue;
        run_g.push_back(gs[i]);
        run_k.push_back(kk[i]);
        run_rb.push_back(rb[i]);
        run_bound.push_back(bound[i]);
        where.push_back(i);
    }
    for (uint32_t i = 0; i < m; ++i) statuses[i] = pre[i];
    if (run_g.empty()) return first_error(statuses, m);
    run_rb.push_back(total_reads);
    std::vector<int32_t> st(run_g.size(), DBG_OK);
    if (total_reads == 0) return first_error(statuses, m);
    batch_device_impl(run_g.data(), (uint32_t)run_g.size(), run_rb.data(), run_k.data(),
                      ctx->reads.as<uint8_t>(), byte_at, ctx->offsets.as<uint64_t>(), run_bound.data(), st.data(),
                      s, ctx, true);
    for (size_t j = 0; j < where.size(); ++j) statuses[where[j]] = st[j];
    return first_error(statuses, m);
}

int dbg_build_batch_device(dbg_graph *const *graphs, uint32_t m, const uint64_t *read_begin,
                           const uint32_t *ks, const uint8_t *d_reads, uint64_t reads_len,
                           const uint64_t *d_offsets, int32_t *statuses, void *stream) {
    if (m == 0) return DBG_OK;
    if (!graphs || !read_begin || !ks || !statuses || !d_offsets || (!d_reads && reads_len))
        return DBG_E_INVAL;
    for (uint32_t i = 0; i < m; ++i)
        if (!graphs[i]) return DBG_E_INVAL;
    if (read_begin[0] != 0) return DBG_E_INVAL;
    const int device = graphs[0]->device;
    DeviceGuard guard(device);
    if (!guard.ok) return DBG_E_DEVICE;
    BatchCtx *ctx = batch_ctx(device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->ready) {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
            ctx->pass.init() != hipSuccess)
            return DBG_E_DEVICE;
        ctx->ready = true;
    }
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
    if (read_begin[m] == 0) {
        for (uint32_t i = 0; i < m; ++i) statuses[i] = check_common(graphs[i], ks[i]);
        return first_error(statuses, m);
    }
    batch_device_impl(graphs, m, read_begin, ks, d_reads, reads_len, d_offsets, nullptr, statuses, s, ctx, true);
    return first_error(statuses, m);
}

int dbg_atomic_roofline(int32_t device, uint32_t kind, uint64_t footprint_bytes, uint64_t n_ops,
                        uint32_t block_size, uint32_t repeats, double *ms) {
    if (!ms || kind > 4 || footprint_bytes < 64 || block_size == 0 || block_size % 64 ||
        block_size > 1024)
        return DBG_E_INVAL;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return DBG_E_DEVICE;
    DeviceGuard guard(device);
    if (!guard.ok) return DBG_E_DEVICE;
    const uint64_t words = footprint_bytes / 8;
    uint64_t *mem = nullptr, *sink = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    std::vector<double> t;
    hipError_t e = hipMalloc(&mem, words * 8);
    if (e == hipSuccess) e = hipMalloc(&sink, 8);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    for (uint32_t r = 0; e == hipSuccess && r <= repeats; ++r) {
        e = dbgk::launch_fill_zero(mem, words, s);
        if (e == hipSuccess) e = hipEventRecord(a, s);
        if (e == hipSuccess) e = dbgk::launch_roofline(mem, words, n_ops, kind, 0x9E3779B97F4A7C15ull * (r + 1),
                                                       block_size, sink, s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float x = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&x, a, b);
        if (e == hipSuccess && r > 0) t.push_back(x);  // launch 0 warms up
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s) (void)hipStreamDestroy(s);
    if (mem) (void)hipFree(mem);
    if (sink) (void)hipFree(sink);
    if (e != hipSuccess) return hip_code(e);
    if (t.empty()) {
        *ms = 0;
        return DBG_OK;
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return DBG_OK;
}

}  // extern "C"
