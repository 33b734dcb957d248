// Build server: read-set requests are admitted first come, first served while
// the table bytes of admitted, unreleased requests fit an HBM budget; admitted
// requests are built by continuous batching (each batched pass takes the
// requests admitted since the previous one, several passes in flight on their
// own streams); tables stay resident until the client releases them.  A table
// that turns out too small (the estimate of distinct vertices was low) is
// rebuilt from scratch at twice the capacity, so a request's result never
// depends on the estimate.
//
// Threads: clients call the dbg_server_* functions from any thread; one
// worker thread per server owns the device work (table allocation, staging,
// the passes) and the pool of idle tables.
#include "dbg_runtime.h"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <thread>
#include <unordered_map>

using namespace dbgrt;

namespace {

// ---------------------------------------------------------------- device

// Offsets of one device-resident request inside a pass's concatenation.
struct RebaseDesc {
    const uint64_t *src;  // the client's offsets (n + 1 entries)
    uint64_t n;           // reads
    uint64_t cum;         // offsets of earlier device requests in this launch
    uint64_t dst_read;    // first read of the request in the concatenation
    uint64_t dst_byte;    // first byte of the request in the concatenation
    uint64_t len;         // the request's byte count
    uint32_t req;         // index in the pass
    uint32_t pad;
};

// Read r of a request starts at dst_byte + (src[r] - src[0]) in the
// concatenation.  Offsets outside [src[0], src[0] + len], or a last offset
// other than src[0] + len, flag the request: its offsets are clamped into its
// own byte range so that no other request's reads change, and its result is
// discarded.  Decreasing offsets stay decreasing and are flagged by the pass.
__global__ __launch_bounds__(256) void k_rebase(const RebaseDesc *__restrict__ d, uint32_t nd,
                                                uint64_t total, uint64_t *__restrict__ dst,
                                                uint32_t *__restrict__ bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += stride) {
        uint32_t lo = 0, hi = nd;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (d[mid].cum <= j) lo = mid;
            else hi = mid;
        }
        const RebaseDesc &x = d[lo];
        const uint64_t r = j - x.cum;
        const uint64_t s0 = x.src[0], v = x.src[r];
        bool b = v < s0 || v - s0 > x.len;
        if (r == 0) {
            const uint64_t e = x.src[x.n];
            if (e < s0 || e - s0 != x.len) b = true;
        }
        const uint64_t rel = v < s0 ? 0 : (v - s0 > x.len ? x.len : v - s0);
        dst[x.dst_read + r] = x.dst_byte + rel;
        if (b) atomicOr(&bad[x.req], 1u);
    }
}

hipError_t launch_rebase(const RebaseDesc *d, uint32_t nd, uint64_t total, uint64_t *dst, uint32_t *bad,
                         hipStream_t s) {
    if (!nd || !total) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rebase, dim3((uint32_t)blocks), dim3(256), 0, s, d, nd, total, dst, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------- host

using Clock = std::chrono::steady_clock;

enum State { kQueued, kReady, kRunning, kDone };

struct Request {
    uint64_t id = 0;
    uint32_t k = 0;
    uint64_t n_reads = 0, reads_len = 0;
    uint64_t slots = 0;  // table capacity class
    uint64_t bytes = 0;  // budget charge
    bool binned = false;
    bool device_input = false;
    const uint8_t *d_reads = nullptr;
    const uint64_t *d_off = nullptr;
    std::vector<uint8_t> h_reads;
    std::vector<uint64_t> h_off;  // relative: h_off[0] == 0
    dbg_graph *g = nullptr;
    State state = kQueued;
    int32_t status = DBG_OK;
    uint32_t retries = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Idle {
    uint64_t slots;
    bool binned;
    uint64_t bytes;
    dbg_graph *g;
};

// One pass in flight: its stream, pass scratch and input staging.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Pass pass;
    DevBuf reads, offsets, descs, bad;
    HostBuf h_reads, h_off, h_descs, h_bad;
    std::vector<Request *> reqs;
    std::vector<dbg_graph *> graphs;
    std::vector<uint64_t> read_begin;
    std::vector<uint32_t> ks;
    std::vector<int32_t> statuses;
    BatchRun br;
    bool busy = false;

    hipError_t init() {
        hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e == hipSuccess) e = pass.init();
        return e;
    }
    void release() {
        if (stream) (void)hipStreamSynchronize(stream);
        pass.release();
        DevBuf *d[] = {&reads, &offsets, &descs, &bad};
        for (DevBuf *b : d) b->release();
        HostBuf *h[] = {&h_reads, &h_off, &h_descs, &h_bad};
        for (HostBuf *b : h) b->release();
        if (done) (void)hipEventDestroy(done);
        if (stream) (void)hipStreamDestroy(stream);
        done = nullptr;
        stream = nullptr;
    }
};

}  // namespace

struct dbg_server {
    dbg_server_config cfg{};
    int device = 0;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_id = 1;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request *> queue;       // waiting for admission, FIFO
    std::vector<dbg_graph *> returned;  // released tables, to be pooled by the worker
    uint64_t resident = 0;              // table bytes of admitted, unreleased requests
    dbg_server_stats st{};

    // worker-only state
    std::thread worker;
    std::deque<Request *> ready;  // admitted, table attached, waiting for a pass
    std::list<Idle> idle;         // pooled tables, oldest first
    uint64_t idle_bytes = 0;
    std::vector<std::unique_ptr<Slot>> slots;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    void admit(std::vector<Request *> &out);
    int attach_table(Request *r);
    void pool_table(dbg_graph *g);
    bool launch(Slot &s);
    void finish(Slot &s);
};

namespace {

// Table capacity class and budget charge of a request of `vertices`
// estimated vertices.
void size_request(const dbg_server_config &cfg, uint64_t vertices, Request &r) {
    r.slots = size_class(capacity_for(vertices, cfg.load_factor), 4096);
    const uint64_t ew = (cfg.flags & DBG_F_ENTRY32) ? 4 : 3;
    uint64_t cap = r.slots, extra = 0;
    uint32_t d1 = 0, fan = 0;
    uint64_t parts = 0;
    if (r.binned && binned_geometry(cap, &d1, &fan, &parts)) {
        cap = parts * dbgk::kSegSlots;
        extra = 4 * parts + 8 * (parts + 1) + 8 * ((parts + 1023) / 1024 + 2) + 8;
    }
    r.bytes = cap * ew * 8 + extra;
}

}  // namespace

// Move queue-head requests whose tables fit the budget to the caller (under mu).
void dbg_server::admit(std::vector<Request *> &out) {
    while (!queue.empty()) {
        Request *r = queue.front();
        if (resident + r->bytes > cfg.hbm_budget) break;
        queue.pop_front();
        resident += r->bytes;
        r->state = kReady;
        ++st.admitted;
        out.push_back(r);
    }
}

// Return a table to the idle pool (worker thread).
void dbg_server::pool_table(dbg_graph *g) {
    if (!g) return;
    dbg_reset(g);  // binned: marks the table empty; direct: zero fill, ordered by event
    dbg_stats s{};
    dbg_get_stats(g, &s);
    Idle x{g->cap_req, g->binned, s.table_bytes, g};
    idle.push_back(x);
    idle_bytes += x.bytes;
}

// Give an admitted request a table of its class: a pooled one, else a new
// one, evicting pooled tables while the budget would be exceeded (worker).
int dbg_server::attach_table(Request *r) {
    for (auto it = idle.begin(); it != idle.end(); ++it)
        if (it->slots == r->slots && it->binned == r->binned) {
            r->g = it->g;
            idle_bytes -= it->bytes;
            idle.erase(it);
            return DBG_OK;
        }
    uint64_t res;
    {
        std::lock_guard<std::mutex> lk(mu);
        res = resident;
    }
    while (!idle.empty() && res + idle_bytes > cfg.hbm_budget) {
        idle_bytes -= idle.front().bytes;
        dbg_destroy(idle.front().g);
        idle.pop_front();
    }
    dbg_config c;
    dbg_config_init(&c);
    c.capacity = r->slots;
    c.load_factor = cfg.load_factor;
    c.device = device;
    c.flags = r->binned ? cfg.flags : (cfg.flags & ~(uint32_t)DBG_F_BINNED);
    int rc = dbg_create(&c, &r->g);
    if (rc == DBG_E_NOMEM && !idle.empty()) {
        while (!idle.empty()) {
            dbg_destroy(idle.front().g);
            idle.pop_front();
        }
        idle_bytes = 0;
        rc = dbg_create(&c, &r->g);
    }
    return rc;
}

// Form a pass from the ready requests (FIFO, one table mode per pass, within
// the batch limits) and enqueue it on the slot's stream (worker).
bool dbg_server::launch(Slot &s) {
    if (ready.empty()) return false;
    const bool binned = ready.front()->binned;
    s.reqs.clear();
    uint64_t bytes = 0, n = 0;
    for (auto it = ready.begin(); it != ready.end() && s.reqs.size() < cfg.max_batch;) {
        Request *r = *it;
        if (r->binned != binned) {
            ++it;
            continue;
        }
        if (!s.reqs.empty() && bytes + r->reads_len > cfg.max_batch_bytes) break;
        bytes += r->reads_len;
        n += r->n_reads;
        s.reqs.push_back(r);
        it = ready.erase(it);
    }
    const uint32_t m = (uint32_t)s.reqs.size();
    s.graphs.assign(m, nullptr);
    s.ks.assign(m, 0);
    s.read_begin.assign(m + 1, 0);
    s.statuses.assign(m, DBG_OK);
    uint64_t host_bytes = 0;
    uint32_t n_dev = 0;
    for (uint32_t i = 0; i < m; ++i) {
        Request *r = s.reqs[i];
        s.graphs[i] = r->g;
        s.ks[i] = r->k;
        s.read_begin[i + 1] = s.read_begin[i] + r->n_reads;
        if (!r->device_input) host_bytes += r->reads_len;
        else if (r->n_reads) ++n_dev;
    }
    const double t = now();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Request *r : s.reqs) {
            r->state = kRunning;
            r->t_start = t;
        }
        ++st.passes;
    }

    hipError_t e;
    const uint64_t bad_words = (m + 1) / 2;
    if ((e = s.reads.reserve(std::max<uint64_t>(bytes, 1))) != hipSuccess ||
        (e = s.offsets.reserve((n + 1) * 8)) != hipSuccess ||
        (e = s.descs.reserve(sizeof(RebaseDesc) * std::max<uint32_t>(n_dev, 1))) != hipSuccess ||
        (e = s.bad.reserve(8 * bad_words)) != hipSuccess ||
        (e = s.h_reads.reserve(std::max<uint64_t>(host_bytes, 1))) != hipSuccess ||
        (e = s.h_off.reserve((n + 1) * 8)) != hipSuccess ||
        (e = s.h_descs.reserve(sizeof(RebaseDesc) * std::max<uint32_t>(n_dev, 1))) != hipSuccess ||
        (e = s.h_bad.reserve(8 * bad_words)) != hipSuccess) {
        for (uint32_t i = 0; i < m; ++i) s.statuses[i] = hip_code(e);
        s.br = BatchRun();
        s.busy = true;
        return true;
    }
    // stage: host requests through pinned memory, device requests by
    // device-to-device copies; offsets rebased on the host or by k_rebase
    uint64_t *hoff = s.h_off.as<uint64_t>();
    RebaseDesc *hd = s.h_descs.as<RebaseDesc>();
    uint8_t *hr = s.h_reads.as<uint8_t>();
    uint8_t *dr = s.reads.as<uint8_t>();
    uint64_t byte_at = 0, host_at = 0, cum = 0;
    uint32_t di = 0;
    e = dbgk::launch_fill_zero(s.bad.as<uint64_t>(), bad_words, s.stream);
    for (uint32_t i = 0; i < m && e == hipSuccess; ++i) {
        Request *r = s.reqs[i];
        const uint64_t rb = s.read_begin[i];
        if (r->device_input && r->n_reads) {
            hd[di] = RebaseDesc{r->d_off, r->n_reads, cum, rb, byte_at, r->reads_len, i, 0};
            cum += r->n_reads;
            ++di;
            if (r->reads_len)
                e = hipMemcpyAsync(dr + byte_at, r->d_reads, r->reads_len, hipMemcpyDeviceToDevice, s.stream);
        } else {
            for (uint64_t j = 0; j < r->n_reads; ++j) hoff[rb + j] = byte_at + r->h_off[j];
            if (r->reads_len) {
                std::memcpy(hr + host_at, r->h_reads.data(), r->reads_len);
                e = hipMemcpyAsync(dr + byte_at, hr + host_at, r->reads_len, hipMemcpyHostToDevice, s.stream);
            }
            host_at += r->reads_len;
        }
        byte_at += r->reads_len;
    }
    hoff[n] = byte_at;
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.offsets.p, hoff, (n + 1) * 8, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess && n_dev)
        e = hipMemcpyAsync(s.descs.p, hd, sizeof(RebaseDesc) * n_dev, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess)
        e = launch_rebase(s.descs.as<RebaseDesc>(), n_dev, cum, s.offsets.as<uint64_t>(), s.bad.as<uint32_t>(),
                          s.stream);
    if (e != hipSuccess) {
        for (uint32_t i = 0; i < m; ++i) s.statuses[i] = hip_code(e);
        s.br = BatchRun();
        s.busy = true;
        return true;
    }
    if (n) {
        std::vector<uint64_t> bounds(m);  // request graphs are sized at admission; this only bounds windows
        for (uint32_t i = 0; i < m; ++i) bounds[i] = s.reqs[i]->reads_len;
        batch_enqueue(s.graphs.data(), m, s.read_begin.data(), s.ks.data(), dr, byte_at, s.offsets.as<uint64_t>(),
                      bounds.data(), s.statuses.data(), s.stream, s.pass, true, s.br);
    } else {
        s.br = BatchRun();
    }
    e = hipMemcpyAsync(s.h_bad.p, s.bad.p, 8 * bad_words, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) (void)hipStreamSynchronize(s.stream);
    s.busy = true;
    return true;
}

// Fold a finished pass: final statuses, rebuilds of overflowed tables (worker).
void dbg_server::finish(Slot &s) {
    const uint32_t m = (uint32_t)s.reqs.size();
    if (!s.br.graphs.empty()) batch_finish(s.br, s.pass, s.statuses.data());
    (void)hipStreamSynchronize(s.stream);
    const uint32_t *bad = s.h_bad.as<uint32_t>();
    const double t = now();
    std::vector<dbg_graph *> to_pool;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint32_t i = 0; i < m; ++i) {
            Request *r = s.reqs[i];
            int32_t rc = s.statuses[i];
            if (rc == DBG_OK && bad && bad[i]) rc = DBG_E_INVAL;
            if (rc == DBG_E_FULL && r->retries < 8) {
                // too small a table: rebuild from scratch at twice the capacity
                to_pool.push_back(r->g);
                r->g = nullptr;
                resident -= r->bytes;
                ++r->retries;
                const uint64_t old = r->bytes;
                Request tmp;
                tmp.binned = r->binned;
                size_request(cfg, (uint64_t)(r->slots * cfg.load_factor) * 2 + 1, tmp);
                r->slots = tmp.slots;
                r->bytes = tmp.bytes;
                --st.admitted;
                if (r->bytes > cfg.hbm_budget || r->bytes <= old) {
                    rc = DBG_E_NOMEM;
                } else {
                    r->state = kQueued;
                    queue.push_front(r);
                    continue;
                }
            }
            r->status = rc;
            r->state = kDone;
            r->t_done = t;
            ++st.completed;
            if (rc != DBG_OK && r->g) {
                // a failed build keeps no table
                to_pool.push_back(r->g);
                r->g = nullptr;
                resident -= r->bytes;
            }
            r->h_reads = std::vector<uint8_t>();
            r->h_off = std::vector<uint64_t>();
        }
    }
    for (dbg_graph *g : to_pool) pool_table(g);
    s.busy = false;
    s.reqs.clear();
    cv_done.notify_all();
}

void dbg_server::run() {
    (void)hipSetDevice(device);
    std::vector<Request *> admitted;
    std::vector<dbg_graph *> back;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        admitted.clear();
        if (!stop) admit(admitted);
        back.swap(returned);
        returned.clear();
        lk.unlock();

        for (dbg_graph *g : back) pool_table(g);
        if (!back.empty()) progress = true;
        back.clear();
        for (Request *r : admitted) {
            const int rc = attach_table(r);
            if (rc == DBG_OK) {
                ready.push_back(r);
                continue;
            }
            std::lock_guard<std::mutex> g2(mu);
            r->status = rc;
            r->state = kDone;
            r->t_done = now();
            resident -= r->bytes;
            ++st.completed;
            cv_done.notify_all();
        }
        if (!admitted.empty()) progress = true;

        uint32_t in_flight = 0;
        for (auto &s : slots) {
            if (s->busy && hipEventQuery(s->done) != hipErrorNotReady) {
                finish(*s);
                progress = true;
            }
        }
        for (auto &s : slots) {
            if (!s->busy && launch(*s)) progress = true;
            if (s->busy) ++in_flight;
        }

        lk.lock();
        st.max_in_flight = std::max<uint64_t>(st.max_in_flight, in_flight);
        if (stop && ready.empty() && !in_flight) break;
        if (progress) continue;
        if (in_flight) {
            cv_work.wait_for(lk, std::chrono::microseconds(50));
        } else {
            cv_work.wait(lk, [&] {
                return stop || !returned.empty() ||
                       (!queue.empty() && resident + queue.front()->bytes <= cfg.hbm_budget);
            });
        }
    }
    // dropped: whatever is still waiting for admission
    for (Request *r : queue) {
        r->status = DBG_E_STATE;
        r->state = kDone;
    }
    queue.clear();
    cv_done.notify_all();
}

namespace {

Request *find_locked(dbg_server *s, uint64_t id) {
    auto it = s->reqs.find(id);
    return it == s->reqs.end() ? nullptr : it->second.get();
}

int submit_common(dbg_server *s, std::unique_ptr<Request> r, uint64_t vertices, uint64_t *id) {
    r->binned = (s->cfg.flags & DBG_F_BINNED) && r->k <= 31;
    size_request(s->cfg, vertices, *r);
    if (r->bytes > s->cfg.hbm_budget) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->st.rejected;
        return DBG_E_NOMEM;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return DBG_E_STATE;
    r->id = s->next_id++;
    r->t_submit = s->now();
    *id = r->id;
    s->queue.push_back(r.get());
    s->reqs.emplace(r->id, std::move(r));
    ++s->st.submitted;
    s->cv_work.notify_one();
    return DBG_OK;
}

}  // namespace

extern "C" {

int dbg_server_create(const dbg_server_config *cfg_in, dbg_server **out) {
    if (!out) return DBG_E_INVAL;
    *out = nullptr;
    dbg_server_config c{};
    if (cfg_in) c = *cfg_in;
    else c.device = -1;
    if (!c.hbm_budget) c.hbm_budget = 200000000000ull;
    if (!c.max_batch_bytes) c.max_batch_bytes = 1ull << 30;
    if (!c.max_batch) c.max_batch = 64;
    if (!c.flags) c.flags = DBG_F_BINNED;
    if (c.load_factor == 0) c.load_factor = 0.5;
    if (!c.slots) c.slots = 2;
    if (!(c.load_factor > 0 && c.load_factor < 1) || c.slots > 8 || c.max_batch > 4096) return DBG_E_INVAL;
    if ((c.flags & DBG_F_BINNED) && c.load_factor > DBG_BINNED_MAX_LOAD) return DBG_E_INVAL;
    int device = c.device;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return DBG_E_DEVICE;
    DeviceGuard guard(device);
    if (!guard.ok) return DBG_E_DEVICE;
    std::unique_ptr<dbg_server> s(new dbg_server());
    s->cfg = c;
    s->device = device;
    s->t0 = Clock::now();
    for (uint32_t i = 0; i < c.slots; ++i) {
        s->slots.emplace_back(new Slot());
        if (s->slots.back()->init() != hipSuccess) {
            for (auto &x : s->slots) x->release();
            return DBG_E_DEVICE;
        }
    }
    dbg_server *p = s.get();
    s->worker = std::thread([p] { p->run(); });
    *out = s.release();
    return DBG_OK;
}

int dbg_server_submit(dbg_server *s, const char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                      uint64_t expected_vertices, uint64_t *id) {
    if (!s || !id || (n_reads && !offsets)) return DBG_E_INVAL;
    if (k < 2 || k > 32) return DBG_E_K;
    uint64_t windows = 0, kmers = 0;
    if (n_reads && !host_counts(offsets, n_reads, k, &windows, &kmers)) return DBG_E_INVAL;
    if (kmers > kCounterLimit) return DBG_E_RANGE;
    const uint64_t base = n_reads ? offsets[0] : 0;
    const uint64_t len = n_reads ? offsets[n_reads] - base : 0;
    if (len && !reads) return DBG_E_INVAL;
    std::unique_ptr<Request> r(new Request());
    r->k = k;
    r->n_reads = n_reads;
    r->reads_len = len;
    r->h_reads.assign(reinterpret_cast<const uint8_t *>(reads) + base,
                      reinterpret_cast<const uint8_t *>(reads) + base + len);
    r->h_off.resize(n_reads);
    for (uint64_t i = 0; i < n_reads; ++i) r->h_off[i] = offsets[i] - base;
    return submit_common(s, std::move(r), expected_vertices ? expected_vertices : std::max<uint64_t>(windows, 1),
                         id);
}

int dbg_server_submit_device(dbg_server *s, const uint8_t *d_reads, uint64_t reads_len, const uint64_t *d_offsets,
                             uint64_t n_reads, uint32_t k, uint64_t expected_vertices, uint64_t *id) {
    if (!s || !id || (n_reads && !d_offsets) || (reads_len && !d_reads)) return DBG_E_INVAL;
    if (k < 2 || k > 32) return DBG_E_K;
    if (reads_len > kCounterLimit + (uint64_t)n_reads * (k - 1)) return DBG_E_RANGE;
    std::unique_ptr<Request> r(new Request());
    r->k = k;
    r->n_reads = n_reads;
    r->reads_len = n_reads ? reads_len : 0;
    r->device_input = true;
    r->d_reads = d_reads;
    r->d_off = d_offsets;
    return submit_common(s, std::move(r), expected_vertices ? expected_vertices : std::max<uint64_t>(reads_len, 1),
                         id);
}

int dbg_server_poll(dbg_server *s, uint64_t id, int32_t *status) {
    if (!s) return DBG_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    Request *r = find_locked(s, id);
    if (!r) return DBG_E_INVAL;
    if (r->state != kDone) return DBG_PENDING;
    if (status) *status = r->status;
    return DBG_OK;
}

int dbg_server_wait(dbg_server *s, uint64_t id, double timeout_s, int32_t *status) {
    if (!s) return DBG_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    Request *r = find_locked(s, id);
    if (!r) return DBG_E_INVAL;
    auto done = [&] { return r->state == kDone; };
    if (timeout_s < 0) s->cv_done.wait(lk, done);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    if (!done()) return DBG_PENDING;
    if (status) *status = r->status;
    return DBG_OK;
}

int dbg_server_graph(dbg_server *s, uint64_t id, dbg_graph **g) {
    if (!s || !g) return DBG_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    Request *r = find_locked(s, id);
    if (!r) return DBG_E_INVAL;
    if (r->state != kDone) return DBG_PENDING;
    if (r->status != DBG_OK) return r->status;
    *g = r->g;
    return DBG_OK;
}

int dbg_server_times(dbg_server *s, uint64_t id, double *t_submit, double *t_start, double *t_done) {
    if (!s) return DBG_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    Request *r = find_locked(s, id);
    if (!r) return DBG_E_INVAL;
    if (t_submit) *t_submit = r->t_submit;
    if (t_start) *t_start = r->t_start;
    if (t_done) *t_done = r->t_done;
    return r->state == kDone ? DBG_OK : DBG_PENDING;
}

int dbg_server_release(dbg_server *s, uint64_t id) {
    if (!s) return DBG_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return DBG_E_INVAL;
    Request *r = it->second.get();
    if (r->state != kDone) return DBG_PENDING;
    if (r->g) {
        s->returned.push_back(r->g);
        s->resident -= r->bytes;
    }
    ++s->st.released;
    s->reqs.erase(it);
    s->cv_work.notify_one();
    return DBG_OK;
}

int dbg_server_get_stats(dbg_server *s, dbg_server_stats *out) {
    if (!s || !out) return DBG_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = s->queue.size();
    out->running = s->st.admitted - s->st.completed;
    out->resident_bytes = s->resident;
    return DBG_OK;
}

void dbg_server_destroy(dbg_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard guard(s->device);
    for (auto &x : s->reqs)
        if (x.second->g) dbg_destroy(x.second->g);
    for (dbg_graph *g : s->returned) dbg_destroy(g);
    for (Idle &x : s->idle) dbg_destroy(x.g);
    for (auto &x : s->slots) x->release();
    delete s;
}

}  // extern "C"
