// lfdbg_cpu.cpp -- the paper's lock-free build on CPU threads, as a baseline.
//
// TEST AND BASELINE INFRASTRUCTURE ONLY.  Nothing in the product library
// links, loads or calls this file; the benchmark times it for context and the
// tests check its result against the oracle.  It shares no code with the GPU
// path.
//
// The design follows the paper's Methods ("Graph data structure",
// "Lock-free graph creation algorithm", Algorithms 1-4): a hash table of
// buckets, each the head of a singly linked list of vertex nodes; a node
// holds its (k-1)-mer and four atomic counters; threads take disjoint subsets
// of the reads and, for every k-mer, find or add its left vertex and raise the
// counter of the k-mer's last letter, then find or add its right vertex.  A
// node is added by a compare-and-swap of the bucket head: on failure the
// thread looks through the nodes that were pushed meanwhile (its vertex may be
// among them) before trying again.  Nodes come from a per-thread pool, so no
// allocator lock is taken (Methods, "Implementation issues").
//
// Departures from the paper's structure, none of which changes the work per
// k-mer or the result: the (k-1)-mer
// is stored packed in a 64-bit word rather than as a view into the reads;
// counters are 32-bit (the paper's 8-bit counters wrap on repeats); the
// explicit out-edge pointers and the `first` flag are not kept (the build's
// result does not depend on them).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

struct Node {
    uint64_t key;
    std::atomic<uint32_t> cnt[4];
    Node *next;
};

// Fixed-size slabs of nodes owned by one thread.
struct Pool {
    std::vector<Node *> slabs;
    size_t used = 0;
    static constexpr size_t kSlab = 1 << 16;
    Node *get() {
        if (slabs.empty() || used == kSlab) {
            Node *slab = new (std::nothrow) Node[kSlab];
            if (!slab) return nullptr;
            slabs.push_back(slab);
            used = 0;
        }
        return &slabs.back()[used++];
    }
    void release() {
        for (Node *s : slabs) delete[] s;
        slabs.clear();
    }
};

struct Table {
    std::vector<std::atomic<Node *>> heads;
    uint64_t mask;
    explicit Table(uint64_t n) : heads(n), mask(n - 1) {
        for (auto &h : heads) h.store(nullptr, std::memory_order_relaxed);
    }
    static uint64_t mixed(uint64_t x) {  // MurmurHash3's 64-bit finalizer
        x ^= x >> 33;
        x *= 0xff51afd7ed558ccdull;
        x ^= x >> 33;
        x *= 0xc4ceb9fe1a85ec53ull;
        x ^= x >> 33;
        return x;
    }
    // Find the node of `key` in the list from `from` up to (not including) `to`.
    static Node *scan(Node *from, Node *to, uint64_t key) {
        for (Node *n = from; n != to; n = n->next)
            if (n->key == key) return n;
        return nullptr;
    }
    Node *find_or_add(uint64_t key, Pool &pool, Node *&spare) {
        std::atomic<Node *> &head = heads[mixed(key) & mask];
        Node *seen = head.load(std::memory_order_acquire);
        if (Node *n = scan(seen, nullptr, key)) return n;
        Node *mine = spare ? spare : pool.get();
        if (!mine) return nullptr;
        spare = nullptr;
        mine->key = key;
        for (auto &c : mine->cnt) c.store(0, std::memory_order_relaxed);
        for (;;) {
            mine->next = seen;
            Node *expected = seen;
            if (head.compare_exchange_weak(expected, mine, std::memory_order_acq_rel, std::memory_order_acquire))
                return mine;
            // other nodes were pushed in front of `seen`: ours may be one of them
            if (Node *n = scan(expected, seen, key)) {
                spare = mine;  // unused; kept for this thread's next addition
                return n;
            }
            seen = expected;
        }
    }
};

int code_of(unsigned char c) {
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'T': case 't': return 2;
    case 'G': case 'g': return 3;
    default: return -1;
    }
}

}  // namespace

extern "C" {

// Build the graph of reads[offsets[i] .. offsets[i+1]) with `threads`
// threads and a table of `buckets` lists (rounded up to a power of two).
// Output: records sorted by key, freed with lfdbg_free.  Returns 0, -1 on bad
// arguments or bytes, -2 on allocation failure.  *seconds: the time of the
// threaded build only (reads are already in memory).
int lfdbg_build(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                uint32_t threads, uint64_t buckets, uint64_t **keys_out, uint32_t **counts_out, uint64_t *n_out,
                double *seconds) {
    if (!keys_out || !counts_out || !n_out || k < 2 || k > 32 || threads == 0 || (n_reads && !offsets))
        return -1;
    uint64_t nb = 1;
    while (nb < buckets) nb <<= 1;
    Table table(nb);
    std::vector<Pool> pools(threads);
    std::atomic<int> failed{0};
    const uint32_t km1 = k - 1;
    const uint64_t kmask = (km1 == 32) ? ~0ull : ((1ull << (2 * km1)) - 1);
    auto work = [&](uint32_t t) {
        Pool &pool = pools[t];
        Node *spare = nullptr;
        const uint64_t r0 = n_reads * t / threads, r1 = n_reads * (t + 1) / threads;
        for (uint64_t r = r0; r < r1 && !failed.load(std::memory_order_relaxed); ++r) {
            const unsigned char *s = reads + offsets[r];
            const uint64_t L = offsets[r + 1] - offsets[r];
            if (L < k) continue;
            uint64_t left = 0;
            bool ok = true;
            for (uint32_t b = 0; b < km1 && ok; ++b) {
                const int c = code_of(s[b]);
                ok = c >= 0;
                left = (left << 2) | (uint64_t)(c < 0 ? 0 : c);
            }
            for (uint64_t j = 0; ok && j + k <= L; ++j) {  // k-mer s[j .. j+k)
                const int c = code_of(s[j + km1]);
                if (c < 0) { ok = false; break; }
                const uint64_t right = ((left << 2) | (uint64_t)c) & kmask;
                Node *ln = table.find_or_add(left, pool, spare);
                if (!ln) { failed = -2; return; }
                ln->cnt[c].fetch_add(1, std::memory_order_relaxed);
                if (!table.find_or_add(right, pool, spare)) { failed = -2; return; }
                left = right;
            }
            if (!ok) { failed = -1; return; }
        }
    };
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    for (uint32_t t = 1; t < threads; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
    *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = failed.load();
    uint64_t n = 0;
    for (auto &h : table.heads)
        for (Node *x = h.load(std::memory_order_relaxed); x; x = x->next) ++n;
    uint64_t *keys = rc ? nullptr : static_cast<uint64_t *>(std::malloc((n ? n : 1) * sizeof(uint64_t)));
    uint32_t *counts = rc ? nullptr : static_cast<uint32_t *>(std::malloc((n ? n : 1) * 4 * sizeof(uint32_t)));
    if (!rc && (!keys || !counts)) rc = -2;
    if (!rc) {
        // order by key: gather pointers, sort
        std::vector<Node *> all;
        all.reserve(n);
        for (auto &h : table.heads)
            for (Node *x = h.load(std::memory_order_relaxed); x; x = x->next) all.push_back(x);
        std::sort(all.begin(), all.end(), [](const Node *a, const Node *b) { return a->key < b->key; });
        for (uint64_t i = 0; i < n; ++i) {
            keys[i] = all[i]->key;
            for (int c = 0; c < 4; ++c) counts[4 * i + c] = all[i]->cnt[c].load(std::memory_order_relaxed);
        }
    }
    for (auto &p : pools) p.release();
    if (rc) {
        std::free(keys);
        std::free(counts);
        return rc;
    }
    *keys_out = keys;
    *counts_out = counts;
    *n_out = n;
    return 0;
}

void lfdbg_free(void *p) { std::free(p); }

}  // extern "C"
