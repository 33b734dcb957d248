/*
 * dbg_oracle.c -- CPU oracle for the A-Bruijn graph build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * What it computes is the plain definition of the graph (Background section,
 * the A-Bruijn graph paragraph; Methods, "Lock-free graph creation algorithm"
 * and the makeGraph / addLeftVertex / addRightVertex description):
 *
 *   - every substring s0..s(k-1) of a read is an edge from the vertex
 *     s0..s(k-2) to the vertex s1..s(k-1);
 *   - the edge carries an integer: how many times that k-mer occurs over all
 *     reads; a vertex keeps one such counter per letter of the alphabet;
 *   - the source vertex has its counter for s(k-1) raised by one, the target
 *     vertex is only made to exist (adding a right vertex never increments).
 *
 * Hence, for a read r of length L >= k, windows j = 0 .. L-k+1 are vertices
 * (the last one only as a target), and for j = 0 .. L-k the counter of vertex
 * r[j..j+k-2] for letter r[j+k-1] is raised by one.  A read shorter than k has
 * no k-mer and contributes nothing.
 *
 * Letter code (Methods, "Graph data structure", the ASCII trick): the counter
 * index of a letter c is (c >> 1) & 3, giving A=0, C=1, T=2, G=3; lower case
 * letters map identically.  Any byte outside ACGTacgt is rejected here.
 *
 * Vertex key: the (k-1)-mer written as 2-bit codes, first base most
 * significant, right-aligned in a uint64 (k <= 32).  Each key is packed from
 * the bases directly, window by window, with no rolling update.  For longer k
 * (up to 64, the paper's runs use k = 51) oracle_build_wide keeps the same
 * packing in a 128-bit integer and reports it as a high and a low word.
 *
 * The store is a separately chained hash map, as in the paper's structure, but
 * single threaded (no atomics are needed: the result is a multiset count and
 * does not depend on the order of insertion).  Output records are sorted by
 * key, which is the canonical form every comparison uses.
 *
 * Partitioned mode: with part_count = P > 1, only keys whose partition
 * (oracle_partition_of) equals part_index are kept.  The union of the P
 * partitions is exactly the unpartitioned result; memory drops by P.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_INVAL (-1)
#define ORACLE_E_K (-2)
#define ORACLE_E_BASE (-3)
#define ORACLE_E_NOMEM (-4)

typedef struct {
    uint64_t key;
    uint32_t cnt[4];
    int64_t next; /* index of the next record in the same bucket, -1 ends */
} orec;

typedef struct {
    int64_t *head;
    uint64_t nbuckets; /* power of two */
    int bits;
    orec *rec;
    uint64_t n, cap;
} omap;

/* Letter -> counter index, as the paper defines it.  Returns -1 for a byte
 * that is not one of ACGTacgt. */
static int letter_index(unsigned char c) {
    switch (c) {
    case 'A': case 'a': case 'C': case 'c':
    case 'G': case 'g': case 'T': case 't':
        return (c >> 1) & 3;
    default:
        return -1;
    }
}

/* Knuth's multiplicative (Fibonacci) hashing of the key into 2^bits buckets. */
static uint64_t bucket_of(uint64_t key, int bits) {
    return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits);
}

uint32_t oracle_partition_of(uint64_t key, uint32_t part_count) {
    if (part_count <= 1) return 0;
    uint64_t h = key * 0xD6E8FEB86659FD93ull;
    h ^= h >> 32;
    return (uint32_t)(h % part_count);
}

/* Partition of each of n keys, for selecting the matching slice of another
 * build's output. */
void oracle_partition_many(const uint64_t *keys, uint64_t n, uint32_t part_count,
                           uint32_t *parts) {
    for (uint64_t i = 0; i < n; ++i) parts[i] = oracle_partition_of(keys[i], part_count);
}

static int omap_init(omap *m, int bits) {
    m->bits = bits;
    m->nbuckets = 1ull << bits;
    m->head = (int64_t *)malloc(m->nbuckets * sizeof(int64_t));
    if (!m->head) return ORACLE_E_NOMEM;
    for (uint64_t i = 0; i < m->nbuckets; ++i) m->head[i] = -1;
    m->cap = 1024;
    m->n = 0;
    m->rec = (orec *)malloc(m->cap * sizeof(orec));
    return m->rec ? ORACLE_OK : ORACLE_E_NOMEM;
}

static void omap_free(omap *m) {
    free(m->head);
    free(m->rec);
    m->head = NULL;
    m->rec = NULL;
}

static int omap_rehash(omap *m) {
    int bits = m->bits + 1;
    int64_t *h = (int64_t *)malloc((1ull << bits) * sizeof(int64_t));
    if (!h) return ORACLE_E_NOMEM;
    for (uint64_t i = 0; i < (1ull << bits); ++i) h[i] = -1;
    for (uint64_t i = 0; i < m->n; ++i) {
        uint64_t b = bucket_of(m->rec[i].key, bits);
        m->rec[i].next = h[b];
        h[b] = (int64_t)i;
    }
    free(m->head);
    m->head = h;
    m->bits = bits;
    m->nbuckets = 1ull << bits;
    return ORACLE_OK;
}

/* Find the record of `key`, creating it with zero counters if absent. */
static orec *omap_find_or_add(omap *m, uint64_t key, int *err) {
    uint64_t b = bucket_of(key, m->bits);
    for (int64_t i = m->head[b]; i >= 0; i = m->rec[i].next)
        if (m->rec[i].key == key) return &m->rec[i];
    if (m->n == m->cap) {
        uint64_t nc = m->cap * 2;
        orec *r = (orec *)realloc(m->rec, nc * sizeof(orec));
        if (!r) { *err = ORACLE_E_NOMEM; return NULL; }
        m->rec = r;
        m->cap = nc;
    }
    if (m->n >= m->nbuckets) {
        if (omap_rehash(m) != ORACLE_OK) { *err = ORACLE_E_NOMEM; return NULL; }
        b = bucket_of(key, m->bits);
    }
    orec *r = &m->rec[m->n];
    r->key = key;
    r->cnt[0] = r->cnt[1] = r->cnt[2] = r->cnt[3] = 0;
    r->next = m->head[b];
    m->head[b] = (int64_t)m->n;
    m->n++;
    return r;
}

/* The (k-1)-mer starting at s, packed from scratch. */
static uint64_t vertex_key(const unsigned char *s, uint32_t len) {
    uint64_t v = 0;
    for (uint32_t i = 0; i < len; ++i) v = (v << 2) | (uint64_t)letter_index(s[i]);
    return v;
}

static int cmp_rec(const void *a, const void *b) {
    uint64_t x = ((const orec *)a)->key, y = ((const orec *)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Checks the inputs the way the boundary is specified to: offsets must be
 * non-decreasing, 2 <= k <= 32, every byte of every read in ACGTacgt. */
int oracle_validate(const unsigned char *reads, const uint64_t *offsets,
                    uint64_t n_reads, uint32_t k) {
    if (k < 2 || k > 32) return ORACLE_E_K;
    if (n_reads == 0) return ORACLE_OK;
    if (!offsets) return ORACLE_E_INVAL;
    for (uint64_t i = 0; i < n_reads; ++i)
        if (offsets[i + 1] < offsets[i]) return ORACLE_E_INVAL;
    if (offsets[n_reads] > offsets[0] && !reads) return ORACLE_E_INVAL;
    for (uint64_t p = offsets[0]; p < offsets[n_reads]; ++p)
        if (letter_index(reads[p]) < 0) return ORACLE_E_BASE;
    return ORACLE_OK;
}

/*
 * Build the graph of reads[offsets[i] .. offsets[i+1]) for i < n_reads.
 * On success *out_keys (sorted ascending) and *out_counts (4 per vertex, in
 * counter-index order A,C,T,G) are malloc'ed and *out_n is the vertex count;
 * free them with oracle_free.  Only keys in partition part_index of
 * part_count are kept.
 */
int oracle_build(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads,
                 uint32_t k, uint32_t part_count, uint32_t part_index,
                 uint64_t **out_keys, uint32_t **out_counts, uint64_t *out_n) {
    if (!out_keys || !out_counts || !out_n) return ORACLE_E_INVAL;
    *out_keys = NULL;
    *out_counts = NULL;
    *out_n = 0;
    if (part_count == 0) part_count = 1;
    if (part_index >= part_count) return ORACLE_E_INVAL;
    int rc = oracle_validate(reads, offsets, n_reads, k);
    if (rc != ORACLE_OK) return rc;

    omap m;
    rc = omap_init(&m, 16);
    if (rc != ORACLE_OK) { omap_free(&m); return rc; }

    for (uint64_t r = 0; r < n_reads; ++r) {
        const unsigned char *s = reads + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        if (L < k) continue; /* no k-mer in this read */
        for (uint64_t j = 0; j + k - 1 <= L; ++j) {
            /* window j: vertex s[j .. j+k-2] */
            uint64_t key = vertex_key(s + j, k - 1);
            if (oracle_partition_of(key, part_count) != part_index) continue;
            int err = ORACLE_OK;
            orec *v = omap_find_or_add(&m, key, &err);
            if (!v) { omap_free(&m); return err; }
            if (j + k <= L) /* an edge leaves: the k-mer s[j .. j+k-1] */
                v->cnt[letter_index(s[j + k - 1])] += 1;
        }
    }

    qsort(m.rec, m.n, sizeof(orec), cmp_rec);
    uint64_t *keys = (uint64_t *)malloc((m.n ? m.n : 1) * sizeof(uint64_t));
    uint32_t *cnts = (uint32_t *)malloc((m.n ? m.n : 1) * 4 * sizeof(uint32_t));
    if (!keys || !cnts) {
        free(keys);
        free(cnts);
        omap_free(&m);
        return ORACLE_E_NOMEM;
    }
    for (uint64_t i = 0; i < m.n; ++i) {
        keys[i] = m.rec[i].key;
        memcpy(&cnts[4 * i], m.rec[i].cnt, 4 * sizeof(uint32_t));
    }
    *out_keys = keys;
    *out_counts = cnts;
    *out_n = m.n;
    omap_free(&m);
    return ORACLE_OK;
}

/* Counters of a single vertex, computed by scanning every window of every
 * read.  This is the one-by-one form used to check sampled outputs of large
 * builds.  Returns 1 if the vertex occurs as a window, 0 if not. */
int oracle_vertex_counts(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads,
                         uint32_t k, uint64_t key, uint32_t *counts4) {
    int seen = 0;
    counts4[0] = counts4[1] = counts4[2] = counts4[3] = 0;
    for (uint64_t r = 0; r < n_reads; ++r) {
        const unsigned char *s = reads + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        if (L < k) continue;
        for (uint64_t j = 0; j + k - 1 <= L; ++j) {
            if (vertex_key(s + j, k - 1) != key) continue;
            seen = 1;
            if (j + k <= L) counts4[letter_index(s[j + k - 1])] += 1;
        }
    }
    return seen;
}

void oracle_free(void *p) { free(p); }

/* ---------------------------------------------------------------- contigs
 *
 * Contigs of a graph (Methods, "Finding contigs", Algorithm 5), computed from
 * the graph's records (keys ascending, four counters each), as this oracle
 * reads the passage:
 *
 *   - first(v) holds when v was only ever added as a left vertex, i.e. no
 *     k-mer ends in v: in-degree 0 (the flag is cleared whenever v is added
 *     as a right vertex);
 *   - v has an out-edge for every letter whose counter is non-zero;
 *   - a contig starts at every vertex with first(v) or with more than one
 *     out-edge, one contig per out-edge, and spells v followed by the letter
 *     of each edge it takes;
 *   - from the edge's target it keeps going while the vertex it stands on has
 *     exactly one out-edge; it stops on a vertex with zero or several
 *     out-edges, and (a case the passage leaves open: a loop of one-edge
 *     vertices would never end) on a vertex it has already stood on.  The
 *     vertex it stops on is part of the contig.
 *
 * first(v) is computed the way the paper maintains it: it starts true for
 * every vertex and is cleared on the target of every edge.  Contigs are
 * produced in the order of their start key, then letter code; comparisons
 * sort them.  Vertices are found through a chained index over the keys.
 */
typedef struct {
    int64_t *head, *next;
    int bits;
} oindex;

static int oindex_build(oindex *x, const uint64_t *keys, uint64_t n) {
    x->bits = 1;
    while ((1ull << x->bits) < 2 * n) ++x->bits;
    x->head = (int64_t *)malloc((1ull << x->bits) * sizeof(int64_t));
    x->next = (int64_t *)malloc((n ? n : 1) * sizeof(int64_t));
    if (!x->head || !x->next) return ORACLE_E_NOMEM;
    for (uint64_t b = 0; b < (1ull << x->bits); ++b) x->head[b] = -1;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t b = bucket_of(keys[i], x->bits);
        x->next[i] = x->head[b];
        x->head[b] = (int64_t)i;
    }
    return ORACLE_OK;
}

static int64_t oindex_find(const oindex *x, const uint64_t *keys, uint64_t key) {
    for (int64_t i = x->head[bucket_of(key, x->bits)]; i >= 0; i = x->next[i])
        if (keys[i] == key) return i;
    return -1;
}

static uint32_t out_degree(const uint32_t *counts, uint64_t i) {
    uint32_t d = 0;
    for (int c = 0; c < 4; ++c) d += counts[4 * i + c] ? 1u : 0u;
    return d;
}

typedef struct {
    unsigned char *seq;
    uint64_t len, cap;
    uint64_t *off;
    uint64_t n, off_cap;
} ocontigs;

static int push_base(ocontigs *o, unsigned char b) {
    if (o->len == o->cap) {
        const uint64_t cap = o->cap ? 2 * o->cap : 1 << 16;
        unsigned char *p = (unsigned char *)realloc(o->seq, cap);
        if (!p) return ORACLE_E_NOMEM;
        o->seq = p;
        o->cap = cap;
    }
    o->seq[o->len++] = b;
    return ORACLE_OK;
}

static int push_offset(ocontigs *o, uint64_t v) {
    if (o->n + 1 >= o->off_cap) {
        const uint64_t cap = o->off_cap ? 2 * o->off_cap : 1 << 12;
        uint64_t *p = (uint64_t *)realloc(o->off, cap * sizeof(uint64_t));
        if (!p) return ORACLE_E_NOMEM;
        o->off = p;
        o->off_cap = cap;
    }
    o->off[o->n] = v;
    return ORACLE_OK;
}

/* Output: *seq_out (ASCII, contigs back to back) and *off_out (n_contigs + 1
 * offsets into it); both freed with oracle_free. */
int oracle_contigs(const uint64_t *keys, const uint32_t *counts, uint64_t n, uint32_t k,
                   unsigned char **seq_out, uint64_t **off_out, uint64_t *n_contigs, uint64_t *seq_len) {
    static const unsigned char letters[4] = {'A', 'C', 'T', 'G'};
    if (!seq_out || !off_out || !n_contigs || !seq_len || (n && (!keys || !counts))) return ORACLE_E_INVAL;
    if (k < 2 || k > 32) return ORACLE_E_K;
    *seq_out = NULL;
    *off_out = NULL;
    *n_contigs = 0;
    *seq_len = 0;
    const uint32_t km1 = k - 1;
    const uint64_t mask = (1ull << (2 * km1)) - 1;
    ocontigs o = {0};
    oindex ix = {0};
    uint64_t *stamp = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t)); /* walk id of the last visit */
    unsigned char *first = (unsigned char *)malloc(n ? n : 1);
    int rc = (stamp && first) ? oindex_build(&ix, keys, n) : ORACLE_E_NOMEM;
    for (uint64_t i = 0; i < n && rc == ORACLE_OK; ++i) first[i] = 1;
    for (uint64_t i = 0; i < n && rc == ORACLE_OK; ++i)
        for (uint64_t c = 0; c < 4; ++c) {
            if (!counts[4 * i + c]) continue;
            const int64_t j = oindex_find(&ix, keys, ((keys[i] << 2) | c) & mask);
            if (j < 0) { rc = ORACLE_E_INVAL; break; } /* a target is always a vertex */
            first[j] = 0;
        }
    uint64_t walk = 0;
    for (uint64_t i = 0; i < n && rc == ORACLE_OK; ++i) {
        const uint64_t v = keys[i];
        const uint32_t deg = out_degree(counts, i);
        if (deg == 0) continue;
        if (!(deg >= 2 || first[i])) continue;
        for (uint32_t c = 0; c < 4 && rc == ORACLE_OK; ++c) {
            if (!counts[4 * i + c]) continue;
            ++walk;
            rc = push_offset(&o, o.len);
            for (uint32_t b = 0; b < km1 && rc == ORACLE_OK; ++b)
                rc = push_base(&o, letters[(v >> (2 * (km1 - 1 - b))) & 3]);
            if (rc == ORACLE_OK) rc = push_base(&o, letters[c]);
            stamp[i] = walk;
            uint64_t cur = ((v << 2) | c) & mask;
            while (rc == ORACLE_OK) {
                const int64_t j = oindex_find(&ix, keys, cur);
                if (j < 0) { rc = ORACLE_E_INVAL; break; }
                if (out_degree(counts, (uint64_t)j) != 1 || stamp[j] == walk) break;
                stamp[j] = walk;
                uint32_t only = 0;
                while (!counts[4 * (uint64_t)j + only]) ++only;
                rc = push_base(&o, letters[only]);
                cur = ((cur << 2) | only) & mask;
            }
            ++o.n;
        }
    }
    free(stamp);
    free(first);
    free(ix.head);
    free(ix.next);
    if (rc == ORACLE_OK) rc = push_offset(&o, o.len);
    if (rc != ORACLE_OK) {
        free(o.seq);
        free(o.off);
        return rc;
    }
    *seq_out = o.seq;
    *off_out = o.off;
    *n_contigs = o.n;
    *seq_len = o.len;
    return ORACLE_OK;
}

/* Order-free digest of a set of strings (for comparing very large contig
 * sets): the sum, modulo 2^64, of a 64-bit FNV-1a hash of each string passed
 * through MurmurHash3's 64-bit finalizer (fmix64). */
uint64_t oracle_strings_digest(const unsigned char *seq, const uint64_t *off, uint64_t n) {
    uint64_t sum = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t h = 0xcbf29ce484222325ull;
        for (uint64_t p = off[i]; p < off[i + 1]; ++p) h = (h ^ seq[p]) * 0x100000001b3ull;
        h ^= h >> 33;
        h *= 0xff51afd7ed558ccdull;
        h ^= h >> 33;
        h *= 0xc4ceb9fe1a85ec53ull;
        h ^= h >> 33;
        sum += h;
    }
    return sum;
}

/* ---------------------------------------------------------------- normalization
 *
 * Normalized counters (Methods, "Normalization of graph"): every counter is
 * divided by the number of times a k-mer of the genome is expected to be
 * read, reads * (read length - k + 1) / genome size.  With reads of any
 * length the numerator is the total number of k-mers read, `total`, so
 *   normalized(c) = c * genome / total, rounded half up,
 * computed exactly in 128-bit integers; saturated at 2^32 - 1.  With
 * genome = 0 the counters are left as they are.  out8 (if not NULL) receives
 * the same values saturated at 255, the paper's 8-bit counter.
 */
void oracle_normalize(const uint32_t *counts, uint64_t n, uint64_t genome, uint64_t total,
                      uint32_t *out32, unsigned char *out8) {
    for (uint64_t i = 0; i < n; ++i) {
        unsigned __int128 v = counts[i];
        if (genome && total) {
            const unsigned __int128 num = 2 * (unsigned __int128)counts[i] * genome + total;
            v = num / (2 * (unsigned __int128)total);
        }
        const uint32_t v32 = v > 0xffffffffu ? 0xffffffffu : (uint32_t)v;
        if (out32) out32[i] = v32;
        if (out8) out8[i] = v32 > 255 ? 255 : (unsigned char)v32;
    }
}

/* ---------------------------------------------------------------- long k
 *
 * The same graph for 2 <= k <= 64: a (k-1)-mer of up to 63 bases is packed
 * from scratch into a 128-bit integer (first base most significant), split
 * into a high and a low 64-bit word.  A separately chained map of its own;
 * output sorted by (high, low).
 */
typedef unsigned __int128 u128;

typedef struct {
    u128 key;
    uint32_t cnt[4];
    int64_t next;
} wrec;

static uint64_t wide_bucket(u128 key, int bits) {
    const uint64_t x = (uint64_t)(key >> 64) * 0xC2B2AE3D27D4EB4Full ^ (uint64_t)key;
    return (x * 0x9E3779B97F4A7C15ull) >> (64 - bits);
}

static int cmp_wrec(const void *a, const void *b) {
    const u128 x = ((const wrec *)a)->key, y = ((const wrec *)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int oracle_build_wide(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                      uint64_t **out_hi, uint64_t **out_lo, uint32_t **out_counts, uint64_t *out_n) {
    if (!out_hi || !out_lo || !out_counts || !out_n) return ORACLE_E_INVAL;
    *out_hi = *out_lo = NULL;
    *out_counts = NULL;
    *out_n = 0;
    if (k < 2 || k > 64) return ORACLE_E_K;
    if (n_reads && !offsets) return ORACLE_E_INVAL;
    for (uint64_t i = 0; i < n_reads; ++i)
        if (offsets[i + 1] < offsets[i]) return ORACLE_E_INVAL;
    if (n_reads && offsets[n_reads] > offsets[0] && !reads) return ORACLE_E_INVAL;
    for (uint64_t p = n_reads ? offsets[0] : 0; n_reads && p < offsets[n_reads]; ++p)
        if (letter_index(reads[p]) < 0) return ORACLE_E_BASE;

    int bits = 16;
    uint64_t cap = 1024, n = 0;
    int64_t *head = (int64_t *)malloc((1ull << bits) * sizeof(int64_t));
    wrec *rec = (wrec *)malloc(cap * sizeof(wrec));
    if (!head || !rec) { free(head); free(rec); return ORACLE_E_NOMEM; }
    for (uint64_t b = 0; b < (1ull << bits); ++b) head[b] = -1;
    for (uint64_t r = 0; r < n_reads; ++r) {
        const unsigned char *s = reads + offsets[r];
        const uint64_t L = offsets[r + 1] - offsets[r];
        if (L < k) continue;
        for (uint64_t j = 0; j + k - 1 <= L; ++j) {
            u128 key = 0;
            for (uint32_t i = 0; i < k - 1; ++i) key = (key << 2) | (u128)letter_index(s[j + i]);
            int64_t at = -1;
            for (int64_t i = head[wide_bucket(key, bits)]; i >= 0; i = rec[i].next)
                if (rec[i].key == key) { at = i; break; }
            if (at < 0) {
                if (n == cap) {
                    wrec *x = (wrec *)realloc(rec, 2 * cap * sizeof(wrec));
                    if (!x) { free(head); free(rec); return ORACLE_E_NOMEM; }
                    rec = x;
                    cap *= 2;
                }
                if (n >= (1ull << bits)) { /* keep chains short: double the buckets */
                    ++bits;
                    int64_t *h = (int64_t *)malloc((1ull << bits) * sizeof(int64_t));
                    if (!h) { free(head); free(rec); return ORACLE_E_NOMEM; }
                    for (uint64_t b = 0; b < (1ull << bits); ++b) h[b] = -1;
                    for (uint64_t i = 0; i < n; ++i) {
                        const uint64_t b = wide_bucket(rec[i].key, bits);
                        rec[i].next = h[b];
                        h[b] = (int64_t)i;
                    }
                    free(head);
                    head = h;
                }
                const uint64_t b = wide_bucket(key, bits);
                rec[n].key = key;
                rec[n].cnt[0] = rec[n].cnt[1] = rec[n].cnt[2] = rec[n].cnt[3] = 0;
                rec[n].next = head[b];
                head[b] = (int64_t)n;
                at = (int64_t)n++;
            }
            if (j + k <= L) rec[at].cnt[letter_index(s[j + k - 1])] += 1;
        }
    }
    free(head);
    qsort(rec, n, sizeof(wrec), cmp_wrec);
    uint64_t *hi = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t *lo = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint32_t *cnts = (uint32_t *)malloc((n ? n : 1) * 4 * sizeof(uint32_t));
    if (!hi || !lo || !cnts) { free(hi); free(lo); free(cnts); free(rec); return ORACLE_E_NOMEM; }
    for (uint64_t i = 0; i < n; ++i) {
        hi[i] = (uint64_t)(rec[i].key >> 64);
        lo[i] = (uint64_t)rec[i].key;
        memcpy(&cnts[4 * i], rec[i].cnt, 4 * sizeof(uint32_t));
    }
    free(rec);
    *out_hi = hi;
    *out_lo = lo;
    *out_counts = cnts;
    *out_n = n;
    return ORACLE_OK;
}
