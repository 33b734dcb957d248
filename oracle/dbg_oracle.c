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
 * the bases directly, window by window, with no rolling update.
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
