/*
 * oracle_sanitize.c -- drives every entry point of the CPU oracle
 * (oracle/dbg_oracle.c, linked in directly) over seeded random inputs, for a
 * build under AddressSanitizer and UndefinedBehaviorSanitizer: ragged reads
 * (empty, shorter than k, exactly k), mixed case, rejected bytes, k from 2
 * to 64, partitioned builds, one-vertex scans, contigs, normalization.  It
 * checks only what any correct graph satisfies (total count = sum of
 * max(0, L - k + 1), partitions add up to the whole), so that a memory or
 * arithmetic fault, not a wrong value, is what this run looks for.  Exit
 * status 0 and "ok" on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_validate(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k);
int oracle_build(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                 uint32_t part_count, uint32_t part_index, uint64_t **out_keys, uint32_t **out_counts,
                 uint64_t *out_n);
int oracle_vertex_counts(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                         uint64_t key, uint32_t *out);
void oracle_partition_many(const uint64_t *keys, uint64_t n, uint32_t part_count, uint32_t *parts);
int oracle_contigs(const uint64_t *keys, const uint32_t *counts, uint64_t n, uint32_t k, unsigned char **seq_out,
                   uint64_t **off_out, uint64_t *n_contigs, uint64_t *seq_len);
uint64_t oracle_strings_digest(const unsigned char *seq, const uint64_t *off, uint64_t n);
void oracle_normalize(const uint32_t *counts, uint64_t n, uint64_t genome, uint64_t total, uint32_t *out32,
                      uint8_t *out8);
int oracle_build_wide(const unsigned char *reads, const uint64_t *offsets, uint64_t n_reads, uint32_t k,
                      uint64_t **out_hi, uint64_t **out_lo, uint32_t **out_counts, uint64_t *out_n);
void oracle_free(void *p);

static uint64_t rng_state = 0x243F6A8885A308D3ull;
static uint64_t next_u64(void) { /* xorshift64* (Vigna, 2016) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}
static uint32_t below(uint32_t n) { return (uint32_t)(next_u64() % n); }

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            if (failures < 20) printf("FAIL line %d: %s\n", __LINE__, #c); \
            ++failures;                                            \
        }                                                          \
    } while (0)

int main(void) {
    const char *alpha = "ACGTacgt";
    for (int round = 0; round < 300; ++round) {
        const uint32_t k = 2 + below(63);
        const uint64_t n = below(40);
        uint64_t *off = malloc((n + 1) * sizeof *off);
        off[0] = below(3);
        for (uint64_t i = 0; i < n; ++i) off[i + 1] = off[i] + (below(4) == 0 ? below(k + 1) : below(3 * k + 4));
        const uint64_t len = off[n] + 1;
        unsigned char *reads = malloc(len);
        const uint32_t letters = round % 3 == 0 ? 2 : 8; /* few letters: repeated vertices */
        for (uint64_t p = 0; p < len; ++p) reads[p] = (unsigned char)alpha[below(letters)];
        uint64_t kmers = 0;
        for (uint64_t i = 0; i < n; ++i)
            if (off[i + 1] - off[i] >= k) kmers += off[i + 1] - off[i] - k + 1;
        if (k <= 32) {
            CHECK(oracle_validate(reads, off, n, k) == 0);
            uint64_t *keys = NULL, nv = 0;
            uint32_t *counts = NULL;
            CHECK(oracle_build(reads, off, n, k, 1, 0, &keys, &counts, &nv) == 0);
            uint64_t total = 0;
            for (uint64_t v = 0; v < 4 * nv; ++v) total += counts[v];
            CHECK(total == kmers);
            uint64_t parts_v = 0;
            for (uint32_t p = 0; p < 3; ++p) {
                uint64_t *pk = NULL, pn = 0;
                uint32_t *pc = NULL;
                CHECK(oracle_build(reads, off, n, k, 3, p, &pk, &pc, &pn) == 0);
                parts_v += pn;
                oracle_free(pk);
                oracle_free(pc);
            }
            CHECK(parts_v == nv);
            if (nv) {
                uint32_t *part = malloc(nv * sizeof *part);
                oracle_partition_many(keys, nv, 5, part);
                for (uint64_t v = 0; v < nv; ++v) CHECK(part[v] < 5);
                free(part);
                uint32_t one[4];
                CHECK(oracle_vertex_counts(reads, off, n, k, keys[nv / 2], one) == 1);
                CHECK(memcmp(one, counts + 4 * (nv / 2), sizeof one) == 0);
                uint32_t *o32 = malloc(4 * nv * sizeof *o32);
                uint8_t *o8 = malloc(4 * nv);
                oracle_normalize(counts, 4 * nv, below(1000000), kmers, o32, o8);
                free(o32);
                free(o8);
                unsigned char *seq = NULL;
                uint64_t *coff = NULL;
                uint64_t nc = 0, sl = 0;
                CHECK(oracle_contigs(keys, counts, nv, k, &seq, &coff, &nc, &sl) == 0);
                (void)oracle_strings_digest(seq, coff, nc);
                oracle_free(seq);
                oracle_free(coff);
            }
            oracle_free(keys);
            oracle_free(counts);
        }
        {
            uint64_t *hi = NULL, *lo = NULL;
            uint32_t *wc = NULL;
            uint64_t wn = 0;
            CHECK(oracle_build_wide(reads, off, n, k, &hi, &lo, &wc, &wn) == 0);
            uint64_t total = 0;
            for (uint64_t v = 0; v < 4 * wn; ++v) total += wc[v];
            CHECK(total == kmers);
            oracle_free(hi);
            oracle_free(lo);
            oracle_free(wc);
        }
        if (n && off[n] > off[0]) { /* a rejected byte */
            reads[off[0] + below((uint32_t)(off[n] - off[0]))] = 'N';
            if (k <= 32) CHECK(oracle_validate(reads, off, n, k) != 0);
        }
        free(reads);
        free(off);
    }
    if (failures) return failures > 100 ? 100 : failures;
    printf("ok\n");
    return 0;
}
