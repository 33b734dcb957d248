/*
 * record_compare.c -- test helper: exact comparison of a graph's records with
 * the oracle's, without sorting the graph's records (test infrastructure; it
 * shares nothing with the library and computes no part of the graph).
 *
 * The oracle's records for one key-space partition (keys ascending, four
 * counters each) are indexed in an open-addressing hash set; every graph
 * record of that partition (part[i] == p, or every record when part is NULL)
 * is looked up and its counters compared, and each oracle record is marked
 * when found.  The graph equals the oracle on the partition exactly when no
 * record is missing, none differs, none is found twice and every oracle
 * record is found.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t selected;   /* graph records of the partition */
    uint64_t missing;    /* their keys absent from the oracle */
    uint64_t wrong;      /* present, with different counters */
    uint64_t repeated;   /* a key met a second time */
    uint64_t found;      /* oracle records met */
    uint64_t first_bad;  /* index of the first bad graph record, or ~0 */
} cmp_result;

/* Fibonacci hashing (Knuth, TAOCP vol. 3, 6.4): the top bits of key * 2^64/phi. */
static uint64_t home(uint64_t key, int bits) { return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits); }

int cmp_records(const uint64_t *okeys, const uint32_t *ocounts, uint64_t V, const uint64_t *gkeys,
                const uint32_t *gcounts, uint64_t n, const uint32_t *part, uint32_t p, cmp_result *out) {
    memset(out, 0, sizeof *out);
    out->first_bad = ~0ull;
    uint64_t cap = 64;
    int bits = 6;
    while (cap < 2 * V) cap <<= 1, ++bits;
    uint32_t *slot = (uint32_t *)malloc(cap * sizeof(uint32_t)); /* oracle index + 1; 0 = empty */
    uint8_t *seen = (uint8_t *)calloc(V ? V : 1, 1);
    if (!slot || !seen || V >= 0xffffffffull) {
        free(slot);
        free(seen);
        return -1;
    }
    memset(slot, 0, cap * sizeof(uint32_t));
    const uint64_t mask = cap - 1;
    for (uint64_t j = 0; j < V; ++j) {
        uint64_t s = home(okeys[j], bits);
        while (slot[s]) s = (s + 1) & mask;
        slot[s] = (uint32_t)(j + 1);
    }
    for (uint64_t i = 0; i < n; ++i) {
        if (part && part[i] != p) continue;
        ++out->selected;
        const uint64_t key = gkeys[i];
        uint64_t s = home(key, bits);
        uint64_t j = ~0ull;
        while (slot[s]) {
            if (okeys[slot[s] - 1] == key) {
                j = slot[s] - 1;
                break;
            }
            s = (s + 1) & mask;
        }
        int bad = 0;
        if (j == ~0ull) {
            ++out->missing;
            bad = 1;
        } else {
            if (seen[j]) {
                ++out->repeated;
                bad = 1;
            } else {
                seen[j] = 1;
                ++out->found;
            }
            if (memcmp(gcounts + 4 * i, ocounts + 4 * j, 16) != 0) {
                ++out->wrong;
                bad = 1;
            }
        }
        if (bad && out->first_bad == ~0ull) out->first_bad = i;
    }
    free(slot);
    free(seen);
    return 0;
}
