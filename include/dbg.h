/*
 * dbg.h -- C ABI of the MI355X A-Bruijn graph builder (libdbg.so).
 *
 * The graph is the one defined in the paper's Background section: every
 * length-k substring s0..s(k-1) of every read is an edge from the (k-1)-mer
 * vertex s0..s(k-2) to the (k-1)-mer vertex s1..s(k-1); a vertex has at most
 * four out-edges, one per letter, and each edge carries the number of times
 * its k-mer occurs in the reads.  The build follows the paper's makeGraph
 * (Methods, "Lock-free graph creation algorithm", Algorithms 2-4): for each
 * k-mer the source vertex is found or added and its counter for the last
 * letter is raised by one; the target vertex is only made to exist.  Here
 * vertices live in an open-addressing table in HBM, a slot is claimed with a
 * 64-bit compare-and-swap (the paper's CAS, Algorithm 1) and counters are
 * raised with 32-bit atomic adds; no lock is taken.
 *
 * Conventions used by every call:
 *   - Reads: read i is reads[offsets[i] .. offsets[i+1]) (bytes), so offsets
 *     has n_reads + 1 non-decreasing entries.  Bytes must be in ACGTacgt.  A
 *     read shorter than k has no k-mer and adds nothing.
 *   - Letter code (Methods, "Graph data structure"): (c >> 1) & 3, so A=0,
 *     C=1, T=2, G=3.
 *   - Vertex key: the (k-1)-mer as 2-bit letter codes, first base most
 *     significant, right-aligned in a uint64, for 2 <= k <= 32.  Longer k
 *     (33 <= k <= 64; the paper's runs use k = 51) is taken by dbg_build and
 *     dbg_build_device: the key K then has up to 126 bits and is given as two
 *     uint64 words, K >> 64 then K mod 2^64, so every key array holds two
 *     words per vertex.  Batches, the server and contigs take k <= 32.
 *   - Counts: four uint32 per vertex in letter-code order (A, C, T, G).
 *     Sink vertices (no out-edge) are vertices with four zero counters.
 *   - Return values: DBG_OK (0) or a negative DBG_E_* code.
 *   - Threads: one handle must not be used from two threads at once;
 *     different handles are independent.
 *   - Streams: a NULL stream means the handle's own stream.  A stream is a
 *     hipStream_t passed as void*.
 */
#ifndef DBG_H
#define DBG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

/* ---- error codes ---------------------------------------------------- */
#define DBG_OK 0
#define DBG_E_INVAL (-1)  /* NULL pointer, bad offsets, bad configuration */
#define DBG_E_K (-2)      /* k outside [2, 64] ([2, 32] for batches, the server and
                             contigs), or differs from the handle's k */
#define DBG_E_BASE (-3)   /* a read byte outside ACGTacgt */
#define DBG_E_NOMEM (-4)  /* device allocation refused */
#define DBG_E_FULL (-5)   /* table capacity exhausted; the handle is poisoned */
#define DBG_E_SPACE (-6)  /* output buffer smaller than the vertex count */
#define DBG_E_DEVICE (-7) /* HIP runtime error */
#define DBG_E_RANGE (-8)  /* cumulative k-mers on the handle would exceed 2^32-1 */
#define DBG_E_STATE (-9)  /* handle poisoned by an earlier DBG_E_FULL */
#define DBG_E_SCRATCH (-10) /* input needs more than the static scratch of dbg_build_device_static */

/* ---- configuration flags ------------------------------------------- */
#define DBG_F_MERGE 0x1u   /* merge equal vertices within a wavefront first */
#define DBG_F_TIMING 0x2u  /* time each build kernel with HIP events */
#define DBG_F_ENTRY32 0x4u /* 32-byte table entries (default 24 bytes) */
#define DBG_F_BINNED 0x8u  /* binned build: records partitioned by table segment,
                              claimed and counted in LDS (k <= 31, and 33 <= k <= 63
                              with two-word records; a graph whose first build has
                              k = 32 or k = 64 falls back to the direct build) */
#define DBG_F_GRAPH 0x10u  /* capture each build pass as HIP graphs on first use of
                              its size class and replay them afterwards */
#define DBG_F_STATS 0x20u  /* count probes and compare-and-swap races of every build
                              of the graph (dbg_get_probe_stats); its builds run the
                              counting kernels, which are slower (in a binned
                              segment they read each slot before any compare-and-
                              swap, where the other kernels probe with the compare-
                              and-swap itself; both find the same slots); batched
                              builds and dbg_build_device_static do not count */
#define DBG_F_TEST_HASH 0x40u /* tests only: every key's home slot is the low 3 bits
                              of its key (of its image in a binned segment), so all
                              keys of a table (of a segment) share one probe chain
                              and race for its slots; results are unchanged, builds
                              are far slower, and a direct table whose chain passes
                              the probe limit of 65,536 slots reports DBG_E_FULL.
                              A batched launch takes graphs of one setting only
                              (DBG_E_INVAL otherwise). */

typedef struct dbg_graph dbg_graph;

/*
 * Table sizing follows the paper's constructor, where the user gives the hash
 * table size (Methods, "Code organization").  capacity, when non-zero, is the
 * exact number of slots; otherwise capacity = ceil(expected_vertices /
 * load_factor).  With both zero the table is sized at the first build as
 * ceil(windows / load_factor): the number of windows bounds the number of
 * distinct vertices, so a direct table cannot run out of slots in that build
 * (if that first input is rejected, the next build sizes the table instead).
 *
 * A binned table (DBG_F_BINNED) is cut into segments of 2048 slots, and a key
 * can only take a slot of its own segment, so DBG_E_FULL comes when one
 * segment receives more than 2048 distinct vertices, not when the table is
 * full.  Keys reach segments through a bijective mix, so a segment's vertex
 * count is close to Poisson with mean 2048 x (vertices / capacity); the
 * chance that a given segment overflows is below 1e-22 at a load of 0.8 and
 * 3.6e-13 at 0.85 (so below 1e-6 for a table of a million segments, 49 GB),
 * but 1.3e-6 at 0.9 (one in two for a 25 GB table).  dbg_create therefore
 * refuses load_factor > 0.85 for binned graphs; a caller who passes capacity
 * or expected_vertices sets the load itself and should keep it there.
 */
#define DBG_BINNED_MAX_LOAD 0.85
typedef struct {
    uint64_t expected_vertices;  /* estimate of distinct (k-1)-mers; 0 = from input */
    uint64_t capacity;           /* exact slot count; 0 = derive as above */
    double load_factor;          /* in (0, 1); 0 = 0.5 */
    int32_t device;              /* HIP device ordinal; -1 = current device */
    uint32_t flags;              /* DBG_F_* */
    uint32_t block_size;         /* build kernel threads per block; 0 = 256 */
    uint32_t windows_per_thread; /* windows per thread per tile; 0 = 4 */
    void *stream;                /* hipStream_t for all work; NULL = own stream */
    /* binned build launch shape: the partition passes work on chunks of
     * consecutive tiles, about bin_chunks per resident scatter workgroup
     * (0 = 32; at most 16384 chunks a pass).  bin_shape1 and bin_shape2
     * set the shape of the first and second partition scatter: 1 = plain
     * tiles of 4096 records, stored as each tile sorts them (in runs of a
     * few records when there are many runs); 2 = staged: each run's
     * records wait in LDS until they fill a 128-byte line, and only whole
     * lines are stored; 3 = big tiles of 128 KB of records (16384, or
     * 8192 for k > 32; in the first scatter for k <= 31 up to 384 runs,
     * 8192 records in 64 KB), runs two to four times longer; 4 = big
     * tiles of 128 KB in every case; 0 = automatic (big tiles for the
     * second scatter, and for the first when k <= 31 or beyond 384 runs,
     * else plain tiles).  A shape whose LDS does not fit one workgroup
     * falls back to a smaller one.
     * bin_scatter_div divides the resident grid of a second scatter of
     * plain tiles (0 = automatic: 2 when a level-1 bucket spans more than
     * 384 table segments, else 1). */
    uint32_t bin_chunks;
    uint32_t bin_scatter_div;
    uint32_t bin_shape1;
    uint32_t bin_shape2;
} dbg_config;

typedef struct {
    uint64_t capacity;        /* table slots */
    uint64_t table_bytes;     /* device bytes held by the table */
    uint64_t vertices;        /* occupied slots (distinct (k-1)-mers) */
    uint64_t inserts;         /* k-mers counted so far: sum of max(0, L-k+1) */
    uint64_t windows;         /* windows seen so far: vertices looked up */
    uint64_t builds;          /* completed build calls */
    uint32_t k;               /* 0 until the first build */
    int32_t status;           /* DBG_OK, or the code that poisoned the handle */
    double last_build_ms;     /* build kernel time of the last build (DBG_F_TIMING) */
    double last_total_ms;     /* whole device pass of the last build (DBG_F_TIMING) */
    uint32_t block_size;      /* launch shape in use */
    uint32_t windows_per_thread;
    uint32_t grid_size;
    uint32_t entry_bytes;     /* 24 or 32 */
    uint64_t graph_captures;  /* build passes captured as graphs (DBG_F_GRAPH) */
    uint64_t graph_replays;   /* build passes replayed from a captured graph */
    uint32_t binned;          /* 1 if the graph uses the binned build */
    uint32_t pad;
    uint32_t bin_chunks;      /* binned launch shape in use (0 = defaults) */
    uint32_t bin_scatter_div;
    uint32_t bin_shape1;      /* scatter shapes of the last binned pass (as dbg_config; 0 before one) */
    uint32_t bin_shape2;
} dbg_stats;

/* Probe statistics of a graph created with DBG_F_STATS, summed over its
 * builds since creation or the last dbg_reset.  A lookup is the search for
 * one vertex's slot: in the global table for a direct graph (one per window,
 * or per merged group of windows with DBG_F_MERGE), in the LDS copy of a
 * table segment for a binned graph (one per window).  It examines slots one
 * after another (linear probing) until it finds its key or claims an empty
 * slot with a compare-and-swap; a compare-and-swap is lost when another
 * thread wrote the slot first (the paper's retry case of Algorithms 1 and 3).
 * For a build into an empty table, cas_attempts - cas_lost is the number of
 * vertices. */
typedef struct {
    uint64_t lookups;
    uint64_t probes;        /* slots examined by the lookups */
    uint64_t cas_attempts;  /* compare-and-swaps issued to claim a slot */
    uint64_t cas_lost;      /* of those, the ones another thread won first */
    uint64_t probe_hist[8]; /* lookups by slots examined: 1, 2, 3-4, 5-8, 9-16, 17-32, 33-64, more */
} dbg_probe_stats;

/* Fill *cfg with the defaults (all zero, device -1). */
void dbg_config_init(dbg_config *cfg);

/* Create a graph handle.  The table is allocated here when its size is known
 * (capacity or expected_vertices given), else at the first build.  On success
 * *out owns all device memory of the graph until dbg_destroy.
 * Errors: DBG_E_INVAL (NULL, load_factor outside (0,1), or above
 * DBG_BINNED_MAX_LOAD with DBG_F_BINNED), DBG_E_NOMEM, DBG_E_DEVICE. */
int dbg_create(const dbg_config *cfg, dbg_graph **out);

/* Add the k-mers of host-resident reads (makeGraph over all reads).  The
 * input is copied; the caller may free it on return.  Synchronous: returns
 * after the device work and the status readback.  Builds on one handle
 * accumulate (counts add), and all must use the same k.  2 <= k <= 64; the
 * first build with k > 32 re-allocates the table with 32-byte entries (two
 * key words); binned graphs stay binned up to k = 63, and direct builds of
 * long k do not merge within a wavefront.
 * Errors: DBG_E_INVAL (NULL pointers, decreasing offsets), DBG_E_K,
 * DBG_E_BASE, DBG_E_RANGE -- in all of these nothing was modified;
 * DBG_E_FULL (counts are partial, handle poisoned), DBG_E_NOMEM,
 * DBG_E_DEVICE. */
int dbg_build(dbg_graph *g, const char *reads, const uint64_t *offsets, uint64_t n_reads,
              uint32_t k);

/* Same, from device-resident input: d_reads holds reads_len bytes and
 * d_offsets n_reads + 1 entries, both device pointers that stay valid until
 * the work on `stream` has finished.  Offsets are taken relative to the first
 * one: read i is d_reads[d_offsets[i] - d_offsets[0] .. d_offsets[i+1] -
 * d_offsets[0]), and d_offsets[n_reads] - d_offsets[0] must equal reads_len
 * (so a slice of a larger concatenation can be passed as is).
 * Stream-ordered: the call enqueues the work and returns; device-side errors
 * (DBG_E_BASE, DBG_E_INVAL, DBG_E_RANGE, DBG_E_FULL) are reported by the next
 * dbg_sync.  As with dbg_build, a rejected input modifies nothing. */
int dbg_build_device(dbg_graph *g, const uint8_t *d_reads, uint64_t reads_len,
                     const uint64_t *d_offsets, uint64_t n_reads, uint32_t k, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * build as dbg_build_device (arguments, layout and result alike) with every
 * scratch buffer of the pass taken from a static device array of 256 MiB
 * that each device holds from its first call until the process ends, and no
 * allocation of any kind (device, pinned or library).  Limits: 2 <= k <= 32;
 * the graph's table must already exist (created with capacity or
 * expected_vertices, or sized by an earlier build), else DBG_E_INVAL; an
 * input whose pass needs more scratch than the array holds is refused with
 * DBG_E_SCRATCH before any device work (direct graphs take about 0.3 bytes
 * per read base, binned graphs about 16.3, so roughly 800 MB and 15 MB of
 * reads).  Synchronous: it returns after the build and its status readback,
 * with the codes of dbg_build.  Calls on one device share its array: the
 * library serialises them with a lock, so they never overlap on it; the array
 * keeps the last call's contents, and the pass rewrites all it reads. */
int dbg_build_device_static(dbg_graph *g, const uint8_t *d_reads, uint64_t reads_len, const uint64_t *d_offsets,
                            uint64_t n_reads, uint32_t k, void *stream);

/* dbg_build_device followed by dbg_extract_device, as one call: build from
 * device-resident input (arguments as dbg_build_device), then write every
 * vertex of the resulting graph to d_keys / d_counts (as dbg_extract_device:
 * cap entries, d_counts 16-byte aligned, unspecified order) and set
 * *n_vertices.  The graph is the paper's makeGraph result (Algorithms 2-4)
 * over all builds of the handle so far.  For a binned graph (k <= 31 or
 * 33 <= k <= 63) the output is written by the build's last kernel, while
 * each table segment is still on chip, instead of by a second pass over the
 * table; otherwise the call builds and then extracts.  Synchronous (it waits for the build's
 * status).  With d_keys == NULL only *n_vertices is set.  Errors: those of
 * dbg_build_device (reported here, not by dbg_sync) and DBG_E_SPACE when cap
 * is smaller than the vertex count: the graph is built, *n_vertices is set,
 * and the output holds an unspecified subset of the vertices. */
int dbg_build_extract_device(dbg_graph *g, const uint8_t *d_reads, uint64_t reads_len,
                             const uint64_t *d_offsets, uint64_t n_reads, uint32_t k, uint64_t *d_keys,
                             uint32_t *d_counts, uint64_t cap, uint64_t *n_vertices, void *stream);

/* Wait for the handle's outstanding work and return its status: DBG_OK or
 * the first error the device reported since the previous dbg_sync. */
int dbg_sync(dbg_graph *g);

/* Copy the graph out as records in unspecified order: keys[i] and
 * counts[4*i .. 4*i+3] for i < *n_vertices; for k > 32 the key of record i
 * is keys[2*i] (high word) and keys[2*i+1] (low word), and keys must hold
 * 2 * cap words.  With keys == NULL only
 * *n_vertices is set.  Synchronous.  Errors: DBG_E_SPACE when cap is smaller
 * than the vertex count (*n_vertices is still set, nothing is written),
 * DBG_E_INVAL, DBG_E_DEVICE.  Allowed on a poisoned handle (partial counts). */
int dbg_extract(dbg_graph *g, uint64_t *keys, uint32_t *counts, uint64_t cap,
                uint64_t *n_vertices);

/* Same into device buffers d_keys (cap entries, 2 * cap for k > 32) and d_counts (4 * cap,
 * 16-byte aligned: a vertex's four counters are stored with one 16-byte write),
 * stream-ordered up to the vertex count, which the call reads back
 * (synchronising on the stream). */
int dbg_extract_device(dbg_graph *g, uint64_t *d_keys, uint32_t *d_counts, uint64_t cap,
                       uint64_t *n_vertices, void *stream);

/* Empty the table (all vertices and counts), keeping its memory; clears a
 * poisoned state and the handle's k.  Stream-ordered. */
int dbg_reset(dbg_graph *g);

/* Counters and launch shape of the handle (synchronises first). */
int dbg_get_stats(dbg_graph *g, dbg_stats *out);

/* Device time of each phase of the handle's last timed build (DBG_F_TIMING),
 * in ms, in this order: setup (argument copy, prepare, pack, window scan),
 * then, for a binned build launched without a graph, ten phases -- plan,
 * pass-1 count, pass-1 scan, pass-1 scatter, pass-2 plan, pass-2 count,
 * pass-2 scan, pass-2 scatter, segment starts, segment reduce -- else the
 * whole build.  Writes min(cap, *n_phases) values; *n_phases is 0 before any
 * timed build. */
int dbg_get_phase_times(dbg_graph *g, double *ms, uint32_t cap, uint32_t *n_phases);

/* Probe statistics of the handle's builds (synchronises first).  All zero for
 * a graph created without DBG_F_STATS.  Errors: DBG_E_INVAL, DBG_E_DEVICE. */
int dbg_get_probe_stats(dbg_graph *g, dbg_probe_stats *out);

/* Release all device memory of the handle.  NULL is ignored. */
void dbg_destroy(dbg_graph *g);

/* Static description of a DBG_* code. */
const char *dbg_strerror(int code);

/* ---- batched build ---------------------------------------------------
 * Many independent read sets built in one persistent launch over per-graph
 * table segments.  Graph i takes the reads of inputs[i]; its k must match the
 * graph's k if set.  Each graph's result is exactly that of dbg_build on the
 * same reads.  Host-resident inputs are concatenated and copied once.
 * Synchronous; statuses[i] receives graph i's status (DBG_OK, DBG_E_BASE,
 * DBG_E_INVAL, DBG_E_K, DBG_E_RANGE, DBG_E_FULL).  The call's own return is
 * DBG_OK when every graph succeeded, else the first failing graph's code.
 * All graphs must be on the same device. */
typedef struct {
    const char *reads;
    const uint64_t *offsets;
    uint64_t n_reads;
    uint32_t k;
} dbg_input;

int dbg_build_batch(dbg_graph *const *graphs, const dbg_input *inputs, uint32_t m,
                    int32_t *statuses, void *stream);

/* Same from one device-resident concatenation: graph i takes reads
 * [read_begin[i], read_begin[i+1]) of d_reads/d_offsets (read j is
 * d_reads[d_offsets[j] - d_offsets[0] .. d_offsets[j+1] - d_offsets[0]),
 * d_offsets has read_begin[m] + 1 entries, d_offsets[read_begin[m]] -
 * d_offsets[0] == reads_len).  read_begin (m + 1 entries, read_begin[0] == 0)
 * and ks (m entries) are host arrays.  A graph that fails a host check keeps
 * its reads in the launch but they are skipped.  Synchronous. */
int dbg_build_batch_device(dbg_graph *const *graphs, uint32_t m, const uint64_t *read_begin,
                           const uint32_t *ks, const uint8_t *d_reads, uint64_t reads_len,
                           const uint64_t *d_offsets, int32_t *statuses, void *stream);

/* ---- normalization ----------------------------------------------------
 * Normalized counters (Methods, "Normalization of graph"): the paper divides
 * every counter by the number of times a k-mer of the genome is expected to
 * be read, reads * (read length - k + 1) / genome size.  Here the numerator
 * is the graph's total k-mer count (the same number for reads of one length,
 * and defined for any mix of lengths), so each counter c becomes
 * c * genome_size / total_kmers rounded half up, computed exactly in integer
 * arithmetic and saturated at 2^32 - 1.  genome_size = 0 leaves the counters
 * as they are.  With DBG_NORM_U8 the counters are written as uint8 saturated
 * at 255, the paper's 8-bit counter (counts then points to 4 * cap bytes).
 * Otherwise as dbg_extract: keys and counts in the same unspecified order. */
#define DBG_NORM_U8 0x1u

int dbg_extract_normalized(dbg_graph *g, uint64_t genome_size, uint32_t flags, uint64_t *keys, void *counts,
                           uint64_t cap, uint64_t *n_vertices);

/* ---- contigs ----------------------------------------------------------
 * Contigs of the graph (Methods, "Finding contigs", Algorithm 5): a vertex is
 * marked `first` when no k-mer ends in it (the paper clears the flag whenever
 * the vertex is added as a right vertex); a contig starts at every vertex that
 * is `first` or has more than one out-edge, once per out-edge, spells the
 * vertex and the letter of each edge it takes, and goes on while the vertex
 * it reaches has exactly one out-edge.  It stops on a vertex with zero or
 * several out-edges, or on a vertex it has already passed (loops of one-edge
 * vertices, which the paper's walk would follow forever); the vertex it stops
 * on is part of the contig.  Loops without a start vertex yield no contig.
 *
 * Output: ASCII contigs back to back in seq, contig i being
 * seq[offsets[i] .. offsets[i+1]); n_contigs + 1 offsets.  The set is unique;
 * the order is unspecified.  With seq and offsets NULL only *n_contigs and
 * *seq_len are set (the result is kept on the device until the next build or
 * reset, so a second call to fetch it does not recompute).  Errors:
 * DBG_E_INVAL, DBG_E_K (k > 32), DBG_E_STATE (graph poisoned), DBG_E_SPACE (a buffer is too
 * small; the sizes are set), DBG_E_NOMEM, DBG_E_DEVICE. */
int dbg_contigs(dbg_graph *g, char *seq, uint64_t seq_cap, uint64_t *offsets, uint64_t offsets_cap,
                uint64_t *n_contigs, uint64_t *seq_len);

/* The same into device buffers, ordered on `stream` (NULL: the handle's). */
int dbg_contigs_device(dbg_graph *g, uint8_t *d_seq, uint64_t seq_cap, uint64_t *d_offsets,
                       uint64_t offsets_cap, uint64_t *n_contigs, uint64_t *seq_len, void *stream);

/* ---- serving ----------------------------------------------------------
 * A build server: requests (read sets) are admitted first come, first served
 * while the table bytes of the admitted, unreleased requests stay within an
 * HBM budget; admitted requests are built by continuous batching -- every
 * pass of the server's worker thread takes the requests admitted since the
 * previous one, and up to `slots` passes run on separate streams at once, so
 * requests that arrive while others are on the GPU overlap with them.  Each
 * request's graph is built exactly as dbg_build would build it alone, and
 * stays resident on the device until the client releases it.
 * Thread safety: every dbg_server_* call may come from any client thread. */
#define DBG_PENDING 1 /* positive: the request has not finished yet */

typedef struct dbg_server dbg_server;

typedef struct {
    uint64_t hbm_budget;      /* table bytes admitted at once; 0 = 200 GB */
    uint64_t max_batch_bytes; /* read bytes per batched pass; 0 = 1 GiB */
    uint32_t max_batch;       /* requests per batched pass; 0 = 64 */
    uint32_t flags;           /* DBG_F_* of the request graphs; 0 = DBG_F_BINNED */
    double load_factor;       /* table sizing; 0 = 0.5 */
    int32_t device;           /* HIP device; -1 = current */
    uint32_t slots;           /* passes in flight at once (one stream each); 0 = 2 */
} dbg_server_config;

typedef struct {
    uint64_t submitted, admitted, completed, released, rejected;
    uint64_t queued;          /* waiting for admission */
    uint64_t running;         /* admitted, not completed */
    uint64_t resident_bytes;  /* table bytes of admitted, unreleased requests */
    uint64_t passes;          /* batched passes launched */
    uint64_t max_in_flight;   /* most passes on the device at once */
} dbg_server_stats;

/* Start a server and its worker thread.  Errors: DBG_E_INVAL, DBG_E_DEVICE. */
int dbg_server_create(const dbg_server_config *cfg, dbg_server **out);

/* Submit host-resident reads (copied; the caller may free them on return).
 * expected_vertices sizes the request's table as dbg_config does (0 = bound
 * from the input).  *id identifies the request.  Errors (nothing queued):
 * DBG_E_INVAL (NULL pointers, decreasing offsets), DBG_E_K, DBG_E_RANGE,
 * DBG_E_NOMEM (its table alone exceeds the budget). */
int dbg_server_submit(dbg_server *s, const char *reads, const uint64_t *offsets, uint64_t n_reads,
                      uint32_t k, uint64_t expected_vertices, uint64_t *id);

/* Submit device-resident reads (read i is d_reads[d_offsets[i] - d_offsets[0]
 * .. d_offsets[i+1] - d_offsets[0]), reads_len bytes).  The buffers must stay
 * valid and unchanged until the request has finished.  Errors as above;
 * offset consistency is checked on the device and reported as the request's
 * status. */
int dbg_server_submit_device(dbg_server *s, const uint8_t *d_reads, uint64_t reads_len,
                             const uint64_t *d_offsets, uint64_t n_reads, uint32_t k,
                             uint64_t expected_vertices, uint64_t *id);

/* DBG_PENDING while the request is queued or running; DBG_OK once finished,
 * with *status its build result (DBG_OK or a DBG_E_* code).  DBG_E_INVAL for
 * an unknown id. */
int dbg_server_poll(dbg_server *s, uint64_t id, int32_t *status);

/* Wait up to timeout_s seconds (negative: forever) for the request; returns
 * as dbg_server_poll. */
int dbg_server_wait(dbg_server *s, uint64_t id, double timeout_s, int32_t *status);

/* The finished request's graph (owned by the server until release): extract
 * it with dbg_extract / dbg_extract_device.  DBG_PENDING if not finished. */
int dbg_server_graph(dbg_server *s, uint64_t id, dbg_graph **g);

/* Seconds on the server's steady clock at which the request was submitted,
 * started on the device (its pass was enqueued) and finished. */
int dbg_server_times(dbg_server *s, uint64_t id, double *t_submit, double *t_start, double *t_done);

/* Free a finished request's graph, returning its bytes to the budget.
 * DBG_PENDING if it has not finished. */
int dbg_server_release(dbg_server *s, uint64_t id);

int dbg_server_get_stats(dbg_server *s, dbg_server_stats *out);

/* Finish every admitted request, drop queued ones, free everything. */
void dbg_server_destroy(dbg_server *s);

/* ---- autotuning -------------------------------------------------------
 * Picks the build configuration of a workload by timing complete builds of a
 * calibration input (the workload itself, or a slice of it that the caller
 * passes): the table mode (binned or direct) and the load factor; for the
 * binned build, the chunks per workgroup of its partition passes, the
 * shapes of its scatters, and the grid divisor of its second scatter; for
 * the direct build, block size,
 * windows per thread and wavefront merging.  The search goes one axis at a
 * time from the defaults.  Every candidate must produce the same vertex and
 * k-mer totals; one that does not, or that fails (a table overflow at a high
 * load factor), is discarded.  The graph itself never depends on the
 * choice: only the speed does (the GPU tests build the oracle's graph under
 * every configuration of dbg_autotune_space). */
typedef struct {
    double load_factor;
    uint32_t flags;              /* chosen DBG_F_BINNED / DBG_F_MERGE bits (others 0) */
    uint32_t block_size;         /* direct build launch shape (0 for binned) */
    uint32_t windows_per_thread;
    uint32_t candidates;         /* configurations timed (0 when served from a cache) */
    double best_ms;              /* median build time of the choice */
    double default_ms;           /* median build time of binned mode at load factor 0.5 */
    uint32_t from_cache;         /* 0: timed now; 1: this process's cache; 2: the cache file */
    uint32_t bin_chunks;         /* binned launch shape (dbg_config), 0 = default */
    uint32_t bin_scatter_div;
    uint32_t bin_shape1;
    uint32_t bin_shape2;
    uint32_t pad;
} dbg_tuning;

#define DBG_TUNE_FORCE 0x1u /* ignore the caches (and refresh them) */

/* Tune for m instances given as in dbg_build_batch_device (m = 1: a plain
 * build).  expected_vertices[i] sizes instance i's table as dbg_config does
 * (NULL or 0 = bound from the input).  keep_flags are DBG_F_* bits every
 * candidate keeps (DBG_F_GRAPH, DBG_F_ENTRY32, DBG_F_TIMING).  repeats timed
 * builds per candidate (0 = 3) after one warm-up.  Results are cached by
 * device model (architecture, compute units, memory), instance count, k
 * values, half-octave size classes of the input and flags: in the process,
 * and in a cache file that later processes read -- the path in the
 * environment variable DBG_TUNE_CACHE, else
 * $XDG_CACHE_HOME/libdbg/autotune.tsv or $HOME/.cache/libdbg/autotune.tsv
 * (DBG_TUNE_CACHE set but empty: no file).  Lines are appended, the last
 * line of a key wins.
 * k may exceed 32 (up to 64) only for m = 1; such a graph is tuned over the
 * direct build's launch shape and load factor.
 * Errors: DBG_E_INVAL, or the error of the default configuration's build. */
int dbg_autotune(int32_t device, uint32_t m, const uint64_t *read_begin, const uint32_t *ks,
                 const uint64_t *expected_vertices, const uint8_t *d_reads, uint64_t reads_len,
                 const uint64_t *d_offsets, uint32_t keep_flags, uint32_t repeats, uint32_t tune_flags,
                 dbg_tuning *out);

/* Every configuration the tuner's search may time, for the binned (binned
 * != 0) or the direct build: the cross product of its axes (load factor,
 * and binned chunks, scatter shapes (five pairs) and scatter divisor, or
 * direct block size, windows per thread and merging).  Writes min(cap, *n) entries (only the configuration
 * fields are set); *n is the size of the space. */
int dbg_autotune_space(uint32_t binned, dbg_tuning *out, uint32_t cap, uint32_t *n);

/* Copy a tuning into a configuration (load factor, launch shapes, mode and
 * merge bits; the configuration's other fields are left as they are). */
void dbg_config_apply_tuning(dbg_config *cfg, const dbg_tuning *t);

/* ---- measurement -----------------------------------------------------
 * Random-access roofline of the device: n_ops operations at indices drawn by
 * a 64-bit mixer over a footprint of footprint_bytes (no index array is
 * read).  kind: 0 = 64-bit load, 1 = 32-bit atomic add (no return),
 * 2 = 64-bit atomic compare-and-swap (returning), 3 = 64-bit load then a
 * 32-bit atomic add into the same 24-byte entry, 4 = streaming copy of the
 * first half of the footprint onto the second with 16-byte loads and stores
 * (n_ops ignored; a copy of known size for scaling traffic counters).
 * Returns the median kernel
 * time over `repeats` timed launches (after one warm-up) in *ms.  Allocates
 * and frees its own footprint. */
int dbg_atomic_roofline(int32_t device, uint32_t kind, uint64_t footprint_bytes, uint64_t n_ops,
                        uint32_t block_size, uint32_t repeats, double *ms);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* DBG_H */
