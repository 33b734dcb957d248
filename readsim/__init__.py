"""Seeded synthetic genomes and sequencing reads.

This module only draws random data: a genome over {A,C,G,T}, optional repeat
copies written into it, reads sampled from its forward strand and independent
per-base substitution errors.  It holds none of the graph-building arithmetic
(no letter codes, no packing, no k-mer windows), so both the CPU oracle and
the GPU path may take their inputs from it.

Read sets are returned in the boundary's input form: one ``uint8`` array of
ASCII bases with all reads concatenated, and ``uint64`` offsets of length
``n_reads + 1`` (read ``i`` is ``reads[offsets[i]:offsets[i+1]]``).

The paper evaluates on E. coli, yeast and human chromosome 1 reads sampled at
10-50x coverage with k = 31 (Results, "Data preparation") and with 1-10 %
read errors (Results, "The impact of read errors").  Those datasets are not
available here; the recipes below stand in for them with the same shape:
uniform random start positions on the forward strand, a fixed read length,
a coverage target and uniform substitutions.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "ReadSet",
    "config_seed",
    "instance_seed",
    "random_genome",
    "place_repeats",
    "sample_reads",
    "simulate",
    "make_config",
    "instance_params",
    "make_instance",
    "reads_from_strings",
    "CONFIG_NAMES",
]

_ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)

# Reads are drawn in fixed-size chunks so that a seed gives the same bytes
# regardless of the total size requested.
_CHUNK_READS = 1 << 16

CONFIG_NAMES = {
    1: "tiny: 10 kbp genome, 100 bp reads, 10x, 0.5% subs, k=21",
    2: "bacterial: 5 Mbp genome + 50 x 1 kbp repeat copies, 150 bp reads, 30x, 1% subs, k=31",
    3: "large: 100 Mbp genome, 2% in 300-5000 bp repeats, 150 bp reads, 20x, 1% subs, k=31",
    4: "batched: 256 read sets, genome logU[10 kbp, 2 Mbp], cov U[10,50], L in {100,150}, "
       "subs U[0.5,1]%, k in {21,31}",
    5: "served: Poisson stream of read sets drawn as the batched ones with genomes up to 20 Mbp",
}


def config_seed(i: int) -> int:
    """Seed of workload configuration ``i`` (1-based)."""
    return 0x5EED0000 + int(i)


def instance_seed(i: int, j: int) -> int:
    """Seed of instance (or request) ``j`` of configuration ``i``."""
    return config_seed(i) * 1000003 + int(j)


@dataclasses.dataclass
class ReadSet:
    reads: np.ndarray              # uint8 ASCII, all reads concatenated
    offsets: np.ndarray            # uint64, n_reads + 1
    k: int                         # graph dimension used for this workload
    starts: np.ndarray | None = None   # int64 genome start of each read
    genome: np.ndarray | None = None   # uint8 ASCII genome (kept when asked)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def total_bases(self) -> int:
        return int(self.offsets[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))

    def read(self, i: int) -> bytes:
        return self.reads[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()


def random_genome(rng: np.random.Generator, length: int) -> np.ndarray:
    """iid uniform genome as indices 0..3 (A, C, G, T in that order)."""
    return rng.integers(0, 4, size=int(length), dtype=np.uint8)


def place_repeats(rng: np.random.Generator, genome: np.ndarray,
                  copies: list[tuple[int, int]]) -> list[tuple[int, int]]:
    """Write repeat copies over random non-overlapping positions.

    ``copies`` is a list of (unit_id, unit_length); every copy of one unit
    holds the same random bases.  Positions are uniform among all
    non-overlapping placements: sorted uniform cut points in the free length,
    shifted by the lengths of the copies placed before them.  The genome length
    does not change.  Returns (position, length) of each copy.
    """
    if not copies:
        return []
    units: dict[int, np.ndarray] = {}
    for uid, ulen in copies:
        if uid not in units:
            units[uid] = rng.integers(0, 4, size=int(ulen), dtype=np.uint8)
    total = sum(ulen for _, ulen in copies)
    free = genome.shape[0] - total
    if free < 0:
        raise ValueError("repeat copies longer than the genome")
    order = rng.permutation(len(copies))
    cuts = np.sort(rng.integers(0, free + 1, size=len(copies)))
    placed = []
    shift = 0
    for cut, ci in zip(cuts, order):
        uid, ulen = copies[ci]
        pos = int(cut) + shift
        genome[pos:pos + ulen] = units[uid]
        placed.append((pos, int(ulen)))
        shift += ulen
    return placed


def sample_reads(rng: np.random.Generator, genome: np.ndarray, read_len: int,
                 n_reads: int, err: float) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Sample reads uniformly from the forward strand with substitutions.

    Start positions are uniform in [0, G - L].  Each base is independently
    replaced, with probability ``err``, by one of the other three bases chosen
    uniformly.  Returns (ASCII reads, uint64 offsets, int64 starts).
    """
    G = int(genome.shape[0])
    L = int(read_len)
    n = int(n_reads)
    if L > G:
        raise ValueError("read length exceeds genome length")
    starts = np.empty(n, dtype=np.int64)
    out = np.empty(n * L, dtype=np.uint8)
    col = np.arange(L, dtype=np.int64)
    for c0 in range(0, n, _CHUNK_READS):
        m = min(_CHUNK_READS, n - c0)
        s = rng.integers(0, G - L + 1, size=m, dtype=np.int64)
        starts[c0:c0 + m] = s
        block = genome[s[:, None] + col[None, :]]
        if err > 0.0:
            hit = rng.random((m, L), dtype=np.float32) < np.float32(err)
            nh = int(np.count_nonzero(hit))
            if nh:
                delta = rng.integers(1, 4, size=nh, dtype=np.uint8)
                block[hit] = (block[hit] + delta) & np.uint8(3)
        out[c0 * L:(c0 + m) * L] = _ALPHABET[block].reshape(-1)
    offsets = np.arange(n + 1, dtype=np.uint64) * np.uint64(L)
    return out, offsets, starts


def simulate(genome_len: int, read_len: int, coverage: float, err: float, k: int,
             seed: int, repeats: list[tuple[int, int]] | None = None,
             keep_genome: bool = False, n_reads: int | None = None) -> ReadSet:
    """One read set: genome, repeats, reads.  ``n = round(G * cov / L)``."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    genome = random_genome(rng, genome_len)
    placed = place_repeats(rng, genome, repeats or [])
    n = int(round(genome_len * coverage / read_len)) if n_reads is None else int(n_reads)
    reads, offsets, starts = sample_reads(rng, genome, read_len, n, err)
    meta = dict(genome_len=int(genome_len), read_len=int(read_len), coverage=float(coverage),
                err=float(err), seed=int(seed), n_reads=n, repeat_copies=len(placed),
                repeat_bases=int(sum(l for _, l in placed)))
    return ReadSet(reads=reads, offsets=offsets, k=int(k), starts=starts,
                   genome=_ALPHABET[genome] if keep_genome else None, meta=meta)


def _c3_repeats(rng: np.random.Generator, genome_len: int) -> list[tuple[int, int]]:
    """Repeat families for the large workload: unit length U[300, 5000],
    2-10 copies each, added until the copies cover 2 % of the genome."""
    target = int(0.02 * genome_len)
    copies: list[tuple[int, int]] = []
    covered = 0
    uid = 0
    while True:
        ulen = int(rng.integers(300, 5001))
        nc = int(rng.integers(2, 11))
        if covered + ulen * nc > target:
            nc = (target - covered) // ulen
            if nc < 2:
                break
        copies.extend([(uid, ulen)] * nc)
        covered += ulen * nc
        uid += 1
    return copies


def expected_vertices(genome_len: int, read_len: int, n_reads: int, err: float, k: int) -> int:
    """Sizing estimate of distinct (k-1)-mers: genome positions plus the
    windows that contain at least one substitution.  This is the "table size"
    a user supplies (Code organization: the user provides the hash table size);
    it is an estimate, not a bound."""
    w = max(0, read_len - k + 2)
    p_err_free = (1.0 - err) ** (k - 1)
    return int(genome_len + n_reads * w * (1.0 - p_err_free))


def make_config(i: int, keep_genome: bool = False, scale: float = 1.0) -> ReadSet:
    """Workload configuration ``i`` in {1, 2, 3} as one read set.

    ``scale`` shrinks the genome (and so the read count) for quick tests; the
    full workload is ``scale=1``.
    """
    seed = config_seed(i)
    if i == 1:
        G, L, cov, err, k, reps = 10_000, 100, 10.0, 0.005, 21, None
    elif i == 2:
        G, L, cov, err, k = 5_000_000, 150, 30.0, 0.01, 31
        reps = [(0, 1000)] * 50
    elif i == 3:
        G, L, cov, err, k = 100_000_000, 150, 20.0, 0.01, 31
        reps = "c3"
    else:
        raise ValueError("configs 4 and 5 are sets of instances: use make_instance")
    G = max(L, int(G * scale))
    if reps == "c3":
        rng0 = np.random.Generator(np.random.PCG64(seed ^ 0xC3C3))
        reps = _c3_repeats(rng0, G)
    elif reps is not None and scale != 1.0:
        reps = reps[:max(0, min(len(reps), int(len(reps) * scale)))]
    rs = simulate(G, L, cov, err, k, seed, repeats=reps, keep_genome=keep_genome)
    rs.meta["config"] = i
    rs.meta["name"] = CONFIG_NAMES[i]
    rs.meta["expected_vertices"] = expected_vertices(G, L, rs.n_reads, err, k)
    return rs


def instance_params(i: int, j: int) -> dict:
    """Parameters of instance ``j`` of the batched (i=4) or served (i=5) workload."""
    if i not in (4, 5):
        raise ValueError("instances exist for configurations 4 and 5")
    rng = np.random.Generator(np.random.PCG64(instance_seed(i, j)))
    gmax = 2_000_000 if i == 4 else 20_000_000
    G = int(round(math.exp(rng.uniform(math.log(10_000), math.log(gmax)))))
    cov = float(rng.uniform(10.0, 50.0))
    L = int(rng.choice([100, 150]))
    err = float(rng.uniform(0.005, 0.01))
    k = int(rng.choice([21, 31]))
    n = int(round(G * cov / L))
    return dict(genome_len=G, coverage=cov, read_len=L, err=err, k=k, n_reads=n,
                seed=instance_seed(i, j) ^ 0xA5A5A5A5,
                inserts=n * max(0, L - k + 1),
                expected_vertices=expected_vertices(G, L, n, err, k))


def make_instance(i: int, j: int, keep_genome: bool = False) -> ReadSet:
    p = instance_params(i, j)
    rs = simulate(p["genome_len"], p["read_len"], p["coverage"], p["err"], p["k"], p["seed"],
                  keep_genome=keep_genome, n_reads=p["n_reads"])
    rs.meta.update(config=i, instance=j, expected_vertices=p["expected_vertices"])
    return rs


def reads_from_strings(reads: list[str] | list[bytes], k: int) -> ReadSet:
    """Pack literal reads into the boundary's input form."""
    bs = [r.encode() if isinstance(r, str) else bytes(r) for r in reads]
    lens = np.array([len(b) for b in bs], dtype=np.uint64)
    offsets = np.zeros(len(bs) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    data = np.frombuffer(b"".join(bs), dtype=np.uint8).copy() if bs else np.zeros(0, np.uint8)
    return ReadSet(reads=data, offsets=offsets, k=int(k))
