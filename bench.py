"""Benchmark of the A-Bruijn graph build on one MI355X.

One step is one pass of the whole plain-build path over the large workload
(100 Mbp genome with 2 % of its length in repeat copies of 300-5000 bp units,
150 bp reads at 20x = 13,333,333 reads, 1 % substitutions, k = 31; binned
table at load factor 0.5: 1.04 G slots, 25 GB), with the ASCII reads and
offsets already resident in HBM:

    table reset -> pack -> window scan -> build (records partitioned by table
    segment, find-or-claim + count in LDS) -> every vertex written to device
    buffers -> status readback

(one dbg_build_extract_device call: in binned mode the build's reduce kernel
writes the vertices while each table segment is on chip), and the metric is
k-mer inserts per second, inserts = sum over reads of max(0, L - k + 1) =
1,599,999,960 per step.

Besides the driver's JSON fields the line carries:
  * phases         -- device time and algorithmic bytes of every kernel group
                      of the step, from an uncaptured timed pass with HIP
                      events between the kernels;
  * roofline       -- the longest kernel against HBM peak (its algorithmic
                      bytes per launch over its event time), its HBM traffic
                      from the committed counter profile, and under "step"
                      the whole step against HBM peak with the byte model of
                      the hot-path scope table (per k-mer an 8-byte key probe,
                      a 4-byte counter add and the packed read; per table slot
                      24 bytes initialised and 24 read by the extraction; per
                      vertex 24 bytes written);
  * atomic_roofline-- measured random-access rates (64-bit compare-and-swap,
                      32-bit add, ...) at the table's footprint and op count,
                      the bound of the direct design, with the step against
                      them;
  * bacterial      -- the bacterial-scale workload (5 Mbp + 50 copies of a
                      1 kbp repeat, 1,000,000 reads, k = 31) at the
                      autotuner's configuration, with its own phases and
                      roofline, the direct-mode step, long k, contigs and
                      host input;
  * batched, served-- 256 read sets in one pass; a Poisson request stream;
  * cpu_baseline   -- the CPU oracle on a bounded sample of the step's reads.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(n_reads: int, total_bases: int, windows: int, inserts: int,
                      vertices_new: int) -> int:
    """Bytes the direct build kernel must move per launch, by its algorithm:
    one 8-byte key read per window looked up, one 4-byte counter read and
    written per k-mer, one 8-byte key written per vertex claimed, the packed
    reads (2 bits per base) and, per read, its offset and window prefix."""
    return (8 * windows + 8 * inserts + 8 * vertices_new + total_bases // 4 + 16 * n_reads)


def code_digest(paths: list) -> str:
    """SHA-256 of C/C++ sources with comments, blank lines and surrounding
    whitespace removed: it changes when the code changes, not its comments."""
    import hashlib
    import re

    h = hashlib.sha256()
    for p in paths:
        text = open(p, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.strip() for ln in text.splitlines() if ln.strip()]
        h.update(("\n".join(lines) + "\n").encode())
    return h.hexdigest()


def committed_traffic(profile: str, workload: dict, kernel: str) -> int | None:
    """HBM bytes per launch of `kernel` recorded by the counter runs in
    `profile` (a line "traffic_bytes_per_launch[<kernel>]: N"), or None when
    the profile does not exist, the code of its kernel sources changed since
    the counters were taken (code_digest), or the run's workload parameters
    (`workload`, e.g. load factor and mode) differ from the ones recorded
    there."""

    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    srcs = fields.get("sources", "").split()
    if not srcs or code_digest([os.path.join(ROOT, s) for s in srcs]) != fields.get("code_sha256"):
        return None
    for k, v in workload.items():
        if fields.get(k) != str(v):
            return None
    v = fields.get("traffic_bytes_per_launch[%s]" % kernel)
    return int(v) if v else None


def binned_kernel_bytes(n_reads: int, total_bases: int, windows: int, vertices: int, fused: bool) -> dict:
    """Algorithmic bytes of each kernel group of a binned build of one-word
    records into an empty table (8-byte window records, 24-byte vertex
    entries); None where the work is bookkeeping of a size the host does not
    know (plans, histogram scans, segment starts):
      setup     ASCII in, packed reads out, offsets in, window prefix out;
      count1    packed reads and each read's offset and window start read;
      scatter1  the same, and every window's record written;
      count2    records read;
      scatter2  records read and written;
      reduce    records read, packed vertex entries written and, with the
                fused extraction, every vertex's key and counters written."""
    packed = total_bases // 4 + 16 * n_reads
    return {"setup": total_bases + total_bases // 4 + 24 * n_reads, "plan": None, "count1": packed,
            "scan1": None, "scatter1": packed + 8 * windows, "plan2": None, "count2": 8 * windows,
            "scan2": None, "scatter2": 16 * windows, "starts": None,
            "reduce": 8 * windows + 24 * vertices * (2 if fused else 1)}


def scope_step_bytes(inserts: int, total_bases: int, capacity: int, vertices: int) -> int:
    """Bytes of one step under the hot-path scope table's model of the build:
    per k-mer an 8-byte key probe and a 4-byte counter add, the packed reads
    (2 bits a base), 24 bytes per table slot initialised and 24 read by the
    extraction, 24 bytes per vertex written."""
    return 12 * inserts + total_bases // 4 + 48 * capacity + 24 * vertices


def batched_bench(dbg, torch, dev, n_inst: int, reps: int, graphs_on: bool) -> dict:
    """256 independent read sets (genomes log-uniform in [10 kbp, 2 Mbp],
    coverage U[10, 50], L in {100, 150}, substitutions U[0.5, 1] %, k in
    {21, 31}) built (a) in one batched call over one device-resident
    concatenation and (b) one plain build per set on slices of the same
    buffers, into the same per-set tables.  Aggregate k-mer inserts/s of each,
    with build passes only (tables reset lazily between repetitions)."""
    import concurrent.futures
    import readsim

    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        sets = list(ex.map(lambda j: readsim.make_instance(4, j), range(n_inst)))
    gen_s = time.perf_counter() - t0
    lens = np.concatenate([x.lengths() for x in sets])
    offs = np.zeros(lens.shape[0] + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    rb = np.zeros(n_inst + 1, np.uint64)
    np.cumsum([x.n_reads for x in sets], out=rb[1:])
    ks = [x.k for x in sets]
    inserts = int(sum(int(np.maximum(x.lengths() - x.k + 1, 0).sum()) for x in sets))
    d_reads = torch.from_numpy(np.concatenate([x.reads for x in sets])).to(dev)
    d_off = torch.from_numpy(offs).to(dev)
    del sets
    keep = dbg.F_GRAPH if graphs_on else 0
    ev = [readsim.instance_params(4, j)["expected_vertices"] for j in range(n_inst)]
    t1 = time.perf_counter()
    tune = dbg.autotune(rb, ks, d_reads, d_off, ev, keep_flags=keep, force=True)
    tune_s = time.perf_counter() - t1
    kw = tune.graph_kwargs()
    kw["flags"] |= keep
    gs = [dbg.Graph(expected_vertices=e, device=0, **kw) for e in ev]

    def batched():
        for g in gs:
            g.reset()
        st = dbg.build_batch_device(gs, rb, ks, d_reads, d_off)
        assert st == [0] * n_inst, st

    def plain():
        for j, g in enumerate(gs):
            g.reset()
            a, z = int(rb[j]), int(rb[j + 1])
            g.build_device(d_reads[int(offs[a]):int(offs[z])], d_off[a:z + 1], ks[j])
            g.sync()

    out = {"workload": "batched: %d read sets, %d k-mer inserts, %.2f Gbp" % (n_inst, inserts, offs[-1] / 1e9),
           "generation_s": round(gen_s, 1),
           "autotune": dict(tune.as_dict(), seconds=round(tune_s, 2))}
    for name, fn in (("batched", batched), ("plain_per_instance", plain)):
        fn()  # warm-up (allocates scratch, captures graphs)
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t1 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t1)
        best = float(np.median(t))
        out[name] = {"ms": round(best * 1e3, 3), "ginserts_s": round(inserts / best / 1e9, 4)}
    vb = sum(g.vertex_count() for g in gs)
    out["vertices"] = vb
    out["batched_over_plain"] = round(out["batched"]["ginserts_s"] / out["plain_per_instance"]["ginserts_s"], 3)
    for g in gs:
        g.close()
    return out


def served_bench(dbg, torch, dev, n_payloads: int, n_requests: int, loads, ref_gips: float,
                 budget: int = 200_000_000_000) -> dict:
    """Serving: a pool of n_payloads device-resident read sets of the served
    workload (genomes log-uniform in [10 kbp, 20 Mbp], coverage U[10, 50], L
    in {100, 150}, substitutions U[0.5, 1] %, k in {21, 31}); n_requests
    requests, each carrying a seeded random payload of the pool, arrive as a
    Poisson process whose insert rate is `load` x ref_gips; tables are
    admitted against `budget` bytes of HBM; a client thread releases each
    request when it finishes.  Latency = finish - arrival on the server's
    clock; aggregate rate = inserts of all requests / (last finish - first
    arrival)."""
    import concurrent.futures
    import threading
    import readsim

    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        pool = list(ex.map(lambda j: readsim.make_instance(5, j), range(n_payloads)))
    gen_s = time.perf_counter() - t0
    pay = []
    for rs in pool:
        pay.append(dict(d_reads=torch.from_numpy(rs.reads).to(dev),
                        d_off=torch.from_numpy(rs.offsets.astype(np.int64)).to(dev),
                        k=rs.k, ev=rs.meta["expected_vertices"],
                        inserts=int(np.maximum(rs.lengths() - rs.k + 1, 0).sum())))
    del pool
    rng = np.random.default_rng(0x5E4E)
    choice = rng.integers(0, n_payloads, n_requests)
    ins = np.array([pay[c]["inserts"] for c in choice], dtype=np.float64)
    out = {"workload": "served: %d requests, each carrying one of a pool of %d read sets drawn as the served "
                       "workload states (a fresh read set per request would take about 100 GB of reads), "
                       "%.1f M k-mer inserts per request (mean), %.0f GB table budget"
                       % (n_requests, n_payloads, ins.mean() / 1e6, budget / 1e9),
           "generation_s": round(gen_s, 1), "reference_ginserts_s": round(ref_gips, 3), "runs": []}

    srv = dbg.Server(hbm_budget=budget, flags=dbg.F_BINNED)
    # warm-up: every payload once (scratch sized, tables pooled); its vertex
    # count is what every later request with that payload must reproduce
    ids = [srv.submit_device(p["d_reads"], p["d_off"], p["k"], p["ev"]) for p in pay]
    want_v = []
    for rid in ids:
        assert srv.wait(rid) == dbg.OK
        want_v.append(srv.graph(rid).vertex_count())
        srv.release(rid)
    for load in loads:
        rate = load * ref_gips * 1e9 / ins.mean()  # requests per second
        arrive = np.cumsum(rng.exponential(1.0 / rate, n_requests))
        s0 = srv.stats()
        rids = [None] * n_requests
        got = threading.Semaphore(0)
        lat, first_t, last_t, bad = [], [float("inf")], [0.0], []

        def reaper():
            for i in range(n_requests):
                got.acquire()
                rid = rids[i]
                st = srv.wait(rid)
                ts, _, td = srv.times(rid)
                if st != dbg.OK or srv.graph(rid).vertex_count() != want_v[choice[i]]:
                    bad.append((i, st))
                srv.release(rid)
                lat.append(td - ts)
                first_t[0] = min(first_t[0], ts)
                last_t[0] = max(last_t[0], td)

        th = threading.Thread(target=reaper)
        th.start()
        t_start = time.perf_counter()
        for i in range(n_requests):
            wait_s = t_start + arrive[i] - time.perf_counter()
            if wait_s > 0:
                time.sleep(wait_s)
            p = pay[choice[i]]
            rids[i] = srv.submit_device(p["d_reads"], p["d_off"], p["k"], p["ev"])
            got.release()
        th.join()
        s1 = srv.stats()
        assert not bad, bad[:5]
        lat_ms = np.array(lat) * 1e3
        span = last_t[0] - first_t[0]
        passes = s1["passes"] - s0["passes"]
        run = {"load": load, "offered_requests_s": round(rate, 1),
               "offered_ginserts_s": round(load * ref_gips, 3),
               "achieved_ginserts_s": round(ins.sum() / span / 1e9, 3),
               "p50_ms": round(float(np.percentile(lat_ms, 50)), 2),
               "p99_ms": round(float(np.percentile(lat_ms, 99)), 2),
               "mean_ms": round(float(lat_ms.mean()), 2), "max_ms": round(float(lat_ms.max()), 2),
               "passes": passes, "mean_batch": round(n_requests / max(passes, 1), 2),
               "max_in_flight": s1["max_in_flight"], "span_s": round(span, 3)}
        out["runs"].append(run)
        log("served load %.2f: %s" % (load, json.dumps(run)))
    srv.close()
    return out


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rs, sample_reads: int) -> dict:
    import oracle

    n = min(sample_reads, rs.n_reads)
    end = int(rs.offsets[n])
    reads = rs.reads[:end]
    offs = rs.offsets[:n + 1]
    t0 = time.perf_counter()
    keys, counts = oracle.build_graph(reads, offs, rs.k)
    dt = time.perf_counter() - t0
    ins = int(counts.sum())
    out = {"value": ins / dt / 1e9, "unit": "G k-mer inserts/s", "cores": 1, "kind": "oracle",
           "sample": "first %d of %d reads (%d k-mer inserts, %d vertices), single-threaded C "
                     "oracle, %.1f s" % (n, rs.n_reads, ins, keys.shape[0], dt),
           "host_cpu": host_cpu(), "host_threads": os.cpu_count()}
    # the oracle's key-partitioned mode on the host's cores (each partition
    # scans every read, so it scales with threads but not perfectly)
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    pk, pc = oracle.build_graph_parallel(reads, offs, rs.k, threads=threads)
    dtp = time.perf_counter() - t0
    assert pk.shape[0] == keys.shape[0]
    out["parallel"] = {"value": ins / dtp / 1e9, "cores": threads, "seconds": round(dtp, 2)}
    return out


def cpu_lfdbg_scaling(rs, sample_reads: int) -> dict:
    """The paper's own design (chained buckets, CAS on list heads, per-thread
    node pools, two find-or-adds per k-mer) on the host's CPU threads, on the
    same sample as the oracle baseline: the thread-scaling context the paper's
    missing figures held."""
    import oracle

    n = min(sample_reads, rs.n_reads)
    reads = rs.reads[:int(rs.offsets[n])]
    offs = rs.offsets[:n + 1]
    ins = int(np.maximum(np.diff(offs.astype(np.int64)) - rs.k + 1, 0).sum())
    out = {"kind": "paper design on CPU threads (oracle/lfdbg_cpu.cpp)", "unit": "G k-mer inserts/s",
           "sample": "first %d reads (%d k-mer inserts), table of one bucket per window" % (n, ins),
           "host_cpu": host_cpu(), "rates": {}}
    t = 1
    while t <= min(16, os.cpu_count() or 1):
        _, _, sec = oracle.lfdbg_build(reads, offs, rs.k, t)
        out["rates"][str(t)] = round(ins / sec / 1e9, 5)
        t *= 2
    return out


def measure_step(dbg, torch, dev, rs, inserts: int, mode: str, lf: float, steps: int, warmup: int,
                 graphs: bool, block: int = 0, wpt: int = 0, merge: bool = False, shape: dict | None = None) -> dict:
    """Steps of reset + dbg_build_extract_device (the whole path, every vertex
    written to device buffers, status read back) on device-resident reads;
    host wall time over the timed steps."""
    flags = dbg.F_TIMING | (dbg.F_MERGE if merge else 0) | (dbg.F_BINNED if mode == "binned" else 0)
    if graphs:
        flags |= dbg.F_GRAPH
    d_reads, d_off = rs.d_reads, rs.d_off
    g = dbg.Graph(expected_vertices=rs.meta["expected_vertices"], load_factor=lf, device=0, flags=flags,
                  block_size=block, windows_per_thread=wpt, **(shape or {}))
    cap_out = int(g.stats()["capacity"])
    d_keys = torch.empty(cap_out, dtype=torch.int64, device=dev)
    d_counts = torch.empty((cap_out, 4), dtype=torch.int32, device=dev)

    def step():
        g.reset()
        return g.build_extract_device(d_reads, d_off, rs.k, d_keys, d_counts)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    build_ms, phases = [], []
    V = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        V = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s = g.stats()
    build_ms = s["last_build_ms"]
    phases = g.phase_times()
    tx = []
    for _ in range(3):  # extraction alone, host-timed around the synchronous call
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.extract_device(d_keys, d_counts)
        tx.append((time.perf_counter() - t1) * 1000.0)
    st = g.stats()
    assert st["inserts"] == inserts, (st["inserts"], inserts)
    g.close()
    del d_keys, d_counts
    torch.cuda.empty_cache()
    return dict(V=V, cap=cap_out, st=st, ms_step=dt * 1000.0 / steps, value=inserts / (dt / steps) / 1e9,
                kern_ms=build_ms, phases=phases, extract_ms=float(np.median(tx)))


def kernel_roofline(dbg, rs, windows: int, inserts: int, V: int, cap: int, ms_step: float, phases: list,
                    mode: str, lf: float, entry_bytes: int, workload: str, profile: str) -> tuple:
    """Per-kernel phase table, and the roofline of the longest kernel group
    (plus the whole step under the scope table's byte model)."""
    table = []
    if mode == "binned":
        kb = binned_kernel_bytes(rs.n_reads, rs.total_bases, windows, V, True)
        for name, ms in zip(dbg.BINNED_PHASES, phases):
            b = kb[name]
            table.append({"phase": name, "ms": round(ms, 4), "algorithmic_bytes": b,
                          "gbs": round(b / (ms * 1e-3) / 1e9, 1) if b and ms > 0 else None})
        cand = [p for p in table if p["algorithmic_bytes"] and p["phase"] != "setup"]
        dom = max(cand, key=lambda p: p["ms"])
        kernels = {"count1": "k_bin<false> (pass-1 count)", "scatter1": "k_bin<true> (pass-1 scatter)",
                   "count2": "k_refine<false> (pass-2 count)", "scatter2": "k_refine<true> (pass-2 scatter)",
                   "reduce": "k_reduce (segment reduce with the fused extraction)"}
        kname, k_ms, bytes_alg = kernels[dom["phase"]], dom["ms"], dom["algorithmic_bytes"]
        short = {"count1": "k_bin_count", "scatter1": "k_bin_scatter", "count2": "k_refine_count",
                 "scatter2": "k_refine_scatter", "reduce": "k_reduce"}[dom["phase"]]
    else:
        bytes_alg = algorithmic_bytes(rs.n_reads, rs.total_bases, windows, inserts, V)
        k_ms = phases[-1] if phases else 0.0
        kname, short = "k_build (direct find-or-claim + count)", "k_build"
    traffic = committed_traffic(profile, {"workload": workload, "load_factor": lf, "mode": mode,
                                          "entry_bytes": entry_bytes}, short)
    achieved = bytes_alg / (k_ms * 1e-3) / 1e9
    step_bytes = scope_step_bytes(inserts, rs.total_bases, cap, V)
    step_gbs = step_bytes / (ms_step * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
            "kernel_ms": round(k_ms, 4), "algorithmic_bytes": bytes_alg,
            "step": {"algorithmic_bytes": step_bytes, "ms": round(ms_step, 4), "achieved": round(step_gbs, 1),
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                     "model": "12 B per k-mer + packed reads + 48 B per table slot + 24 B per vertex"}}
    return table, roof


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3],
                    help="workload of the headline step (3: large, the default)")
    ap.add_argument("--load-factor", type=float, default=0.5, help="headline table load factor")
    ap.add_argument("--mode", choices=["direct", "binned"], default="binned")
    ap.add_argument("--tune", action="store_true", help="autotune the headline workload too")
    ap.add_argument("--bin-chunks", type=int, default=0, help="headline binned launch shape: chunks per workgroup")
    ap.add_argument("--bin-div", type=int, default=0, help="headline binned launch shape: pass-2 scatter grid divisor")
    ap.add_argument("--bin-shape1", type=int, default=0, help="headline binned launch shape: first scatter shape "
                    "(0 automatic, 1 plain tiles, 2 staged lines, 3 big tiles)")
    ap.add_argument("--bin-shape2", type=int, default=0, help="headline binned launch shape: second scatter shape")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels without HIP graphs")
    ap.add_argument("--no-compare", action="store_true", help="skip the direct-mode comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--cpu-sample-reads", type=int, default=250_000)
    ap.add_argument("--no-bacterial", action="store_true", help="skip the bacterial-scale leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-build comparison")
    ap.add_argument("--batched-sets", type=int, default=256)
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--no-served", action="store_true", help="skip the serving benchmark")
    ap.add_argument("--no-long-k", action="store_true", help="skip the k = 51 build of the bacterial reads")
    ap.add_argument("--long-k", type=int, default=51)
    ap.add_argument("--no-tune", action="store_true", help="bacterial leg: no autotuned run beside the one at the "
                    "configuration's load factor 0.5")
    ap.add_argument("--served-payloads", type=int, default=64)
    ap.add_argument("--served-requests", type=int, default=1000)
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a streaming copy of known size (1 GiB read, 1 GiB written), "
                         "to scale hardware traffic counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch
    import readsim
    import paper_2401_02756_amd as dbg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    dbg.lib()
    graphs_on = not args.no_graph

    def load(cfg: int):
        t0 = time.perf_counter()
        rs = readsim.make_config(cfg)
        log("generated config %d: %d reads, %d bases in %.1f s" % (cfg, rs.n_reads, rs.total_bases,
                                                                  time.perf_counter() - t0))
        rs.d_reads = torch.from_numpy(rs.reads).to(dev)
        rs.d_off = torch.from_numpy(rs.offsets.astype(np.int64)).to(dev)
        rs.inserts = int(np.maximum(rs.lengths() - rs.k + 1, 0).sum())
        rs.windows = int(np.where(rs.lengths() >= rs.k, rs.lengths() - rs.k + 2, 0).sum())
        return rs

    def tuned(rs) -> tuple:
        t1 = time.perf_counter()
        t = dbg.autotune([0, rs.n_reads], [rs.k], rs.d_reads, rs.d_off, [rs.meta["expected_vertices"]],
                         keep_flags=dbg.F_GRAPH if graphs_on else 0, force=True)
        info = dict(t.as_dict(), seconds=round(time.perf_counter() - t1, 2))
        log("autotune: %s" % json.dumps(info))
        mode = "binned" if t.flags & dbg.F_BINNED else "direct"
        return (info, mode, t.load_factor, t.block_size, t.windows_per_thread, bool(t.flags & dbg.F_MERGE),
                dict(bin_chunks=t.bin_chunks, bin_scatter_div=t.bin_scatter_div, bin_shape1=t.bin_shape1,
                     bin_shape2=t.bin_shape2))

    names = {1: "tiny", 2: "bacterial_c2", 3: "large_c3"}
    profile = "hbm_traffic_%s.md"

    def leg(rs, cfg: int, mode: str, lf: float, block: int, wpt: int, merge: bool, steps: int, warmup: int,
            shape: dict) -> dict:
        r = measure_step(dbg, torch, dev, rs, rs.inserts, mode, lf, steps, warmup, graphs_on, block, wpt, merge,
                         shape)
        log("%s %s: step %.3f ms (%.2f G/s), V=%d, cap=%d" % (names[cfg], mode, r["ms_step"], r["value"],
                                                              r["V"], r["cap"]))
        # phase times: an uncaptured timed pass with events between the kernels
        pr = r if not graphs_on else measure_step(dbg, torch, dev, rs, rs.inserts, mode, lf, 2, 1, False, block,
                                                  wpt, merge, shape)
        table, roof = kernel_roofline(dbg, rs, rs.windows, rs.inserts, r["V"], r["cap"], r["ms_step"],
                                      pr["phases"], mode, lf, r["st"]["entry_bytes"], names[cfg],
                                      profile % names[cfg])
        return dict(r=r, phases=table, roofline=roof)

    def long_k_rate(rs, k: int, binned: bool, lf: float, steps: int = 5) -> dict:
        """The same reads at long k (two-word keys, 32-byte entries), binned
        or direct: whole step (reset, build, extraction) and build pass."""
        kins = int(np.maximum(rs.lengths() - k + 1, 0).sum())
        ev = readsim.expected_vertices(int(rs.meta["genome_len"]), int(rs.meta["read_len"]), rs.n_reads,
                                       float(rs.meta["err"]), k)
        flags = dbg.F_TIMING | (dbg.F_GRAPH if graphs_on else 0) | (dbg.F_BINNED if binned else 0)
        g = dbg.Graph(expected_vertices=ev, load_factor=lf if binned else 0.5, device=0, flags=flags)
        g.build_device(rs.d_reads, rs.d_off, k)
        g.sync()
        cap = int(g.stats()["capacity"])
        d_keys = torch.empty(2 * cap, dtype=torch.int64, device=dev)
        d_counts = torch.empty((cap, 4), dtype=torch.int32, device=dev)

        def step():
            g.reset()
            return g.build_extract_device(rs.d_reads, rs.d_off, k, d_keys, d_counts)

        step()
        torch.cuda.synchronize()
        kern = []
        t0 = time.perf_counter()
        for _ in range(steps):
            nv = step()
            kern.append(g.stats()["last_build_ms"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = g.stats()
        assert st["inserts"] == kins, (st["inserts"], kins)
        g.close()
        del d_keys, d_counts
        km = float(np.mean(kern))
        return {"k": k, "mode": "binned" if st["binned"] else "direct", "inserts_per_step": kins,
                "vertices": nv, "capacity": cap, "load_factor": lf if binned else 0.5,
                "entry_bytes": st["entry_bytes"], "ms_per_step": round(dt * 1e3, 3),
                "value": round(kins / dt / 1e9, 4), "build_ms": round(km, 4),
                "build_ginserts_s": round(kins / (km * 1e-3) / 1e9, 4)}

    def host_input_rate(rs, mode: str, lf: float, reps: int = 3) -> dict:
        """dbg_build from host memory: the ASCII reads and offsets cross PCIe
        inside each timed build (pageable numpy buffers)."""
        g = dbg.Graph(expected_vertices=rs.meta["expected_vertices"], load_factor=lf, device=0,
                      flags=dbg.F_BINNED if mode == "binned" else 0)
        g.build(rs.reads, rs.offsets, rs.k)  # warm-up
        t = []
        for _ in range(reps):
            g.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.build(rs.reads, rs.offsets, rs.k)
            t.append(time.perf_counter() - t0)
        g.close()
        ms = float(np.median(t)) * 1e3
        return {"ms": round(ms, 3), "ginserts_s": round(rs.inserts / ms / 1e6, 4),
                "bytes_over_pcie": int(rs.total_bases + 8 * (rs.n_reads + 1))}

    def contig_rate(rs, mode: str, lf: float, reps: int = 3) -> dict:
        """Contigs (findContigs, Algorithm 5) of the built graph, on the
        device: walk table, starts, walks, layout, spelling."""
        g = dbg.Graph(expected_vertices=rs.meta["expected_vertices"], load_factor=lf, device=0,
                      flags=dbg.F_BINNED if mode == "binned" else 0)
        t = []
        n = ln = V = 0
        for _ in range(reps + 1):
            g.reset()
            g.build_device(rs.d_reads, rs.d_off, rs.k)
            g.sync()
            V = g.vertex_count()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n, ln = g.contig_sizes()
            t.append(time.perf_counter() - t0)
        g.close()
        ms = float(np.median(t[1:])) * 1e3
        return {"ms": round(ms, 3), "contigs": n, "bases": ln, "vertices_per_s": round(V / ms * 1e3, 1)}

    if args.calibrate:
        # k_stream_copy: reads 1 GiB and writes 1 GiB with 16-byte accesses
        # (run twice: one warm-up, one timed launch)
        dbg.atomic_roofline(dbg.ROOF_COPY, 2 << 30, 0, 256, 1)
        log("calibration: streaming copy of 1 GiB")

    # ---------------------------------------------------------------- headline
    rs = load(args.config)
    tuning = None
    mode, lf, block, wpt, merge = args.mode, args.load_factor, 0, 0, False
    shape = dict(bin_chunks=args.bin_chunks, bin_scatter_div=args.bin_div, bin_shape1=args.bin_shape1,
                 bin_shape2=args.bin_shape2)
    if args.tune:
        tuning, mode, lf, block, wpt, merge, shape = tuned(rs)
    h = leg(rs, args.config, mode, lf, block, wpt, merge, args.steps, args.warmup, shape)
    r = h["r"]
    st = r["st"]
    line = {
        "metric": "k-mer inserts/sec (G/s)",
        "value": round(r["value"], 4),
        "unit": "G k-mer inserts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain build, %s" % rs.meta["name"],
                   "reads": rs.n_reads, "read_len": int(rs.meta["read_len"]), "k": rs.k,
                   "inserts_per_step": rs.inserts, "vertices": r["V"], "capacity": r["cap"],
                   "table_bytes": int(st["table_bytes"]), "load_factor": lf, "entry_bytes": st["entry_bytes"],
                   "mode": mode, "hip_graphs": graphs_on, "bin_chunks": shape["bin_chunks"],
                   "bin_scatter_div": shape["bin_scatter_div"],
                   "bin_shapes": [int(st["bin_shape1"]), int(st["bin_shape2"])],
                   "step": "reset + dbg_build_extract_device (build, every vertex written to device "
                           "buffers, status read back)"},
        "build_kernel_ginserts_s": round(rs.inserts / (r["kern_ms"] * 1e-3) / 1e9, 4),
        "extract_separate_ms": round(r["extract_ms"], 4),  # dbg_extract_device on the built graph
        "autotune": tuning,
        "roofline": h["roofline"],
        "phases": h["phases"],
    }
    log("roofline %s" % json.dumps(h["roofline"]))
    if not args.no_compare:
        other = "direct" if mode == "binned" else "binned"
        o = measure_step(dbg, torch, dev, rs, rs.inserts, other, lf, 3, 1, graphs_on)
        line["compare_" + other] = {"value": round(o["value"], 4), "ms_per_step": round(o["ms_step"], 4),
                                   "build_ginserts_s": round(rs.inserts / (o["kern_ms"] * 1e-3) / 1e9, 4),
                                   "build_ms": round(o["kern_ms"], 4)}
        log("%s: %s" % (other, json.dumps(line["compare_" + other])))
    if not args.no_roofline:
        foot = int(st["table_bytes"])
        ar = {"footprint_bytes": foot, "ops": rs.inserts}
        for name, kind in (("cas64", dbg.ROOF_CAS64), ("add32", dbg.ROOF_ADD32),
                           ("load64", dbg.ROOF_LOAD64), ("load_add", dbg.ROOF_LOAD_ADD)):
            best = min(dbg.atomic_roofline(kind, foot, rs.inserts, b, 3) for b in (256, 1024))
            ar[name + "_gops"] = round(rs.inserts / (best * 1e-3) / 1e9, 4)
        ar["build_frac_of_cas64"] = round(line["build_kernel_ginserts_s"] / ar["cas64_gops"], 4)
        ar["step_frac_of_cas64"] = round(r["value"] / ar["cas64_gops"], 4)
        line["atomic_roofline"] = ar
        log("atomic roofline %s" % json.dumps(ar))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(rs, args.cpu_sample_reads)
        log("cpu baseline %s" % json.dumps(line["cpu_baseline"]))
        line["cpu_lfdbg"] = cpu_lfdbg_scaling(rs, args.cpu_sample_reads)
        log("cpu lfdbg %s" % json.dumps(line["cpu_lfdbg"]))
    del rs.d_reads, rs.d_off
    del rs
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- bacterial scale
    if not args.no_bacterial and args.config != 2:
        b = load(2)
        # the configuration's own table load factor (0.5), default launch shape
        bmode, blf = "binned", 0.5
        bl = leg(b, 2, bmode, blf, 0, 0, False, max(args.steps, 10), args.warmup, {})
        br = bl["r"]
        bac = {"workload": "plain build, %s" % b.meta["name"], "inserts_per_step": b.inserts,
               "vertices": br["V"], "capacity": br["cap"], "load_factor": blf, "mode": bmode,
               "bin_shapes": [int(br["st"]["bin_shape1"]), int(br["st"]["bin_shape2"])],
               "value": round(br["value"], 4), "ms_per_step": round(br["ms_step"], 4),
               "build_kernel_ginserts_s": round(b.inserts / (br["kern_ms"] * 1e-3) / 1e9, 4),
               "roofline": bl["roofline"], "phases": bl["phases"]}
        if not args.no_tune:
            # the autotuner's choice for the same reads, timed the same way
            btune, tmode, tlf, tblock, twpt, tmerge, tshape = tuned(b)
            tr = measure_step(dbg, torch, dev, b, b.inserts, tmode, tlf, max(args.steps, 10), args.warmup, graphs_on,
                              tblock, twpt, tmerge, tshape)
            bac["autotuned"] = {"tuning": btune, "value": round(tr["value"], 4), "ms_per_step": round(tr["ms_step"], 4),
                                "vertices": tr["V"], "capacity": tr["cap"]}
            log("bacterial autotuned: %s" % json.dumps(bac["autotuned"]))
        if not args.no_compare:
            o = measure_step(dbg, torch, dev, b, b.inserts, "direct", 0.5, 5, 1, graphs_on)
            bac["compare_direct"] = {"value": round(o["value"], 4), "ms_per_step": round(o["ms_step"], 4),
                                     "build_ginserts_s": round(b.inserts / (o["kern_ms"] * 1e-3) / 1e9, 4)}
        if not args.no_long_k:
            bac["long_k"] = long_k_rate(b, args.long_k, True, blf)
            bac["long_k"]["compare_direct"] = long_k_rate(b, args.long_k, False, blf)
        bac["contigs"] = contig_rate(b, bmode, blf)
        bac["host_input"] = host_input_rate(b, bmode, blf)
        line["bacterial"] = bac
        log("bacterial %s" % json.dumps(bac))
        del b.d_reads, b.d_off
        torch.cuda.empty_cache()

    if not args.no_batched:
        line["batched"] = batched_bench(dbg, torch, dev, args.batched_sets, args.batched_reps, graphs_on)
        log("batched %s" % json.dumps(line["batched"]))

    if not args.no_served:
        ref = line["batched"]["batched"]["ginserts_s"] if "batched" in line else line["value"]
        line["served"] = served_bench(dbg, torch, dev, args.served_payloads, args.served_requests,
                                      (0.7, 0.5, 0.9), ref)

    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
