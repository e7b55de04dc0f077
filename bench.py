"""Benchmark: kernel entries per second of the gapped k-mer Gram path on one MI355X.

Workload: the protein Gram configuration -- N=3312 sequences over Sigma=20,
lengths U{50..500}, Zipf(1.1) symbol composition, g=7, k=4 (M=3) -- computed
in full: N_m for m=0..3 (int64, exact) and the FP64 cosine-normalised K.
One step = one gakco_gram call over device-resident inputs into preallocated
device outputs (validation, extraction, every position set's partition, sort
and segmentation, row accumulation, int8 matrix-core products,
inclusion-exclusion, K and normalisation).

Prints ONE JSON line:
  value / ms_per_step  from the timed steps (no profiler attached);
  roofline             the dominant kernel of separate profiled steps (HIP
                       events around each launch on the library's stream),
                       its algorithmic bytes per launch over its mean launch
                       time, and the HBM traffic measured by rocprofv3 PMC
                       runs when those were taken from the current sources;
  accumulate_lds       the row accumulation's sequence-pair updates per second
                       over a probe's rate of random LDS atomic adds;
  dense_mfma           the int8 count-matrix products' TOP/s over the dense
                       int8 peak;
  sort_accumulate      the partition, sort and accumulation kernels together:
                       the method's bytes (three passes over 12-byte records
                       per position set and g-mer, one write of every C_m)
                       over their summed launch times, against HBM peak;
  cpu_baseline         the CPU oracle on the whole workload with its position
                       sets dealt to the host's cores, and single-threaded on
                       a sub-Gram;
  serving              continuous-batching rows of the serving workload
                       (resident 20000 DNA support sequences, g=10, k=6): the
                       server's saturation rate (a burst), then Poisson
                       arrivals at 30/60/90 % of it -- p50/p99 latency and
                       rows/s -- beside the plain path (one gakco_rows call
                       per query), and the row kernel's pair updates/s;
  batched              the 64-job batched workload replayed from its captured
                       hipGraph, with default and autotuned settings, beside
                       the same jobs run one by one;
  other_configs        the DNA (N=200) and text (N=2000, M=6) Gram workloads
                       timed the same way, with their sort + accumulate
                       fraction of HBM peak.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_protein_gram.json")

# profiler phase -> kernel name as rocprofv3 reports it
PHASE_KERNEL = {
    "fill": "k_fill_u64", "validate": "k_validate", "extract": "k_extract", "bucket_count": "k_bucket_count",
    "bucket_scan": "k_bucket_scan", "bucket_scatter": "k_bucket_scatter", "sort_wave": "k_sort_wave<false>",
    "sort_wave_big": "k_sort_wave<true>", "sort_block": "k_sort_block", "sort_global": "k_sort_global",
    "accumulate": "k_accumulate", "dense_syrk": "k_dense_syrk", "dense_clear": "k_dense_clear",
    "diag": "k_diag", "finalize": "k_finalize", "direct_count": "k_direct_count", "direct_excess": "k_direct_excess",
    "rows_qdiag": "k_query_diag", "rows_count": "k_count_rows", "rows_gemm": "k_rows_gemm",
}

# headline workloads (--workload); the protein Gram is the measured metric's
WORKLOADS = {
    "protein": "protein Gram: N=3312, Sigma=20 Zipf(1.1), l~U{50..500}, g=7, k=4 (M=3); "
               "outputs N_m int64 [4,N,N] + normalised K f64 [N,N]",
    "text": "text Gram: N=2000, Sigma=36 Markov-1 Dirichlet(0.3), l~U{200..1000}, g=10, k=4 (M=6); "
            "outputs N_m int64 [7,N,N] + normalised K f64 [N,N]",
    "dna": "DNA Gram: N=200, Sigma=4 iid, l=100, g=6, k=4 (M=2); outputs N_m int64 [3,N,N] + normalised K f64 [N,N]",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="protein",
                    help="the Gram workload timed as the headline (protein: the metric's configuration)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=5, help="profiled steps for the per-kernel times")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1200,
                    help="sequences in the single-threaded oracle's sub-Gram")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-queries", type=int, default=2000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the DNA and text Gram legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB elementwise copy (scale for PMC byte counters)")
    ap.add_argument("--profile-phases", action="store_true", help="print the per-kernel table to stderr")
    ap.add_argument("--dense-tau", type=int, default=None, help="override the int8 matrix-core threshold")
    ap.add_argument("--bucket-avg", type=int, default=None, help="override the partition bucket size")
    ap.add_argument("--no-overlap", action="store_true",
                    help="all kernels on one stream (per-kernel traces without side-stream overlap)")
    return ap.parse_args()


def algorithmic(d, masks, prof_stats, dense_rows, ntile):
    """Per-call algorithmic bytes (or int8 ops) of each kernel: what the
    method must move, not what a kernel happens to move."""
    N, M = d.N, d.M
    T = int(sum(max(0, int(l) - d.g + 1) for l in d.lens))
    S = sum(masks)
    nsym = int(sum(int(l) for l in d.lens))
    tri = N * (N + 1) // 2
    # every (mask, g-mer) passes one sort kernel: packed (4-byte composite)
    # or wide (8-byte); the partition reads the g-mer key (and the sequence
    # id, unless it fits above the key) and writes that composite and the index
    pk_all = sum(prof_stats.get(k, 0) for k in ("wave", "block", "global"))
    wide_all = sum(prof_stats.get(k + "_wide", 0) for k in ("wave", "block", "global"))
    b = max(1, (d.sigma - 1).bit_length())
    sb = max(1, (N - 1).bit_length())
    key_read = 8 if d.g * b + sb <= 64 else 12
    scatter = key_read * T * S + 4 * pk_all + 8 * wide_all + 4 * (pk_all + wide_all)
    sortb = {}
    for kind in ("wave", "block", "global"):
        pk, wide = prof_stats.get(kind, 0), prof_stats.get(kind + "_wide", 0)
        # read the composite and index, write the g-mer's info (run entries,
        # at most one 4-byte word per g-mer, are not counted)
        sortb["sort_" + kind] = pk * (4 + 4 + 8) + wide * (8 + 4 + 8)
    return {
        "extract": nsym + 12 * T,
        "bucket_count": 8 * T * S,
        "bucket_scatter": scatter,
        **sortb,
        # the method's bytes for this step: every (mask, g-mer) grouped
        # (reduced key, sequence) record of 12 bytes read once, and every
        # C_m written once (8 N^2 per level)
        "accumulate": 12 * T * S + 8 * (M + 1) * N * N,
        # each count-matrix row read once (bytes); ops below
        "dense_syrk": ntile * dense_rows,
        "finalize": 8 * (M + 1) * tri + 8 * (M + 1) * N * N + 8 * N * N,
        "fill": 8 * (M + 1) * N * N,
    }, T


def traffic_for(kernel):
    """Measured HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy kernel's counters), or None when the stored counters
    were taken from other sources."""
    try:
        from paper_1704_07468_amd.profiling import source_sha
        t = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if t.get("source_sha") != source_sha():
        return None
    k = t["kernels"].get(kernel)
    c = t["copy"]
    if not k or k.get("write_kib") is None or not c.get("fetch_kib") or not c.get("write_kib"):
        return None
    f_scale = c["bytes_read"] / (c["fetch_kib"] * 1024.0)
    w_scale = c["bytes_written"] / (c["write_kib"] * 1024.0)
    return k["fetch_kib"] * 1024.0 * f_scale + k["write_kib"] * 1024.0 * w_scale


def note(msg):
    print("[bench %7.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


T_START = time.perf_counter()


def host_cpu():
    """(cores this process may use, at most 16 -- the host share of one GPU --,
    the CPU model)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return max(1, min(16, n)), model


def cpu_baseline(d, n_single):
    """The oracle (Algorithm 1) on the whole workload with the position sets
    dealt to every host core (Section S:5.3), and single-threaded on the
    sub-Gram of the first n_single sequences (a bounded sample)."""
    from oracle import oracle as orc
    cores, model = host_cpu()
    t0 = time.perf_counter()
    orc.kernel(d.seqs, d.lens, d.g, d.k, threads=cores, per_mask=True, want_c=False)
    dt = time.perf_counter() - t0
    n_single = min(n_single, d.N)
    sub = d.subset(range(n_single))
    t0 = time.perf_counter()
    orc.kernel(sub.seqs, sub.lens, sub.g, sub.k, threads=1, want_c=False)
    dt1 = time.perf_counter() - t0
    return {"value": d.N * d.N / dt, "unit": "kernel entries/s", "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "sample": "oracle (Algorithm 1, position sets dealt to %d threads) on the whole protein workload: "
                      "%dx%d Gram (N_m and K) in %.2f s" % (cores, d.N, d.N, dt),
            "single_thread": {"value": n_single * n_single / dt1, "unit": "kernel entries/s", "cores": 1,
                              "sample": "the same oracle on one thread, sub-Gram of the first %d sequences "
                                        "(%dx%d) in %.2f s" % (n_single, n_single, n_single, dt1)}}


def _drive(srv, queries, tags, arrivals):
    """Submit queries[i] (tag tags[i]) at arrivals[i] seconds from now (all at
    once when arrivals is None) and collect every result."""
    n = len(queries)
    done = {}
    t0 = time.perf_counter()
    i = 0
    if arrivals is None:
        for q, t in zip(queries, tags):
            srv.submit(q, t)
        i = n
    while len(done) < n:
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            srv.submit(queries[i], tags[i])
            i += 1
        wait = 20000 if i >= n else max(20, min(200, int((arrivals[i] - now) * 1e6)))
        for r in srv.poll(256, wait, rows=False):
            done[r["tag"]] = r
    return done, time.perf_counter() - t0


def serving_leg(gakco, wl, n_q, lds_peak):
    """The serving workload: plain path (one gakco_rows call per query, no
    overlap) beside the continuous-batching server -- its saturation rate
    from a burst of n_q queries, then Poisson arrivals at 30/60/90 % of that
    rate, n_q measured queries per rate after n_q / 10 warm-up arrivals."""
    import numpy as np
    import torch
    s = wl.serving_resident()
    n_sv = s.sv.N
    ctx = gakco.Context(0)
    res = gakco.Resident(ctx, s.sv.seqs, s.sv.lens, s.sv.sigma, s.sv.g, s.sv.k, alpha=s.alpha, bias=s.bias)
    try:
        n_warm = max(50, n_q // 10)
        q_seqs, q_lens = wl.serving_queries(n_q + n_warm)
        qoff = np.concatenate([[0], np.cumsum(q_lens)])
        queries = [q_seqs[qoff[i]:qoff[i + 1]] for i in range(len(q_lens))]
        note("serving: resident set built (%d queries, lengths %d..%d)" % (len(queries), q_lens.min(), q_lens.max()))
        # plain: one rows call per query on device-resident queries
        dev_q = [(torch.as_tensor(q).cuda(), torch.as_tensor(np.array([len(q)], dtype=np.int32)).cuda())
                 for q in queries]
        for q, l in dev_q[:n_warm]:
            res.rows(q, l)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for q, l in dev_q[n_warm:]:
            a = time.perf_counter()
            res.rows(q, l)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - a)
        plain_wall = time.perf_counter() - t0
        note("serving: plain path %d queries in %.2f s" % (n_q, plain_wall))
        out = {"workload": "resident N_sv=20000 DNA l=200, g=10, k=6 (M=4); queries l~U{50..1000}, Poisson "
                           "arrivals; %d measured queries per rate after %d warm-up" % (n_q, n_warm),
               "unit": "ms",
               "plain": {"p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                         "qps": n_q / plain_wall, "rows_per_s": n_q * n_sv / plain_wall}}
        # the row kernel against its roofs, on one batch of 256 queries
        bq = torch.as_tensor(np.concatenate(queries[n_warm:n_warm + 256])).cuda()
        bl = torch.as_tensor(q_lens[n_warm:n_warm + 256]).cuda()
        res.rows(bq, bl)
        ctx.set_param("profile", 1)
        ctx.profile_reset()
        reps = 3
        for _ in range(reps):
            res.rows(bq, bl)
        torch.cuda.synchronize()
        prof = ctx.profile()
        upd = ctx.stat("rows_updates") / reps
        ctx.set_param("profile", 0)
        rk_ms = prof["rows"][0] / max(1, prof["rows"][1])
        gm = prof.get("rows_gemm", (0.0, 0))
        rate = upd / (rk_ms / 1e3)
        # bytes the row kernel must move: every gathered (sequence, count)
        # entry (4 B), a 16-byte group lookup per (position set, query g-mer),
        # every C_m row entry added once (4 B)
        ng = int(np.maximum(q_lens[n_warm:n_warm + 256] - s.sv.g + 1, 0).sum())
        npos = sum(math.comb(s.sv.g, m) for m in range(s.sv.g - s.sv.k + 1))
        rbytes = 4 * upd + 16 * npos * ng + 4 * (s.sv.g - s.sv.k + 1) * 256 * n_sv
        out["rows_kernel"] = {"kernel": "k_rows_accumulate", "batch": 256, "mean_launch_ms": round(rk_ms, 4),
                              "updates_per_launch": round(upd), "achieved": round(rate / 1e9, 1),
                              "peak": round(lds_peak / 1e9, 1), "unit": "G updates/s",
                              "frac": round(rate / lds_peak, 4),
                              "hbm": {"algorithmic_bytes": round(rbytes),
                                      "achieved": round(rbytes / (rk_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(rbytes / (rk_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
                              "peak_source": "k_lds_atomic_probe: random adds into a 4096-word LDS row"}
        if gm[1]:
            # the top level as an int8 product: 2 ops per (query, resident
            # sequence, count column) of the padded 256-query tile
            M_ = s.sv.g - s.sv.k
            b_ = max(1, math.ceil(math.log2(s.sv.sigma)))
            cols = math.comb(s.sv.g, M_) * (1 << ((s.sv.g - M_) * b_))
            g_ms = gm[0] / gm[1]
            ops = 2.0 * 256 * n_sv * cols
            out["dense_level_joined"] = {"kernel": "k_rows_gemm", "level": M_, "count_columns": cols,
                                         "mean_launch_ms": round(g_ms, 4),
                                         "achieved": round(ops / (g_ms / 1e3) / 1e12, 1), "peak": 5000.0,
                                         "unit": "TOP/s (int8)", "frac": round(ops / (g_ms / 1e3) / 5e15, 4),
                                         "count_rows_ms": round(prof.get("rows_count", (0.0, 1))[0] / max(1, prof.get("rows_count", (0.0, 1))[1]), 4)}
        srv = gakco.Server(res, max_batch=256, n_streams=2)
        try:
            meas = queries[n_warm:]
            tags = list(range(n_q))
            _drive(srv, queries[:n_warm], [10 ** 6 + i for i in range(n_warm)], None)  # warm-up burst
            done, wall = _drive(srv, meas, tags, None)
            sat = n_q / wall
            out["server_saturation"] = {"qps": sat, "rows_per_s": n_q * n_sv / wall,
                                        "mean_batch": float(np.mean([done[t]["batch_size"] for t in tags])),
                                        "all_ok": all(done[t]["status"] == 0 for t in tags),
                                        "vs_plain_rows_per_s": (n_q * n_sv / wall) / out["plain"]["rows_per_s"]}
            note("serving: saturation %.0f queries/s (burst of %d)" % (sat, n_q))
            for frac in (0.3, 0.6, 0.9):
                rate_q = frac * sat
                arr = wl.poisson_arrivals(n_warm + n_q, rate_q, seed=wl.SEED_BASE + 6 + int(frac * 10))
                alltags = [2 * 10 ** 6 + i for i in range(n_warm)] + tags
                done, wall = _drive(srv, queries[:n_warm] + meas, alltags, arr)
                lat_s = [done[t]["t_done"] - done[t]["t_submit"] for t in tags]
                span = max(done[t]["t_done"] for t in tags) - min(done[t]["t_submit"] for t in tags)
                out["load_%d%%" % round(100 * frac)] = {
                    "offered_qps": rate_q, "p50_ms": 1e3 * float(np.percentile(lat_s, 50)),
                    "p99_ms": 1e3 * float(np.percentile(lat_s, 99)), "rows_per_s": n_q * n_sv / span,
                    "mean_batch": float(np.mean([done[t]["batch_size"] for t in tags])),
                    "all_ok": all(done[t]["status"] == 0 for t in tags)}
                note("serving: %d%% of saturation, %d queries in %.2f s" % (round(100 * frac), n_q, wall))
        finally:
            srv.close()
        # reference: the same server with the top level always on the sparse
        # walk (small batches are as efficient as large ones there, so its
        # latency stays low up to its lower saturation)
        if out.get("dense_level_joined"):
            ctx0 = gakco.Context(0, tune={"rows_dense": 0})
            res0 = gakco.Resident(ctx0, s.sv.seqs, s.sv.lens, s.sv.sigma, s.sv.g, s.sv.k, alpha=s.alpha, bias=s.bias)
            srv0 = gakco.Server(res0, max_batch=256, n_streams=2)
            try:
                meas = queries[n_warm:]
                tags = list(range(n_q))
                _drive(srv0, queries[:n_warm], [10 ** 6 + i for i in range(n_warm)], None)
                done, wall = _drive(srv0, meas, tags, None)
                sat0 = n_q / wall
                ref = {"server_saturation_qps": sat0}
                for frac in (0.9,):
                    arr = wl.poisson_arrivals(n_warm + n_q, frac * sat0, seed=wl.SEED_BASE + 6 + int(frac * 10))
                    alltags = [2 * 10 ** 6 + i for i in range(n_warm)] + tags
                    done, wall = _drive(srv0, queries[:n_warm] + meas, alltags, arr)
                    lat_s = [done[t]["t_done"] - done[t]["t_submit"] for t in tags]
                    ref["load_%d%%" % round(100 * frac)] = {
                        "offered_qps": frac * sat0, "p50_ms": 1e3 * float(np.percentile(lat_s, 50)),
                        "p99_ms": 1e3 * float(np.percentile(lat_s, 99)),
                        "mean_batch": float(np.mean([done[t]["batch_size"] for t in tags])),
                        "all_ok": all(done[t]["status"] == 0 for t in tags)}
                out["sparse_walk_only"] = ref
                note("serving: sparse-walk-only server saturates at %.0f queries/s" % sat0)
            finally:
                srv0.close()
                res0.close()
                ctx0.close()
        return out
    finally:
        res.close()
        ctx.close()


def batched_leg(gakco, wl):
    """The 64-job batched workload: the jobs one by one on the plain path,
    then one batch replayed from its captured hipGraph with the default
    settings and with the settings gakco_autotune picks for these jobs."""
    import torch
    jobs_in = wl.batched()
    ctx = gakco.Context(0)
    try:
        def mk():
            return [{"seqs": j.seqs, "lens": j.lens, "sigma": j.sigma, "g": j.g, "k": j.k} for j in jobs_in]
        entries = sum(j.N * j.N for j in jobs_in)
        # plain: one gakco_gram per job, outputs preallocated
        plain = mk()
        dev = [(torch.as_tensor(j["seqs"]).cuda(), torch.as_tensor(j["lens"]).cuda()) for j in plain]
        outs = [(torch.empty((j.N, j.N), dtype=torch.float64, device="cuda"),
                 torch.empty((j.M + 1, j.N, j.N), dtype=torch.int64, device="cuda")) for j in jobs_in]

        def run_plain():
            for j, (s, l), (K, Nm) in zip(jobs_in, dev, outs):
                ctx.gram_into(s, l, j.N, j.sigma, j.g, j.k, K=K, Nm=Nm)
        run_plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_plain()
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        note("batched: plain serial %.1f ms" % (1e3 * t_plain))
        # plain per position set: the same calls with one position set per
        # launch sequence (count, scan, scatter, sort, accumulate per mask,
        # the loop structure of Algorithm 1)
        ctx.set_param("chunk_masks", 1)
        run_plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_plain()
        torch.cuda.synchronize()
        t_mask = time.perf_counter() - t0
        ctx.set_param("chunk_masks", 0)
        note("batched: plain one position set at a time %.1f ms" % (1e3 * t_mask))

        def graph(c):
            bjobs = mk()
            plan = c.batch_plan(bjobs)
            try:
                plan.run()
                torch.cuda.synchronize()
                reps = 3
                t0 = time.perf_counter()
                for _ in range(reps):
                    st = plan.run()
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / reps
                same = all(torch.equal(b["Nm"], Nm) and torch.equal(b["K"], K) for b, (K, Nm) in zip(bjobs, outs))
            finally:
                plan.close()
            return t, same, all(x == 0 for x in st)
        t_graph, same, ok = graph(ctx)
        note("batched: graph %.1f ms" % (1e3 * t_graph))
        t0 = time.perf_counter()
        table = ctx.autotune(mk(), reps=1)
        t_tune = time.perf_counter() - t0
        t_tuned, same_t, ok_t = graph(ctx)
        note("batched: autotuned graph %.1f ms (tuning took %.1f s)" % (1e3 * t_tuned, t_tune))
        return {"workload": "64 jobs N~U{100..2000}, Sigma in {4,20,36}, l~U{50..600}, g in [6,10], k in [3,g-2]",
                "unit": "kernel entries/s", "entries": entries,
                "plain_serial": {"ms": 1e3 * t_plain, "value": entries / t_plain},
                "plain_per_position_set": {"ms": 1e3 * t_mask, "value": entries / t_mask},
                "graph_replay": {"ms": 1e3 * t_graph, "value": entries / t_graph, "vs_plain": t_plain / t_graph,
                                 "vs_plain_per_position_set": t_mask / t_graph},
                "graph_replay_autotuned": {"ms": 1e3 * t_tuned, "value": entries / t_tuned,
                                           "vs_plain": t_plain / t_tuned,
                                           "vs_plain_per_position_set": t_mask / t_tuned, "tuning_s": round(t_tune, 2),
                                           "table": __import__("json").loads(table)},
                "identical_results": bool(same and same_t), "status_ok": bool(ok and ok_t)}
    finally:
        ctx.close()


def config_leg(gakco, d, label, steps=10):
    """Another Gram workload, timed like the headline one (device-resident
    inputs, preallocated outputs), with its per-kernel profile and the
    sort + accumulate fraction of HBM peak."""
    import torch
    dev = torch.device("cuda", 0)
    seqs = torch.as_tensor(d.seqs).to(dev)
    lens = torch.as_tensor(d.lens).to(dev)
    N, M = d.N, d.M
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    Nm = torch.empty((M + 1, N, N), dtype=torch.int64, device=dev)
    ctx = gakco.Context(0)
    try:
        for _ in range(2):
            ctx.gram_into(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.gram_into(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ctx.set_param("profile", 1)
        ctx.profile_reset()
        P = 2
        for _ in range(P):
            ctx.gram_into(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm)
        torch.cuda.synchronize()
        prof = ctx.profile()
        ctx.set_param("profile", 0)
    finally:
        ctx.close()
    kern = {k_: round(v[0] / P, 4) for k_, v in prof.items() if v[1]}
    T = int(sum(max(0, int(l) - d.g + 1) for l in d.lens))
    S = sum(math.comb(d.g, m) for m in range(M + 1))
    sa_kernels = ("bucket_count", "bucket_scan", "bucket_scatter", "sort_wave", "sort_wave_big", "sort_block",
                  "sort_global", "accumulate", "dense_syrk", "dense_clear", "direct_count", "direct_excess")
    sa_ms = sum(kern.get(k_, 0.0) for k_ in sa_kernels)
    sa_bytes = 3 * 12 * T * S + 8 * (M + 1) * N * N
    note("%s: %.3f ms/step" % (label, ms))
    return {"workload": label, "N": N, "sigma": d.sigma, "g": d.g, "k": d.k, "T_gmers": T, "position_sets": S,
            "ms_per_step": ms, "value": N * N / (ms / 1e3), "unit": "kernel entries/s",
            "sort_accumulate": {"algorithmic_bytes": sa_bytes, "ms_per_step": round(sa_ms, 4),
                                "achieved": round(sa_bytes / (sa_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(sa_bytes / (sa_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
            "kernels_ms_per_step": kern}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1704_07468_amd import gakco, workloads as wl

    if not os.path.exists(gakco.LIB_PATH):
        from paper_1704_07468_amd import build as b
        b.build()
    d = getattr(wl, args.workload)()
    dev = torch.device("cuda", 0)
    seqs = torch.as_tensor(d.seqs).to(dev)
    lens = torch.as_tensor(d.lens).to(dev)
    N, M = d.N, d.M
    K = torch.empty((N, N), dtype=torch.float64, device=dev)
    Nm = torch.empty((M + 1, N, N), dtype=torch.int64, device=dev)
    tune = {}
    if args.dense_tau is not None:
        tune["dense_tau"] = args.dense_tau
    if args.bucket_avg is not None:
        tune["bucket_avg"] = args.bucket_avg
    if args.no_overlap:
        tune["overlap"] = 0
    ctx = gakco.Context(0, tune=tune or None)
    for _ in range(args.warmup):
        ctx.gram_into(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.gram_into(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    value = N * N / (ms / 1000.0)

    # per-kernel launch times from separate profiled steps
    ctx.set_param("profile", 1)
    ctx.profile_reset()
    P = max(1, args.profile_steps)
    for _ in range(P):
        ctx.gram_into(seqs, lens, N, d.sigma, d.g, d.k, K=K, Nm=Nm)
    torch.cuda.synchronize()
    prof = ctx.profile()
    sstat = {k: ctx.stat("sort_gmers_" + k) / P for k in ("wave", "wave_wide", "block", "block_wide", "global", "global_wide")}
    dense_rows = ctx.stat("dense_rows")
    acc_updates = ctx.stat("acc_updates") / P
    ctx.set_param("profile", 0)
    lds_peak = ctx.probe_lds_atomics(4096)  # reference rate of random LDS adds
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    masks = [math.comb(d.g, m) for m in range(M + 1)]
    ntile = -(-N // 128) * 128
    alg, T = algorithmic(d, masks, sstat, dense_rows, ntile)
    kern = {}
    for ph, (tot_ms, n) in prof.items():
        if n:
            kern[ph] = {"ms_per_step": tot_ms / P, "launches_per_step": n / P, "mean_launch_ms": tot_ms / n}
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    dk = kern[dom]
    launch_s = dk["mean_launch_ms"] / 1000.0
    if dom == "dense_syrk":
        ops = ntile * ntile * dense_rows / dk["launches_per_step"]  # 2 ops per MAC over the upper triangle
        roof = {"bound": "mfma", "kernel": PHASE_KERNEL[dom], "achieved": round(ops / launch_s / 1e12, 2),
                "peak": 5000.0, "unit": "TOP/s", "frac": round(ops / launch_s / 1e12 / 5000.0, 4), "traffic": None}
    else:
        per_launch = alg.get(dom, 0) / dk["launches_per_step"]
        achieved = per_launch / launch_s / 1e9
        tr = traffic_for(PHASE_KERNEL.get(dom, dom))
        roof = {"bound": "hbm", "kernel": PHASE_KERNEL.get(dom, dom), "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if tr is None else round(tr),
                "algorithmic_bytes": round(per_launch), "mean_launch_ms": round(dk["mean_launch_ms"], 4)}
    # the accumulation against its other roofs: LDS atomic adds (pair
    # updates per second over the probe's rate) and, for the count-matrix
    # groups, int8 MFMA
    extra = {}
    if "accumulate" in kern:
        rate = acc_updates / (kern["accumulate"]["ms_per_step"] / 1e3)
        extra["accumulate_lds"] = {"kernel": "k_accumulate", "updates_per_step": round(acc_updates),
                                   "achieved": round(rate / 1e9, 1), "peak": round(lds_peak / 1e9, 1),
                                   "unit": "G updates/s", "frac": round(rate / lds_peak, 4),
                                   "peak_source": "k_lds_atomic_probe: random adds into a 4096-word LDS row"}
    if "dense_syrk" in kern and dense_rows:
        ops = ntile * ntile * dense_rows
        tops = ops / (kern["dense_syrk"]["ms_per_step"] / 1e3) / 1e12
        extra["dense_mfma"] = {"kernel": "k_dense_syrk", "rows": int(dense_rows), "achieved": round(tops, 1),
                               "peak": 5000.0, "unit": "TOP/s", "frac": round(tops / 5000.0, 4)}
    # sort + accumulate as one phase of the path (the method's bytes over the
    # summed launch times of its kernels): every (mask, g-mer) record of 12
    # bytes read by the partition, written grouped and read once to
    # accumulate, and every C_m written once
    sa_kernels = ("bucket_count", "bucket_scan", "bucket_scatter", "sort_wave", "sort_wave_big", "sort_block",
                  "sort_global", "accumulate", "dense_syrk", "dense_clear", "direct_count", "direct_excess")
    sa_ms = sum(kern[k_]["ms_per_step"] for k_ in sa_kernels if k_ in kern)
    sa_bytes = 3 * 12 * T * sum(masks) + 8 * (M + 1) * N * N
    extra["sort_accumulate"] = {"kernels": [PHASE_KERNEL[k_] for k_ in sa_kernels if k_ in kern],
                                "algorithmic_bytes": sa_bytes, "ms_per_step": round(sa_ms, 4),
                                "achieved": round(sa_bytes / (sa_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": round(sa_bytes / (sa_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    if args.profile_phases:
        for k_, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms_per_step"]):
            a = alg.get(k_)
            gbs = "" if not a else "%8.1f GB/s algorithmic" % (a / (v["ms_per_step"] / 1e3) / 1e9)
            print("%-15s %8.3f ms/step %5.1f launches/step %s" % (k_, v["ms_per_step"], v["launches_per_step"], gbs),
                  file=sys.stderr)
    ctx.close()

    note("gram: %.3f ms/step" % ms)
    cpu = None if args.no_cpu_baseline else cpu_baseline(d, args.cpu_sample)
    if cpu:
        note("cpu baseline: " + cpu["sample"])
    batched = None if args.no_batched else batched_leg(gakco, wl)
    configs = None
    if not args.no_configs:
        configs = {"dna": config_leg(gakco, wl.dna(), "DNA Gram: N=200, l=100, Sigma=4, g=6, k=4 (M=2)", steps=50),
                   "text": config_leg(gakco, wl.text(), "text Gram: N=2000, l~U{200..1000}, Sigma=36 Markov-1, "
                                                        "g=10, k=4 (M=6)", steps=5)}
    serving = None if args.no_serving else serving_leg(gakco, wl, args.serving_queries, lds_peak)
    line = {
        "metric": "kernel entries/sec (Gram + query rows) bit-exact; serving p50/p99 latency vs plain",
        "value": value, "unit": "kernel entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "N": N, "sigma": d.sigma, "g": d.g, "k": d.k, "T_gmers": T, "position_sets": sum(masks)},
        "roofline": roof,
        **extra,
        "cpu_baseline": cpu,
        "serving": serving,
        "batched": batched,
        "other_configs": configs,
        "kernels_ms_per_step": {k_: round(v["ms_per_step"], 4) for k_, v in kern.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
