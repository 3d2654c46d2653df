#!/usr/bin/env python3
"""Exact Hamming kNN throughput on one MI355X: multi-index hashing vs the GPU
linear scan, on synthetic codes shaped like the paper's 1B-code experiments.

Default workload: 1e9 uniform 64-bit codes (seed 0), m = 2 substrings of 32
bits, 10,000 queries (seed 1), k = 100.  A step is one mih_knn call over the
whole query batch (tables already built, codes and queries resident in HBM).
Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--config 1..4] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact kNN queries/s, MIH vs GPU linear scan, 1B×64b k=100; p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit integer vector lane-ops per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg: str):
    sys.stderr.write(f"[bench {time.strftime('%H:%M:%S')}] {msg}\n")
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--n", type=int, default=None, help="override the database size")
    ap.add_argument("--nq", type=int, default=None, help="override the number of queries")
    ap.add_argument("--k", type=int, default=None, help="override k (single value)")
    ap.add_argument("--m", type=int, default=None, help="override the number of substrings")
    ap.add_argument("--table-mode", default="auto", choices=["auto", "direct", "sorted", "grouped", "heads"])
    ap.add_argument("--codes-mode", default="auto", choices=["auto", "inline", "indirect", "mixed"])
    ap.add_argument("--inline-tables", type=int, default=0,
                    help="with --codes-mode mixed: tables that keep inline codes")
    ap.add_argument("--linscan-steps", type=int, default=None)
    ap.add_argument("--no-linscan", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=30.0,
                    help="wall-time budget of the CPU oracle sample")
    ap.add_argument("--threads", type=int, default=None, help="host threads for generation/oracle")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch tuning")
    ap.add_argument("--tuning", default="",
                    help="launch tuning fields to set instead of autotuning, e.g. sweep_shift=3,sweep_bits=18")
    ap.add_argument("--autotune-sample", type=int, default=0,
                    help="queries the autotuner times (default: as many as the timed batch); "
                         "they are the rows of the query stream that follow the timed ones")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving loop")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75,0.9",
                    help="fractions of the closed-loop capacity to replay the stream at")
    ap.add_argument("--serve-quantum", type=int, default=1 << 22,
                    help="serving leg: most shell masks a query probes per device round "
                         "(round_masks; 0: whole steps)")
    ap.add_argument("--serve-slots", type=int, default=16384)
    ap.add_argument("--serve-tuning", default="",
                    help="launch tuning fields for the serving leg only, e.g. chunk=8192,lookahead=1 "
                         "(default: the batch tuning with chunk at most 8192)")
    ap.add_argument("--sweep", action="store_true",
                    help="also time the search over a grid of launch tunings")
    ap.add_argument("--m-sweep", default="",
                    help="comma-separated extra m values to build and time (e.g. 3,4)")
    ap.add_argument("--rnn", type=int, default=None,
                    help="radius of the r-neighbour leg (default: the median k-th nearest distance)")
    ap.add_argument("--no-rnn", action="store_true", help="skip the r-neighbour leg")
    ap.add_argument("--no-approx", action="store_true", help="skip the approximate-search leg")
    ap.add_argument("--substring-opt", action="store_true",
                    help="also time the index built with optimised substrings (Section 5.5)")
    ap.add_argument("--choose-m", action="store_true",
                    help="also pick m by timing candidates on 1000 database rows (Section 6)")
    ap.add_argument("--gather-calib", type=float, default=0.0,
                    help="also time 2^27 random 4-byte reads from an array of this many GiB "
                         "(the device's random-line rate, a ceiling for the search kernel)")
    ap.add_argument("--copy-calib", type=float, default=0.0,
                    help="also run one plain device copy of this many GiB (counter calibration)")
    ap.add_argument("--line-calib", type=float, default=0.0,
                    help="also run 2^28 random line reads from an array of this many GiB "
                         "(counter calibration of random reads)")
    ap.add_argument("--no-line-ceiling", action="store_true",
                    help="skip the measurement of the device's random-line rate")
    return ap.parse_args()


def workload(args):
    import datagen
    cfg = dict(datagen.CONFIGS[args.config])
    if args.n is not None:
        cfg["n"] = args.n
    if args.nq is not None:
        cfg["nq"] = args.nq
    if args.m is not None:
        cfg["m"] = args.m
    if args.k is not None:
        cfg["ks"] = (args.k,)
    return cfg


def to_device(codes: np.ndarray, chunk_rows: int = 1 << 24):
    """Copy host codes to a device int64 tensor through a pinned staging buffer."""
    import torch
    n, W = codes.shape
    dev = torch.empty((n, W), dtype=torch.int64, device="cuda")
    if n == 0:
        return dev
    rows = min(chunk_rows, n)
    pinned = torch.empty((rows, W), dtype=torch.int64, pin_memory=True)
    src = codes.view(np.int64)
    for lo in range(0, n, rows):
        hi = min(n, lo + rows)
        pinned[: hi - lo].copy_(torch.from_numpy(src[lo:hi]))
        dev[lo:hi].copy_(pinned[: hi - lo], non_blocking=True)
        torch.cuda.synchronize()
    return dev


def counter_traffic(counters_file, tuning, modes):
    """HBM bytes per launch (device round) of the search from committed
    rocprofv3 counter runs: (bytes, record) for the record whose launch
    tuning matches, or (None, file contents) when the kernel sources or the
    table and codes modes differ from those of the counter runs or no record
    has this tuning, (None, None) when no counters exist for this workload.
    FETCH_SIZE is scaled by its reading for a kernel of known count of random
    64-byte line reads (the search's kind of read), WRITE_SIZE by its reading
    for a plain copy of known size."""
    import hashlib
    path = os.path.join(ROOT, "profiles", counters_file)
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha256_16"]:
        return None, rec
    if tuple(rec.get("modes", ())) != tuple(modes):   # the table and codes modes of the counter runs
        return None, rec
    for r in rec["records"]:
        if all(tuning.get(k) == v for k, v in r["tuning"].items()):
            fetch = np.mean(r["fetch_kib_per_launch"]) * rec["random_line_calibration"]["fetch_factor"]
            write = np.mean(r["write_kib_per_launch"]) * rec["copy_calibration"]["write_factor"]
            return float((fetch + write) * 1024.0), r
    return None, rec


def search_roofline(st, info, n, bits, m, nq, ks, k_list, W, tuning):
    """Roofline object of the multi-index search.  Algorithmic bytes per
    call: 8 B per probed bucket (two 32-bit offsets; 12 B for SORTED tables:
    directory and key), 4 B id + bits/8 B code per candidate, bits/8 B per
    query and 8 B per output entry, over the HIP-event time of the call's
    device rounds, against the 8 TB/s HBM peak.  Counter traffic from the
    committed rocprofv3 runs of the same source and tuning, when they
    exist."""
    per_probe = 12 if info["table_mode"] == "sorted" else 8
    per_cand = 4 + 8 * W
    out_entries = int(np.sum(k_list, dtype=np.int64))
    alg_bytes = (st["probes"] * per_probe + st["candidates"] * per_cand + nq * 8 * W + out_entries * 8)
    kern_ms = st["search_kernel_ms"]
    launches = max(1, st["search_launches"])
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9 if kern_ms > 0 else 0.0
    traffic = None
    lines = None
    if (n, bits, m, nq, tuple(ks)) == (1_000_000_000, 64, 2, 10_000, (100,)):
        traffic, rec = counter_traffic("mih_search_1e9x64_m2_k100_counters.json", tuning,
                                       (info["table_mode"], info["codes_mode"]))
        if traffic is not None:
            # the reads are random 64 B lines; FETCH_SIZE counts each in full
            per_launch = float(np.mean(rec["fetch_kib_per_launch"])) * 1024 / 64
            lines = {"lines_per_launch": round(per_launch),
                     "lines_per_s": round(per_launch / (kern_ms / launches / 1e3))}
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": round(traffic) if traffic is not None else None,
        "traffic_unit": "bytes per launch: FETCH_SIZE scaled by the random-line calibration, "
                        "WRITE_SIZE by the copy calibration",
        "alg_bytes_per_launch": int(alg_bytes / launches),
        "kernel": "device round (search kernels)", "launches_per_step": launches,
        "avg_launch_ms": round(kern_ms / launches, 3),
        "alg_bytes_per_step": int(alg_bytes),
        "per_unit": {"probe_B": per_probe, "candidate_B": per_cand, "query_B": 8 * W, "output_entry_B": 8},
        "probes_per_query": st["probes"] / nq, "candidates_per_query": st["candidates"] / nq,
        "random_lines": lines,
    }


def cpu_description():
    """Host CPU model, sockets and logical CPUs (from /proc/cpuinfo)."""
    model, sockets = None, set()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model is None:
                model = line.split(":", 1)[1].strip()
            elif line.startswith("physical id"):
                sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return {"cpu_model": model, "sockets": max(1, len(sockets)), "logical_cpus": os.cpu_count()}


def serve_bench(mih, idx, kind, bits, k_choices, args, log_fn):
    """Continuous-batching serving loop over the built index.

    Requests (1..4096 queries, log-uniform; one k per request from k_choices)
    arrive as a Poisson stream.  First a closed-loop run (every request
    submitted at once) measures the capacity; then each load level replays
    the stream at that fraction of the capacity and records, per request, the
    time from its arrival to the completion of its last query.
    """
    import torch
    import datagen
    nreq = args.serve_requests
    _, sizes, ks = datagen.request_stream(nreq, 1.0, k_choices)
    total = int(sizes.sum())
    pool = datagen.query_codes(kind, total, bits, first_row=1_000_000)
    dpool = to_device(pool)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    mean_size = float(sizes.mean())

    def run(arrivals):
        srv = mih.Server(idx, max_queries=args.serve_slots)
        tickets, lat = {}, {}
        nxt, t0 = 0, time.perf_counter()
        while len(lat) < nreq:
            now = time.perf_counter() - t0
            while nxt < nreq and arrivals[nxt] <= now:
                tk = srv.submit(dpool[offs[nxt]:offs[nxt + 1]], int(ks[nxt]))
                tickets[tk] = nxt
                nxt += 1
            if len(tickets) > len(lat):
                for tk in srv.step():
                    lat[tickets[tk]] = time.perf_counter() - t0
            elif nxt < nreq:
                time.sleep(max(0.0, min(0.001, arrivals[nxt] - now)))
        end = max(lat.values())
        st = srv.stats()
        # results of a few requests in the mix against the same queries alone
        same = True
        for r in (0, nreq // 2, nreq - 1):
            tk = [t for t, i in tickets.items() if i == r][0]
            mi, md = srv.result(tk)
            bi, bd = idx.knn(dpool[offs[r]:offs[r + 1]], int(ks[r]))
            same &= bool(torch.equal(mi, bi) and torch.equal(md, bd))
        srv.close()
        lat_ms = np.array([(lat[i] - arrivals[i]) * 1e3 for i in range(nreq)])
        return lat_ms, end, st, same

    lat, end, st, same = run(np.zeros(nreq))
    closed_qps = total / end
    log_fn(f"serving closed loop: {nreq} requests, {total} queries in {end:.2f}s -> "
           f"{closed_qps:,.0f} queries/s; rounds {st['rounds']}; mix == alone: {same}")
    out = {"requests": nreq, "queries": total, "mean_request_size": round(mean_size, 1),
           "k_choices": list(k_choices), "slots": args.serve_slots,
           "closed_loop_qps": round(closed_qps, 1), "closed_loop_same_as_alone": same, "loads": []}
    warm = min(args.serve_warmup, nreq // 4)
    for load in [float(x) for x in args.serve_loads.split(",") if x]:
        rate = load * closed_qps / mean_size
        arrivals, _, _ = datagen.request_stream(nreq, rate, k_choices)
        arrivals = arrivals - arrivals[0]
        lat, end, st, same = run(arrivals)
        body = lat[warm:]
        wsz = sizes[warm:]
        qps = total / end
        # per query: a query's results are ready when its request completes
        rec = {"load": load, "rate_req_per_s": round(rate, 2), "p50_ms": round(pct(body, 50), 2),
               "p99_ms": round(pct(body, 99), 2), "mean_ms": round(float(body.mean()), 2),
               "per_query_p50_ms": round(weighted_pct(body, wsz, 50), 2),
               "per_query_p99_ms": round(weighted_pct(body, wsz, 99), 2),
               "qps": round(qps, 1), "rounds": st["rounds"], "same_as_alone": same}
        out["loads"].append(rec)
        log_fn(f"serving at {load:.0%} load ({rate:.1f} req/s): p50 {rec['p50_ms']} ms, "
               f"p99 {rec['p99_ms']} ms (per query {rec['per_query_p50_ms']} / {rec['per_query_p99_ms']} ms), "
               f"{qps:,.0f} queries/s, mix == alone: {same}")
    return out


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


def weighted_pct(a, w, q):
    """Percentile of values a with integer weights w (each request counted
    once per query it carries)."""
    if not len(a):
        return None
    order = np.argsort(a, kind="stable")
    cw = np.cumsum(np.asarray(w, dtype=np.float64)[order])
    i = int(np.searchsorted(cw, q / 100.0 * cw[-1], side="left"))
    return float(np.asarray(a)[order][min(i, len(a) - 1)])


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU search; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    import paper_1307_2982_amd as mih

    mih.load()   # fails loudly if libmih.so is missing
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    threads = args.threads or max(1, min(os.cpu_count() or 1, 16))
    cfg = workload(args)
    n, bits, m, nq = cfg["n"], cfg["bits"], cfg["m"], cfg["nq"]
    W = bits // 64
    kind = cfg["kind"]
    ks = cfg["ks"]
    mixed_k = len(ks) > 1
    log(f"workload {cfg['name']}: n={n} bits={bits} m={m} nq={nq} k={ks} threads={threads}")

    t0 = time.time()
    # large clustered sets are generated on the device (bit-identical to the
    # host generator); the host copy the oracle needs is made on demand
    device_gen = kind == "clustered" and n >= 20_000_000
    codes = None if device_gen else datagen.db_codes(kind, n, bits, threads=threads)
    queries = datagen.query_codes(kind, nq, bits, threads=threads)
    if mixed_k:
        kq = datagen.choice_u32(nq, ks, datagen.SEED_K)
        k_arg = kq.tolist()
        k_list = kq
    else:
        k_arg = int(ks[0])
        k_list = np.full(nq, ks[0], dtype=np.uint32)
    log(f"generated codes on the host in {time.time() - t0:.1f}s")
    t0 = time.time()
    dc = datagen.codes_device(kind, n, bits, datagen.SEED_DB_CLUSTERED) if device_gen else to_device(codes)
    dq = to_device(queries)
    log(f"copied to the device in {time.time() - t0:.1f}s")

    t0 = time.time()
    idx = mih.build(dc, m, table_mode=args.table_mode, codes_mode=args.codes_mode,
                    inline_tables=args.inline_tables)
    torch.cuda.synchronize()
    info = idx.info()
    log(f"built index in {time.time() - t0:.2f}s ({info['table_mode']}/{info['codes_mode']}, "
        f"{info['inline_tables']} of {m} tables with inline codes, {info['device_bytes'] / 2**30:.1f} GiB)")

    if args.copy_calib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the counter readings of the search kernel
        words = int(args.copy_calib * 2**30) // 8
        a = torch.ones(words, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {words * 8} bytes read and written")
        del a, b

    if args.line_calib > 0:
        # 2^28 random line reads of known count: the FETCH_SIZE counter of
        # this kernel calibrates the counter for the search kernel's reads
        arr = torch.ones(int(args.line_calib * 2**30) // 8, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        r = mih.random_read_rate(arr, 1 << 28, 8)
        log(f"line calibration: {r['reads']} random line reads in {r['ms']:.2f} ms")
        del arr
        torch.cuda.synchronize()

    gather = None
    if args.gather_calib > 0:
        # independent random reads: every one touches its own line, as the
        # probes and candidate reads of the search kernel do
        words = int(args.gather_calib * 2**30) // 4
        arr = torch.zeros(words, dtype=torch.int32, device="cuda")
        g = torch.Generator(device="cuda").manual_seed(11)
        nread = 1 << 27
        pos = torch.randint(0, words, (nread,), device="cuda", generator=g)
        torch.take(arr, pos)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            torch.take(arr, pos)
        e1.record()
        torch.cuda.synchronize()
        g_ms = e0.elapsed_time(e1) / 3
        gather = {"array_GiB": args.gather_calib, "reads": nread, "ms": round(g_ms, 3),
                  "random_reads_per_s": round(nread / (g_ms / 1e3), 1),
                  "note": "torch.take over int64 positions: per read 8 B of position and 4 B of "
                          "output stream sequentially beside the random 4 B read"}
        log(f"random reads: {nread} in {g_ms:.2f} ms -> {nread / (g_ms / 1e3) / 1e9:.1f} G reads/s")
        del arr, pos
        torch.cuda.synchronize()

    # ---------------- launch tuning picked on other queries of the same
    # distribution, as many as the timed batch unless told otherwise (how
    # much each round can run ahead depends on the batch size)
    tuned = None
    ns = 0
    if args.tuning:
        idx.set_tuning(**{f: int(v) for f, v in (kv.split("=") for kv in args.tuning.split(","))})
        log(f"tuning set: {idx.get_tuning()}")
    elif not args.no_autotune:
        t = time.time()
        ns = args.autotune_sample or nq
        tq = to_device(datagen.query_codes(kind, ns, bits, first_row=nq, threads=threads))
        tk = datagen.choice_u32(ns, ks, datagen.SEED_K, first=nq).tolist() if mixed_k else k_arg
        tuned = idx.autotune(tq, tk)
        del tq
        log(f"autotuned on {ns} other queries in {time.time() - t:.1f}s: {tuned}")

    # ---------------- multi-index hashing
    for _ in range(args.warmup):
        idx.knn(dq, k_arg)
    torch.cuda.synchronize()
    step_ms, stats = [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ids, dists, st = idx.knn(dq, k_arg, stats=True)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t) * 1e3)
        stats.append(st)
    mih_ms = float(np.mean(step_ms))
    mih_qps = nq / (mih_ms / 1e3)
    log(f"MIH: {mih_ms:.1f} ms/step -> {mih_qps:,.0f} queries/s; last step {stats[-1]}")

    # ---------------- radius histogram: each query's k-th nearest distance
    # (the radius its search had to reach), per value of k
    dk = dists.reshape(-1).cpu().numpy().view(np.uint32)
    ends = np.cumsum(k_list.astype(np.int64)) - 1
    radius_hist = {}
    for kv in sorted(set(int(x) for x in k_list)):
        if kv == 0:
            continue
        sel = ends[(k_list == kv)]
        r = dk[sel]
        r = r[r != 0xFFFFFFFF]
        vals, cnts = np.unique(r, return_counts=True)
        radius_hist[str(kv)] = {str(int(v)): int(c) for v, c in zip(vals, cnts)}

    # ---------------- roofline of the search (one device round = one launch
    # of the graph holding the search kernels)
    st = stats[-1]
    roofline = search_roofline(st, info, n, bits, m, nq, ks, k_list, W, idx.get_tuning())
    ceiling = None
    if not args.no_line_ceiling:
        # the device's random-line rate, measured with several loads per lane
        # in flight, over an array far larger than the caches
        free = torch.cuda.mem_get_info()[0]
        gib = min(16, max(1, int(free * 0.5) >> 30))
        arr = torch.empty((gib << 30) // 8, dtype=torch.int64, device="cuda")
        arr.fill_(1)
        rr = [mih.random_read_rate(arr, 1 << 28, d) for d in (4, 8, 16)]
        best = max(rr, key=lambda r: r["reads_per_s"])
        ceiling = {"array_GiB": gib, "reads": best["reads"], "depth": best["depth"],
                   "lines_per_s": round(best["reads_per_s"]),
                   "kernel": "random_lines_kernel (mih_random_read_rate)"}
        del arr
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"random-line ceiling: {best['reads_per_s'] / 1e9:.1f} G lines/s (depth {best['depth']}, {gib} GiB)")
        if roofline.get("random_lines"):
            rl = roofline["random_lines"]
            rl["ceiling_lines_per_s"] = ceiling["lines_per_s"]
            rl["frac_of_ceiling"] = round(rl["lines_per_s"] / ceiling["lines_per_s"], 4)

    # ---------------- launch tunings (speed only; results must not change)
    sweep = None
    if args.sweep:
        base_t = idx.get_tuning()
        sweep = []
        grid = []
        for occ in ((0, 1) if info["table_mode"] == "direct" else (0,)):
            for J in (4, 8, 16):
                for chunk in (64 * J * 8, 64 * J * 32, 64 * J * 128):
                    grid.append(dict(probes_per_lane=J, chunk=chunk, blocks_per_cu=0,
                                     occupancy_filter=occ, sweep_shift=0, sweep_bits=18))
        for shift in (2, 3, 4):
            for sbits in (16, 18, 20, 22):
                for J in (8,):
                    grid.append(dict(probes_per_lane=J, chunk=64 * J * 32, blocks_per_cu=0,
                                     occupancy_filter=base_t["occupancy_filter"], sweep_shift=shift,
                                     sweep_bits=sbits))
        for tg in grid:
            idx.set_tuning(**tg)
            idx.knn(dq, k_arg)
            torch.cuda.synchronize()
            t = time.perf_counter()
            si, sd, sst = idx.knn(dq, k_arg, stats=True)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3
            same = bool(torch.equal(si, ids) and torch.equal(sd, dists))
            sweep.append(dict(tg, ms=round(ms, 2), kernel_ms=round(sst["search_kernel_ms"], 2),
                              same_result=same))
            log(f"tuning {tg}: {ms:.1f} ms same={same}")
        idx.set_tuning(**base_t)

    m_sweep = None
    if args.m_sweep:
        m_sweep = []
        for mm in [int(x) for x in args.m_sweep.split(",") if x]:
            ix2 = mih.build(dc, mm, table_mode=args.table_mode,
                            codes_mode="auto" if args.codes_mode == "mixed" else args.codes_mode)
            ix2.knn(dq, k_arg)
            torch.cuda.synchronize()
            t = time.perf_counter()
            si, sd, sst = ix2.knn(dq, k_arg, stats=True)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3
            inf2 = ix2.info()
            m_sweep.append({"m": mm, "ms": round(ms, 2), "queries_per_s": round(nq / (ms / 1e3), 1),
                            "same_result": bool(torch.equal(si, ids) and torch.equal(sd, dists)),
                            "probes_per_query": sst["probes"] / nq,
                            "candidates_per_query": sst["candidates"] / nq,
                            "table_mode": inf2["table_mode"], "codes_mode": inf2["codes_mode"],
                            "index_GiB": round(inf2["device_bytes"] / 2**30, 2)})
            log(f"m={mm}: {ms:.1f} ms -> {nq / (ms / 1e3):,.0f} q/s, same={m_sweep[-1]['same_result']}")
            ix2.close()
            del ix2
            torch.cuda.synchronize()

    subopt = None
    if args.substring_opt:
        # Section 5.5: the same index with the greedy bit order from a sample
        t = time.time()
        sample = min(n, 1_000_000)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        counts = mih.bit_cooccurrence(dc[:sample])
        cooc_ms = (time.perf_counter() - tc) * 1e3
        order = mih.greedy_bit_order(counts, sample, m, 0)
        ix2 = mih.build(dc, m, table_mode=args.table_mode, codes_mode=args.codes_mode, bit_order=order,
                        inline_tables=args.inline_tables)
        if tuned is not None:
            ix2.set_tuning(**tuned)
        ix2.knn(dq, k_arg)
        torch.cuda.synchronize()
        oms = []
        for _ in range(max(1, args.steps)):
            t2 = time.perf_counter()
            oi2, od2, ost = ix2.knn(dq, k_arg, stats=True)
            torch.cuda.synchronize()
            oms.append((time.perf_counter() - t2) * 1e3)
        o_ms = float(np.mean(oms))
        subopt = {"sample": sample, "cooccurrence_ms": round(cooc_ms, 2), "ms": round(o_ms, 2),
                  "queries_per_s": round(nq / (o_ms / 1e3), 1), "consecutive_ms": round(mih_ms, 2),
                  "speedup_over_consecutive": round(mih_ms / o_ms, 3),
                  "same_result": bool(torch.equal(oi2, ids) and torch.equal(od2, dists)),
                  "candidates_per_query": ost["candidates"] / nq,
                  "consecutive_candidates_per_query": stats[-1]["candidates"] / nq}
        log(f"optimised substrings: {o_ms:.1f} ms vs {mih_ms:.1f} ms consecutive "
            f"({subopt['candidates_per_query']:,.0f} vs {subopt['consecutive_candidates_per_query']:,.0f} "
            f"candidates/query), same={subopt['same_result']}, counts in {cooc_ms:.1f} ms; "
            f"{time.time() - t:.1f}s in all")
        ix2.close()
        del ix2
        torch.cuda.synchronize()

    chosen_m = None
    if args.choose_m:
        kk = int(ks[-1]) if mixed_k else int(ks[0])
        t = time.time()
        best_m, trials = mih.choose_m(dc, kk, validation=1000, seed=9, table_mode=args.table_mode,
                                      codes_mode="auto" if args.codes_mode == "mixed" else args.codes_mode)
        chosen_m = {"k": kk, "validation": "1000 database rows (seeded permutation)", "best_m": best_m,
                    "model_radius": mih.model_radius(n, bits, kk), "heuristic_b_over_log2n":
                    round(bits / np.log2(n), 3), "trials": trials}
        log(f"choose m (k={kk}): best m={best_m} in {time.time() - t:.1f}s; " +
            ", ".join(f"m={t_['m']}: {t_['search_ms']:.1f} ms (model {t_['model_cost']:.3g})" for t_ in trials))
        torch.cuda.synchronize()

    # ---------------- serving loop (continuous batching)
    serving = None
    if not args.no_serve:
        # the serving streams carry k from {1,10,100,1000} (1e9 x 64-bit) or
        # the configuration's own k values
        serve_k = datagen.CONFIGS[args.config]["ks"] if args.config != 4 else (1, 10, 100, 1000)
        if args.config == 5:
            serve_k = (1, 10, 100)
        batch_t = idx.get_tuning()
        # rounds of a serving loop often hold few queries: smaller work items
        # spread them over more waves (the batch-tuned chunk is for full
        # batches); a work quantum keeps the rounds short, so that a request
        # arriving meanwhile does not wait for whole large steps of others
        # (steps larger than the quantum are not swept: a sweep runs a whole
        # step); requests go through the rounds (the one-launch path is for
        # mih_knn calls)
        serve_t = {"chunk": min(batch_t["chunk"], 8192), "round_masks": args.serve_quantum}
        if args.serve_tuning:
            serve_t = {f: int(v) for f, v in (kv.split("=") for kv in args.serve_tuning.split(","))}
        idx.set_tuning(**serve_t)
        log(f"serving tuning: {idx.get_tuning()}")
        serving = serve_bench(mih, idx, kind, bits, serve_k, args, log)
        serving["tuning"] = idx.get_tuning()
        idx.set_tuning(**batch_t)

    # ---------------- linear scan
    lin = None
    if not args.no_linscan:
        lsteps = args.linscan_steps if args.linscan_steps is not None else args.steps
        li, ld = mih.linscan_knn(dc, dq, k_arg)
        torch.cuda.synchronize()
        parity_mih_vs_linscan = bool(torch.equal(li, ids) and torch.equal(ld, dists))
        lms, lst = [], None
        for _ in range(max(1, lsteps)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            li, ld, lst = mih.linscan_knn(dc, dq, k_arg, stats=True)
            torch.cuda.synchronize()
            lms.append((time.perf_counter() - t) * 1e3)
        lin_ms = float(np.mean(lms))
        lin_qps = nq / (lin_ms / 1e3)
        ops = lst["pairs"] * 4 * W   # per 64-bit word: 2 xor + 2 bit counts (32-bit lanes)
        scan_ms = lst["scan_kernel_ms"]
        achieved_ops = ops / (scan_ms / 1e3) / 1e12 if scan_ms > 0 else 0.0
        lin = {
            "value": round(lin_qps, 1), "unit": "queries/s", "ms_per_step": round(lin_ms, 2),
            "steps": len(lms), "speedup_mih_over_linscan": round(mih_qps / lin_qps, 2),
            "parity_with_mih": parity_mih_vs_linscan,
            "roofline": {"bound": "alu", "achieved": round(achieved_ops, 2), "peak": round(VALU_PEAK_TOPS, 1),
                         "unit": "Tops/s", "frac": round(achieved_ops / VALU_PEAK_TOPS, 4),
                         "kernel": "linscan_kernel", "ops_per_pair": 4 * W,
                         "kernel_ms": round(scan_ms, 2), "sample_kernel_ms": round(lst["sample_kernel_ms"], 2)},
            "appended_per_query": lst["appended"] / nq, "reruns": lst["reruns"],
        }
        log(f"linscan: {lin_ms:.1f} ms/step -> {lin_qps:,.0f} queries/s; parity with MIH: "
            f"{parity_mih_vs_linscan}; kernel {scan_ms:.1f} ms = {achieved_ops:.2f} Tops/s")

    # ---------------- r-neighbour search: MIH vs linear scan, same queries
    rnn = None
    if not args.no_rnn:
        # default radius: the median distance of the last of each query's k
        # nearest codes, so that a query has about k r-neighbours
        kth = dists.reshape(-1).cpu().numpy().view(np.uint32)
        if not mixed_k:
            kth = kth.reshape(nq, -1)[:, -1]
        R = args.rnn if args.rnn is not None else int(np.median(kth[kth != 0xFFFFFFFF]))
        idx.rnn(dq, R)
        torch.cuda.synchronize()
        rms = []
        for _ in range(max(1, args.steps)):
            t = time.perf_counter()
            ro, ri, rd, rst = idx.rnn(dq, R, stats=True)
            torch.cuda.synchronize()
            rms.append((time.perf_counter() - t) * 1e3)
        r_ms = float(np.mean(rms))
        rnn = {"r": R, "mih_queries_per_s": round(nq / (r_ms / 1e3), 1), "mih_ms": round(r_ms, 2),
               "results_per_query": int(ro[-1]) / nq, "probes_per_query": rst["probes"] / nq,
               "candidates_per_query": rst["candidates"] / nq, "reruns": rst["reruns"]}
        if not args.no_linscan:
            t = time.perf_counter()
            lo_, li_, ld_ = mih.linscan_rnn(dc, dq, R)
            torch.cuda.synchronize()
            l_ms = (time.perf_counter() - t) * 1e3
            rnn.update({"linscan_queries_per_s": round(nq / (l_ms / 1e3), 1), "linscan_ms": round(l_ms, 2),
                        "speedup_mih_over_linscan": round(l_ms / r_ms, 2),
                        "parity_with_linscan": bool(torch.equal(ro, lo_) and torch.equal(ri, li_)
                                                    and torch.equal(rd, ld_))})
            del lo_, li_, ld_
        log(f"r-neighbours r={R}: MIH {r_ms:.1f} ms ({rnn['mih_queries_per_s']:,.0f} q/s), "
            f"{rnn['results_per_query']:.1f} results/query; linscan {rnn.get('linscan_ms')} ms, "
            f"same={rnn.get('parity_with_linscan')}")

    # ---------------- approximate variants (Section 7): speed and recall
    approx = None
    if not args.no_approx:
        approx = []
        exact = ids.reshape(-1).cpu().numpy().view(np.uint32)
        off = np.concatenate([[0], np.cumsum(k_list.astype(np.int64))])
        kth = dists.reshape(-1).cpu().numpy().view(np.uint32)[off[1:] - 1]
        med = int(np.median(kth[kth != 0xFFFFFFFF])) if nq else 0
        cand = stats[-1]["candidates"] / max(nq, 1)
        for max_radius, budget in [(med - 2, 0), (med - 1, 0), (None, int(cand / 10)), (None, int(cand / 3))]:
            idx.knn_approx(dq, k_arg, max_radius=max_radius, max_candidates=budget)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ai, ad, ast = idx.knn_approx(dq, k_arg, max_radius=max_radius, max_candidates=budget, stats=True)
            torch.cuda.synchronize()
            a_ms = (time.perf_counter() - t) * 1e3
            got = ai.reshape(-1).cpu().numpy().view(np.uint32)
            hits = 0
            for q in range(nq):
                e = exact[off[q]:off[q + 1]]
                hits += len(np.intersect1d(got[off[q]:off[q + 1]], e[e != 0xFFFFFFFF]))
            recall = hits / max(1, int((exact != 0xFFFFFFFF).sum()))
            approx.append({"max_radius": max_radius, "max_candidates": budget, "ms": round(a_ms, 2),
                           "queries_per_s": round(nq / (a_ms / 1e3), 1), "recall": round(recall, 4),
                           "candidates_per_query": ast["candidates"] / max(nq, 1)})
            log(f"approximate radius={max_radius} budget={budget}: {a_ms:.1f} ms "
                f"({nq / (a_ms / 1e3):,.0f} q/s), recall {recall:.4f}")

    # ---------------- CPU oracle: bounded sample, also a full-size parity check
    cpu = None
    parity_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        if codes is None:
            t = time.time()
            codes = dc.cpu().numpy().view(np.uint64)
            log(f"copied the codes to the host for the oracle in {time.time() - t:.1f}s")
        gi = ids.reshape(-1).cpu().numpy().view(np.uint32)
        gd = dists.reshape(-1).cpu().numpy().view(np.uint32)
        off = np.concatenate([[0], np.cumsum(k_list.astype(np.int64))])
        rng = np.random.default_rng(123)
        order = rng.permutation(nq)
        done, spent, ok = 0, 0.0, True
        half = args.cpu_seconds / 2
        while done < nq and spent < half:
            sel = order[done: done + threads]
            t = time.perf_counter()
            oi, od = oracle.knn(codes, queries[sel], k_list[sel], threads=threads)
            spent += time.perf_counter() - t
            used = oracle.knn.last_threads
            o = 0
            for q in sel:
                kq_ = int(k_list[q])
                ok &= bool(np.array_equal(oi[o:o + kq_], gi[off[q]:off[q + 1]]) and
                           np.array_equal(od[o:o + kq_], gd[off[q]:off[q + 1]]))
                o += kq_
            done += len(sel)
        # the rate on at least 1000 queries (all of them when fewer) within
        # the other half of the budget: against a prefix of the codes when
        # the whole set would take longer, scaled by n / prefix (the
        # oracle's time per query is linear in the number of codes)
        rate_q = order[:min(nq, 1000)]
        per_q = spent / max(done, 1)
        n_s = n if per_q * len(rate_q) <= half else max(1 << 20, int(n * half / (per_q * len(rate_q))))
        n_s = min(n, n_s)
        t = time.perf_counter()
        oracle.knn(codes[:n_s], queries[rate_q], k_list[rate_q], threads=threads)
        rate_s = time.perf_counter() - t
        rate_value = len(rate_q) / rate_s * (n_s / n)
        # the single-thread rate, for the paper's one-core regime: queries
        # of the same subset one at a time on one thread, for about 3 s
        one_done, one_spent = 0, 0.0
        while one_done < nq and one_spent < 3.0:
            q = order[one_done]
            t = time.perf_counter()
            oracle.knn(codes, queries[q:q + 1], k_list[q:q + 1], threads=1)
            one_spent += time.perf_counter() - t
            one_done += 1
        cpu = {"value": round(rate_value, 3), "unit": "queries/s", "cores": int(used),
               "kind": "oracle",
               "sample": (f"{len(rate_q)} of the {nq} queries (seeded random subset), same k, against "
                          + (f"all {n} codes" if n_s == n else
                             f"the first {n_s} of the {n} codes, rate scaled by {n_s}/{n}")
                          + f"; {rate_s:.1f} s wall on {used} host threads"),
               "sample_queries": len(rate_q), "sample_codes": n_s, "threads": int(used),
               "full_set_value": round(done / spent, 3),
               "full_set_sample": f"{done} queries against all {n} codes (checked against MIH), {spent:.1f} s",
               "single_thread_value": round(one_done / one_spent, 4),
               "single_thread_sample": f"{one_done} queries one at a time on 1 thread, {one_spent:.1f} s",
               **cpu_description()}
        parity_oracle = {"queries_checked": done, "bit_exact": ok}
        log(f"oracle: {done} queries in {spent:.1f}s on {used} threads; MIH == oracle: {ok}")
        if rnn is not None:
            # two queries' r-neighbour lists against the oracle's definition
            roff = ro.cpu().numpy()
            rid = ri.cpu().numpy().view(np.uint32)
            rdd = rd.cpu().numpy().view(np.uint32)
            rok = True
            for q in order[:2]:
                oi, od = oracle.rnn(codes, queries[q], rnn["r"])
                rok &= bool(np.array_equal(oi, rid[roff[q]:roff[q + 1]]) and
                            np.array_equal(od, rdd[roff[q]:roff[q + 1]]))
            rnn["parity_with_oracle_2_queries"] = rok
            log(f"r-neighbours of 2 queries == oracle: {rok}")

    # the headline latency: the 50% load level when it was run, else the first
    headline_load = None
    if serving and serving["loads"]:
        half = [x for x in serving["loads"] if abs(x["load"] - 0.5) < 1e-9]
        headline_load = half[0] if half else serving["loads"][0]
    out = {
        "metric": METRIC,
        "value": round(mih_qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mih_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": cfg["name"] + (f", {nq} queries, k={ks[0]}" if not mixed_k else
                                       f", {nq} queries, k drawn from {list(ks)}"),
            "n": n, "bits": bits, "m": m, "nq": nq, "k": list(ks),
            "table_mode": info["table_mode"], "codes_mode": info["codes_mode"],
            "inline_tables": info["inline_tables"],
            "index_GiB": round(info["device_bytes"] / 2**30, 2), "build_ms": round(info["build_ms"], 1),
        },
        "p50_ms": headline_load["p50_ms"] if headline_load else None,
        "p99_ms": headline_load["p99_ms"] if headline_load else None,
        "latency_note": ("per request (arrival to last result), serving loop at "
                         f"{headline_load['load']:.0%} of closed-loop capacity" if headline_load else None),
        "roofline": roofline,
        "serving": serving,
        "linscan": lin,
        "rnn": rnn,
        "approximate": approx,
        "cpu_baseline": cpu,
        "parity": {"mih_vs_oracle_sample": parity_oracle,
                   "mih_vs_linscan_all": lin["parity_with_mih"] if lin else None},
        "mih_step_ms": [round(x, 2) for x in step_ms],
        "radius_histogram": radius_hist,
        "tuning": idx.get_tuning(),
        "autotuned": tuned is not None,
        "autotune_queries": ns,
        "tuning_sweep": sweep,
        "m_sweep": m_sweep,
        "choose_m": chosen_m,
        "substring_optimisation": subopt,
        "random_read_calibration": gather,
        "random_line_ceiling": ceiling,
        "mih_stats": {k_: (round(v, 3) if isinstance(v, float) else v) for k_, v in stats[-1].items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
