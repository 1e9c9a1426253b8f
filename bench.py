#!/usr/bin/env python3
"""Benchmark of the MRG32k3a stream library on one MI355X.

Headline workload (plain bulk fill): 2^20 streams spaced 2^127 apart from a
64-bit master seed, 4096 uint32 outputs per stream per step, stream-major
(a [2^20, 4096] array, 16 GiB), the stream states resident on the device and
advanced by every step.  One step = one pass of the generation path over the
whole batch.  The output buffer is allocated before timing.

Printed: ONE JSON line with the headline value plus
  roofline      -- HBM-write roofline of the fill kernel (bytes it must write
                   per launch / its average duration measured with HIP events
                   on the launch stream), and the counter-measured traffic;
  cpu_baseline  -- the CPU oracle (plain single-threaded C) timed on a bounded
                   sample of the same workload;
  extra         -- FP32 and interleaved fills, jump and create timings, the
                   batched request mix against per-request launches, and
                   p50/p99 latency of the serving engine under Poisson
                   arrivals.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--engine 0|1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "uint32 Gsamples/s (% HBM write roofline), batched vs plain; p50/p99 latency"
# rocprofv3 counters of the headline kernel, taken on the kernel sources whose
# hash is recorded with them: HBM bytes per launch (FETCH_SIZE + WRITE_SIZE,
# scaled by a copy-kernel calibration) and VALU wave instructions per launch
# (SQ_INSTS_VALU).  They are reported only while the sources still hash the
# same; after any change to the kernel they read null until profiled again.
COUNTERS = {
    "traffic": 17230931544,
    "valu_insts": 1079772685,
    "source": "profiles/fill_coop_u32_16lanes_2p20x4096.md",
    "kernel_sources_sha256": "fdf1d4b82e6f25c887b48724d87e72e9abcc9c19d8af3da9f299ede20bbf4698",
}
KERNEL_SOURCES = ["include/mrg_arith.hpp", "include/mrg32k3a_device.h",
                  "paper_1412_8266_amd/csrc/gen_device.hpp", "paper_1412_8266_amd/csrc/kernels.hip",
                  "paper_1412_8266_amd/csrc/kernels.h"]
SIMDS, PEAK_SCLK_MHZ = 1024, 2400  # MI355X: 256 CUs x 4 SIMDs, 2.4 GHz peak shader clock


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counters_current():
    """The recorded counters if they were taken on the current kernel sources."""
    sha = COUNTERS["kernel_sources_sha256"]
    return sha is not None and sha == kernel_sources_sha256()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--engine", type=int, default=None, help="0 integer, 1 binary64")
    ap.add_argument("--tile-bytes", type=int, default=None)
    ap.add_argument("--strategy", type=int, default=None, help="0 auto, 1 lane/stream, 2 wave/stream")
    ap.add_argument("--coop-wgs-per-cu", type=int, default=None)
    ap.add_argument("--coop-lanes", type=int, default=None, help="lanes per stream: 64, 32 or 16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched request mix")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched request mix (prints its JSON object; for profiling)")
    ap.add_argument("--serve-step", type=float, default=0.1,
                    help="arrival-rate multiple step of the sustainable-rate sweep (4 s windows, "
                         "from 1 + step up to the first rate that falls behind)")
    ap.add_argument("--serve-max-speed", type=float, default=3.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the replayed arrival trace (the whole trace is 60 s)")
    ap.add_argument("--quick", action="store_true", help="headline only (for profiling)")
    ap.add_argument("--rows-only", action="store_true",
                    help="only the lane-per-stream fills of short rows")
    ap.add_argument("--partitions-only", action="store_true",
                    help="only the leapfrog, random-spacing and Philox lines (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy 3 times (to scale HBM counters)")
    return ap.parse_args()


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return per, wall


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(streams: int, n: int, chunk: int = 1 << 13):
    """The C oracle (plain, single-threaded) on the first `streams` streams of
    the headline workload, fill only, in chunks of `chunk` streams (outputs
    discarded), then the same streams split over up to 16 threads (the
    oracle's C code runs outside the interpreter lock)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    from paper_1412_8266_amd import workloads as wl
    base = oracle.seed_from_master(wl.MASTER_SEED)
    st = oracle.streams_adjacent(base, 0, streams)
    starts = list(range(0, streams, chunk))

    def run(ids):
        for c0 in ids:
            out, _ = oracle.fill(st[c0:c0 + chunk], n, oracle.U32)
            del out

    t0 = time.perf_counter()
    run(starts)
    dt = time.perf_counter() - t0
    cores = max(1, min(os.cpu_count() or 1, 16))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(run, [starts[i::cores] for i in range(cores)]))
    dt_all = time.perf_counter() - t0
    return {
        "value": streams * n / dt / 1e9,
        "unit": "Gsamples/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d of the 2^20 streams x %d uint32 outputs (%d samples), stream-major; "
                  "single-threaded C oracle, fill only (start states precomputed), %d-stream "
                  "chunks" % (streams, n, streams * n, chunk),
        "seconds": dt,
        "all_cores": {"value": streams * n / dt_all / 1e9, "cores": cores, "seconds": dt_all},
        "cpu": _cpu_model(),
        "host_cpus": os.cpu_count(),
    }


def batched(mg, wl, torch, stream, reps):
    """The 10,000-request mix (stream counts log-uniform in [1, 4096], lengths
    log-uniform in [1, 2^20] per stream, dtypes mixed) as one persistent
    graph launch against one launch per request.  The batch writes about
    1.8 TiB per run, more than HBM holds, so every request's output is placed
    in a 32 GiB arena at a rolling offset (timing only: overlapping requests
    overwrite each other; the outputs are verified in the tests)."""
    req = wl.c4_requests()
    nbytes = req.bytes()
    arena_bytes = 32 << 30
    assert int(nbytes.max()) <= arena_bytes
    arena = torch.empty(arena_bytes // 8, dtype=torch.float64, device="cuda")
    base = arena.data_ptr()
    rows, off = [], 0
    for i in range(len(req)):
        b = int(nbytes[i])
        if off + b > arena_bytes:
            off = 0
        rows.append((int(req.first_stream[i]), int(req.n_streams[i]), int(req.length[i]), 0,
                     base + off, int(req.dtype[i]), 0))
        off = (off + b + 255) // 256 * 256
    S = int(req.n_streams.sum())
    ss = mg.StreamSet(S, master_seed=wl.MASTER_SEED)
    b = mg.Batch(ss, rows)
    # segment length (tile), persistent waves, claiming schedule, and the
    # stream length above which a stream gets a whole wave instead of a lane
    cands = [mg.batch_config(segment_bytes=sb, waves_per_cu=w, schedule=sc, wave_min_bytes=wm)
             for sb, w, sc, wm in [(256 << 10, 16, 1, 16 << 10), (1 << 20, 16, 1, 16 << 10),
                                   (256 << 10, 8, 1, 16 << 10), (1 << 20, 8, 1, 16 << 10),
                                   (64 << 10, 16, 1, 16 << 10), (256 << 10, 8, 2, 16 << 10),
                                   (1 << 20, 16, 1, 4 << 10), (1 << 20, 16, 1, 32 << 10),
                                   (1 << 20, 16, 1, 64 << 10)]]
    t0 = time.perf_counter()
    best, cand_ms = b.autotune(cands, reps=1)
    tune_s = time.perf_counter() - t0
    info = b.info()
    per_b, _ = timed(lambda: b.run(), reps, 1, stream)
    import numpy as np
    done_all = b.request_times()  # of the last graph run
    done = np.sort(done_all[req.samples() > 0])
    # the row items (streams shorter than wave_min_bytes, one lane each) lead
    # the first launch; when the last of them ended, from the run's start
    row = (nbytes // np.maximum(req.n_streams, 1) < info["wave_min_bytes"]) & (req.samples() > 0)
    row_bytes = int(nbytes[row].sum())
    row_done = float(done_all[row].max()) if row.any() else 0.0
    per_r, _ = timed(lambda: b.run_per_request(), reps, 1, stream)
    # the same row requests as a batch of their own (one launch of row items
    # only), under the chosen plan
    alone = None
    if row.any():
        cfg = mg.batch_config(segment_bytes=info["segment_bytes"],
                              wave_min_bytes=info["wave_min_bytes"],
                              waves_per_cu=info["waves_per_cu"], schedule=info["schedule"])
        br = mg.Batch(ss, [rows[i] for i in np.nonzero(row)[0]], cfg)
        per_a, _ = timed(lambda: br.run(), 5, 2, stream)
        ms_a = sum(per_a) / len(per_a)
        alone = {"ms": round(ms_a, 4), "items": br.info()["items"],
                 "TB_s": round(row_bytes / ms_a / 1e9, 3)}
        br.close()
    ms_b = sum(per_b) / len(per_b)
    ms_r = sum(per_r) / len(per_r)
    samples = info["samples"]
    out = {
        "requests": len(req),
        "streams": S,
        "samples_per_run": samples,
        "bytes_per_run": info["bytes"],
        "work_items": info["items"],
        "batched_graph_ms": round(ms_b, 3),
        "per_request_launches_ms": round(ms_r, 3),
        "batched_Gsamples_s": round(samples / ms_b / 1e6, 2),
        "per_request_Gsamples_s": round(samples / ms_r / 1e6, 2),
        "batched_over_per_request": round(ms_r / ms_b, 3),
        # device wall clock from the run's first workgroup start to each
        # request's last work item, over the 10,000 requests
        "request_completion_ms": {"p50": round(float(done[len(done) // 2]), 3),
                                  "p99": round(float(done[int(0.99 * len(done))]), 3),
                                  "max": round(float(done[-1]), 3)},
        "batched_hbm_frac": round(info["bytes"] / ms_b / 1e6 / HBM_PEAK_GBS, 4),
        # bytes of the row items over the time their last one ended: a lower
        # bound on their rate (wave items run beside them at the end)
        "row_items": {"requests": int(row.sum()), "bytes": row_bytes,
                      "done_ms": round(row_done, 3),
                      "TB_s_lower_bound": round(row_bytes / row_done / 1e9, 3) if row_done else None,
                      "alone": alone},
        "autotune": {"chosen": {"segment_bytes": info["segment_bytes"],
                                "wave_min_bytes": info["wave_min_bytes"],
                                "waves_per_cu": info["waves_per_cu"],
                                "schedule": "static" if info["schedule"] == 2 else "dynamic"},
                     "candidate_ms": [round(x, 3) for x in cand_ms], "seconds": round(tune_s, 2)},
    }
    b.close()
    ss.close()
    del arena
    torch.cuda.synchronize()
    return out


def serving(mg, wl, seconds, speed=1.0):
    """Continuous batching under Poisson arrivals: 20,000 requests/s from
    50,000 clients, request sizes drawn as in the batched mix, a 64 GiB
    output arena as the admission cap, outputs freed on completion.  The
    first `seconds` of the 60-second trace are replayed in real time; the
    latency of a request runs from its submission to its completion event."""
    import numpy as np
    arr = wl.c5_arrivals()
    keep = arr.t < seconds * speed  # replayed `speed` times faster
    t, client = arr.t[keep], arr.client[keep]
    k, n, dt = arr.req.n_streams[keep], arr.req.length[keep], arr.req.dtype[keep]
    es = np.where(dt == 2, 8, 4)
    from paper_1412_8266_amd.serve import Server
    srv = Server(wl.C5_CLIENTS, wl.MASTER_SEED, wl.C5_ARENA_BYTES, auto_release=True)
    wall = srv.run_trace(t, client, k, n, dt, time_scale=1.0 / speed)
    res = srv.poll()
    st = srv.stats()
    srv.close()
    lat = np.sort(res["latency_s"]) * 1e3
    que = np.sort(res["queue_s"]) * 1e3
    samples = int((k * n).sum())

    def pct(a, q):
        return round(float(a[min(len(a) - 1, int(q * len(a)))]), 3) if len(a) else None

    return {
        "trace_seconds": seconds, "rate_per_s": wl.C5_RATE * speed, "clients": wl.C5_CLIENTS,
        "arena_GiB": wl.C5_ARENA_BYTES >> 30, "requests": int(keep.sum()),
        "completed": int(len(res)), "ticks": int(st["ticks"]), "wall_s": round(wall, 3),
        "offered_Gsamples_s": round(samples / seconds / 1e9, 2),
        "kept_up": bool(wall < seconds * 1.05),
        "served_Gsamples_s": round(samples / wall / 1e9, 2),
        "served_GB_s": round(float((k * n * es).sum()) / wall / 1e9, 1),
        "latency_ms": {"p50": pct(lat, 0.50), "p99": pct(lat, 0.99), "max": pct(lat, 1.0)},
        "queue_ms": {"p50": pct(que, 0.50), "p99": pct(que, 0.99)},
    }


def short_rows(mg, torch, stream):
    """Stream-major fills of short rows (the lane-per-stream writer), about
    4 GiB per launch: rows of 1000 and 1001 uint32 (off their 128-byte lines,
    each line shared by two rows written once), 1024 and 2000 uint32, 1000
    float64."""
    out = {}
    for i, (dt, n) in enumerate(((0, 1000), (0, 1001), (0, 1024), (0, 2000), (2, 1000))):
        es = 8 if dt == 2 else 4
        S = (1 << 30) // n if es == 4 else (1 << 29) // n
        ss = mg.StreamSet(S, master_seed=5)
        buf = torch.empty(S * n * es // 4, dtype=torch.int32, device="cuda")
        # the first shape also takes the clocks out of their idle state (a
        # burst from idle runs fast for two launches, then dips for several)
        per, _ = timed(lambda: ss.fill_ptr(n, dt, mg.STREAM_MAJOR, buf.data_ptr()), 10,
                       30 if i == 0 else 3, stream)
        ms = sum(per) / len(per)
        out["%s_rows_of_%d" % ("u32" if dt == 0 else "f64", n)] = {
            "streams": S, "ms": round(ms, 4), "TB_s": round(S * n * es / ms / 1e9, 3)}
        ss.close()
        del buf
    torch.cuda.synchronize()
    return out


def partitions(mg, wl, torch, stream):
    """The other partitions of sec. 2.3 and the other generators over 2^32
    uint32 (16 GiB): one stream dealt to 2^16 players x 2^16 cards (in order,
    and each player's cards in a row), random-spacing set creation, a
    Philox4x32-10 set of 2^20 streams x 4096, and a TinyMT32 hybrid set of
    2^20 streams x 4096 (256 streams per parameter set)."""
    extra = {}
    S, n = wl.C2_STREAMS, wl.C2_N
    samples = S * n
    ssl = mg.StreamSet(1, master_seed=wl.MASTER_SEED)
    outl = torch.empty(samples, dtype=torch.uint32, device="cuda")
    for name, lay in (("leapfrog_in_order_2^16x2^16", mg.INTERLEAVED),
                      ("leapfrog_player_rows_2^16x2^16", mg.STREAM_MAJOR)):
        per_l, _ = timed(lambda: ssl.fill_leapfrog(0, 1 << 16, 1 << 16, mg.U32, lay, out=outl),
                         10, 2, stream)
        msl = sum(per_l) / len(per_l)
        extra[name] = {"ms": round(msl, 4), "Gsamples_s": round(samples / msl / 1e6, 2),
                       "hbm_frac": round(samples * 4 / msl / 1e6 / HBM_PEAK_GBS, 4)}
    ssl.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ssr = mg.StreamSet(S, master_seed=wl.MASTER_SEED, spacing="random")
    torch.cuda.synchronize()
    extra["random_spacing_create_2^20_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    ssr.close()
    ssp = mg.StreamSet(S, master_seed=wl.MASTER_SEED, generator="philox")
    outp = outl.view(S, n)
    for name, lay in (("philox_fill_2^20x4096", mg.STREAM_MAJOR),
                      ("philox_interleaved_2^20x4096", mg.INTERLEAVED)):
        per_p, _ = timed(lambda: ssp.fill(n, mg.U32, lay, out=outp), 10, 2, stream)
        msp = sum(per_p) / len(per_p)
        extra[name] = {"ms": round(msp, 4), "Gsamples_s": round(samples / msp / 1e6, 2),
                       "hbm_frac": round(samples * 4 / msp / 1e6 / HBM_PEAK_GBS, 4)}
    ssp.close()
    # TinyMT32 hybrid (sec. 4.2): 256 consecutive streams share a parameter
    # set (4096 sets from the device search), sub-streams 2^64 apart
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sst = mg.StreamSet(S, master_seed=wl.MASTER_SEED, generator="tinymt", per_param=256)
    torch.cuda.synchronize()
    extra["tinymt_create_2^20_streams_4096_sets_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    for name, lay in (("tinymt_fill_2^20x4096", mg.STREAM_MAJOR),
                      ("tinymt_interleaved_2^20x4096", mg.INTERLEAVED)):
        per_t, _ = timed(lambda: sst.fill(n, mg.U32, lay, out=outp), 10, 2, stream)
        mst = sum(per_t) / len(per_t)
        extra[name] = {"ms": round(mst, 4), "Gsamples_s": round(samples / mst / 1e6, 2),
                       "hbm_frac": round(samples * 4 / mst / 1e6 / HBM_PEAK_GBS, 4)}
    sst.close()
    del outl, outp
    torch.cuda.synchronize()
    return extra


def coop_lanes_used(mg, row_bytes):
    """Lanes per stream of the wave-per-stream fill for rows of row_bytes: the
    configured value, or the library's automatic choice (16 under 64 KiB)."""
    cfg = mg.mrg_config_get("coop_lanes")
    return cfg if cfg else (64 if row_bytes >= 65536 else 16)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the stream library has no multi-GPU path "
              "(streams would shard by global index, GPU d taking a contiguous range as a "
              "stream set with first_stream, with no exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 29, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    import paper_1412_8266_amd as mg
    from paper_1412_8266_amd import workloads as wl

    if args.engine is not None:
        mg.mrg_config_set("engine", args.engine)
    if args.tile_bytes is not None:
        mg.mrg_config_set("tile_bytes", args.tile_bytes)
    if args.strategy is not None:
        mg.mrg_config_set("strategy", args.strategy)
    if args.coop_wgs_per_cu is not None:
        mg.mrg_config_set("coop_wgs_per_cu", args.coop_wgs_per_cu)
    if args.coop_lanes is not None:
        mg.mrg_config_set("coop_lanes", args.coop_lanes)
    engine = mg.mrg_config_get("engine")
    tile = mg.mrg_config_get("tile_bytes")
    stream = torch.cuda.current_stream()

    if args.rows_only:
        print("[bench] short rows", file=sys.stderr, flush=True)
        print(json.dumps({"short_rows": short_rows(mg, torch, stream)}), flush=True)
        return

    if args.partitions_only:
        print("[bench] partitions and Philox", file=sys.stderr, flush=True)
        print(json.dumps({"partitions": partitions(mg, wl, torch, stream)}), flush=True)
        return

    if args.batch_only:
        print("[bench] batched request mix", file=sys.stderr, flush=True)
        print(json.dumps({"batched": batched(mg, wl, torch, stream, args.batch_reps)}), flush=True)
        return

    S, n = wl.C2_STREAMS, wl.C2_N
    samples = S * n
    print("[bench] creating %d streams" % S, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ss = mg.StreamSet(S, master_seed=wl.MASTER_SEED)
    torch.cuda.synchronize()
    first_create_s = time.perf_counter() - t0  # includes the device's one-time table setup
    t0 = time.perf_counter()
    ss2 = mg.StreamSet(S, master_seed=wl.MASTER_SEED ^ 1)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    ss2.close()
    out = torch.empty((S, n), dtype=torch.uint32, device="cuda")
    ptr = out.data_ptr()

    def step_u32():
        ss.fill_ptr(n, mg.U32, mg.STREAM_MAJOR, ptr)

    print("[bench] timing u32 fill: %d warmup + %d steps" % (args.warmup, args.steps),
          file=sys.stderr, flush=True)
    per, wall = timed(step_u32, args.steps, args.warmup, stream)
    ms = sum(per) / len(per)
    value = samples / (ms * 1e-3) / 1e9
    alg_bytes = samples * 4 + S * 24 * 2  # outputs + state read and write-back
    achieved = alg_bytes / (ms * 1e-3) / 1e9

    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "plain bulk fill: 2^20 MRG32k3a streams x 4096 uint32 outputs, "
                        "stream-major, streams spaced 2^127 from a 64-bit master seed",
            "streams": S,
            "n_per_stream": n,
            "layout": "stream_major",
            "master_seed": hex(wl.MASTER_SEED),
            "engine": "binary64" if engine == 1 else "int32",
            "tile_bytes": tile,
            "coop_lanes": mg.mrg_config_get("coop_lanes"),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": COUNTERS["traffic"] if counters_current() else None,
            "traffic_source": "%s (kernel sources sha256 %s)" % (
                COUNTERS["source"], COUNTERS["kernel_sources_sha256"][:16]) if counters_current() else
            "none: the kernel sources changed since the last counter profile",
            "kernel": ("fill_coop_kernel<u32, %d lanes per stream>" % coop_lanes_used(mg, n * 4))
                      if n >= 2048 and mg.mrg_config_get("strategy") != 1
                      else "fill_sm_kernel<u32>",
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": round(ms, 4),
        },
        "valu": None if not counters_current() else {
            # issue cycles at 4 clocks per wave instruction (FP64 rate) over the
            # cycles the launch would span at the peak clock: VALU use against peak
            "instr_per_sample": round(COUNTERS["valu_insts"] * 64 / samples, 2),
            "issue_frac_at_peak_clock": round(COUNTERS["valu_insts"] * 4 / SIMDS
                                              / (ms * 1e-3 * PEAK_SCLK_MHZ * 1e6), 4),
            "source": COUNTERS["source"],
        },
        "wall_s_timed": round(wall, 3),
    }

    extra = {"create_streams_ms": round(create_s * 1e3, 2),
             "first_create_streams_ms": round(first_create_s * 1e3, 2)}
    if not args.quick:
        # FP32 fill (same launch, 4-byte floats)
        outf = out.view(torch.float32)
        per_f, _ = timed(lambda: ss.fill_ptr(n, mg.F32, mg.STREAM_MAJOR, outf.data_ptr()),
                         args.steps, 1, stream)
        msf = sum(per_f) / len(per_f)
        extra["f32_fill"] = {"Gsamples_s": round(samples / msf / 1e6, 2), "ms": round(msf, 4),
                             "hbm_frac": round((samples * 4 + S * 48) / msf / 1e6 / HBM_PEAK_GBS, 4)}
        per_i, _ = timed(lambda: ss.fill_ptr(n, mg.U32, mg.INTERLEAVED, ptr), args.steps, 1, stream)
        msi = sum(per_i) / len(per_i)
        extra["u32_interleaved"] = {"Gsamples_s": round(samples / msi / 1e6, 2),
                                    "ms": round(msi, 4)}
        # store-only probes over the same 16 GiB: what the stores alone attain
        probe = {}
        for name, pat in (("streaming_16B", 0), ("fill_lines", 1), ("fill_runs_of_8_lines", 2),
                          ("single_lines", 3)):
            per_p, _ = timed(lambda: mg.write_probe(out, pat, stream), args.steps, 1, stream)
            msp = sum(per_p) / len(per_p)
            probe[name + "_GBs"] = round(out.numel() * 4 / msp / 1e6, 1)
        probe["fill_over_fill_lines"] = round(achieved / probe["fill_lines_GBs"], 4)
        probe["fill_over_streaming"] = round(achieved / probe["streaming_16B_GBs"], 4)
        extra["store_probe"] = probe
        del outf
        del out
        # FP64 fill: half the streams so the output stays at 16 GiB
        outd = torch.empty((S // 2, n), dtype=torch.float64, device="cuda")
        per_d, _ = timed(lambda: ss.fill_ptr(n, mg.F64, mg.STREAM_MAJOR, outd.data_ptr(),
                                             count=S // 2), args.steps, 1, stream)
        msd = sum(per_d) / len(per_d)
        extra["f64_fill_half_streams"] = {"Gsamples_s": round(samples / 2 / msd / 1e6, 2),
                                          "ms": round(msd, 4),
                                          "hbm_frac": round(samples * 4 / msd / 1e6 / HBM_PEAK_GBS, 4)}
        del outd
        # jump: 2^16 streams by random 64-bit offsets + 2^76 (per-stream tables)
        import numpy as np
        ss3 = mg.StreamSet(wl.C3_STREAMS, master_seed=wl.MASTER_SEED)
        ex = torch.from_numpy(wl.c3_exponents(wl.c3_offsets()).view(np.int64)).cuda()
        per_j, _ = timed(lambda: ss3.jump(ex), 10, 1, stream)
        extra["jump_2^16_streams_ms"] = round(sum(per_j) / len(per_j), 4)
        # the jumped set's fill: 2^16 streams x 1024 uint32 (each call continues)
        out3 = torch.empty((wl.C3_STREAMS, wl.C3_N), dtype=torch.uint32, device="cuda")
        per_3, _ = timed(lambda: ss3.fill_ptr(wl.C3_N, mg.U32, mg.STREAM_MAJOR, out3.data_ptr()),
                         10, 1, stream)
        ms3 = sum(per_3) / len(per_3)
        extra["jumped_2^16x1024_fill"] = {"ms": round(ms3, 4),
                                           "Gsamples_s": round(wl.C3_STREAMS * wl.C3_N / ms3 / 1e6, 2)}
        del out3
        ss3.close()
        extra.update(partitions(mg, wl, torch, stream))
        extra["short_rows"] = short_rows(mg, torch, stream)
    ss.close()
    torch.cuda.synchronize()
    if not args.quick and not args.no_batch:
        print("[bench] batched request mix", file=sys.stderr, flush=True)
        extra["batched"] = batched(mg, wl, torch, stream, args.batch_reps)
    if not args.quick and not args.no_serve:
        print("[bench] serving trace (%g s)" % args.serve_seconds, file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extra["serving"] = serving(mg, wl, args.serve_seconds)
        # the highest arrival rate served without falling behind: 4-second
        # windows at rising rates, up to the first one that falls behind
        sweep, best = [], None
        k = 1
        while True:
            speed = round(1.0 + k * args.serve_step, 6)
            if speed > args.serve_max_speed:
                break
            print("[bench] serving at %g x the arrival rate" % speed, file=sys.stderr, flush=True)
            r = serving(mg, wl, 4.0, speed)
            sweep.append({key: r[key] for key in ("rate_per_s", "offered_Gsamples_s",
                                                  "served_Gsamples_s", "kept_up", "latency_ms")})
            if not r["kept_up"]:
                break
            best = r
            k += 1
        if best is not None and sweep and not sweep[-1]["kept_up"]:
            # one more window halfway between the last rate kept up and the
            # first that fell behind
            mid = round((best["rate_per_s"] + sweep[-1]["rate_per_s"]) / 2.0 / wl.C5_RATE, 6)
            print("[bench] serving at %g x the arrival rate" % mid, file=sys.stderr, flush=True)
            r = serving(mg, wl, 4.0, mid)
            sweep.insert(len(sweep) - 1, {key: r[key] for key in (
                "rate_per_s", "offered_Gsamples_s", "served_Gsamples_s", "kept_up", "latency_ms")})
            if r["kept_up"]:
                best = r
        extra["serving_rate_sweep"] = sweep
        behind = [x["rate_per_s"] for x in sweep if not x["kept_up"]]
        extra["serving_max_sustained"] = None if best is None else {
            "rate_per_s": best["rate_per_s"], "offered_Gsamples_s": best["offered_Gsamples_s"],
            "first_rate_behind_per_s": min(behind) if behind else None}
    res["extra"] = extra

    if not args.no_cpu and not args.quick:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(1 << 19, n)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
