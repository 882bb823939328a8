#!/usr/bin/env python3
"""Throughput benchmark of the LOF flagging hot path on one MI355X.

Workload: one LOFAR-like second of pre-beamformer data, 48 stations x 2
polarisations x 64 subbands = 6144 independent blocks of 64 channels x 3072
times of complex int8 voltages (synthetic, seeded; see synth).  One step flags
every block in one lof_flag_blocks call (power, median, stddev, SumThreshold
time then frequency, SIR, history flagger against per-channel history of each
(station, pol, subband) stream) and commits the staged history values with
lof_history_update.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `roofline` is for the dominant kernel of the path (the
phase kernel with the largest share of a call): the bytes that phase must move
per sample times the samples of a launch, divided by its mean launch time, from
HIP events the library records on the launch stream between the phase kernels
(LOF_OPT_PHASE_TIMING).  `path_roofline` is the whole call: input + one flag
byte per sample + history ring traffic over the call's time.  `traffic` is the
HBM traffic of that kernel from rocprofv3 counters (profiles/), or null when the
kernel sources changed since the counters were taken.  `cpu_baseline` times the
CPU reference on a bounded sample of the same blocks.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import multiprocessing as mp
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

C, T = synth.CFG1_C, synth.CFG1_T
HBM_PEAK_GBS = 8000.0
DEADLINE_S = T * (64.0 / 195.3125e3)   # 3072 samples of 327.68 us

# kernel of each phase for this workload (complex int8, 48 samples per lane)
DOMINANT_KERNEL = {"stats": "lof_stats_kernel<true>", "sumthreshold_time": "lof_time_kernel<true, 48>",
                   "sumthreshold_freq": "lof_freq_kernel<true>", "sir_time": "lof_sir_time_kernel<48>",
                   "sir_freq": "lof_sir_freq_kernel", "history_write": "lof_final_kernel<true>"}
# bytes each phase must move per sample here: 2 B of complex int8 input, 1 bit of
# mask per read or write, 1 flag byte (written by the SIR frequency pass for
# blocks of up to 64 channels); the history pass reads the mask (its reads of
# flagged samples depend on the data, and the ring traffic is below 3%)
DOMINANT_BYTES_PER_SAMPLE = {"stats": 2.0, "sumthreshold_time": 2.125, "sumthreshold_freq": 2.25,
                             "sir_time": 0.25, "sir_freq": 1.25, "history_write": 0.125}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_config1.txt")
KERNEL_SOURCES = ("lof_device.hpp", "lof_kernels.hpp", "lof.hip")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1701_08197_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (JSON
    lines: kernel, fetch_bytes, write_bytes, source_hash), or None when absent
    or taken from other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    cur = kernel_source_hash()
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if not line.startswith("{"):
                continue
            rec = json.loads(line)
            if rec.get("kernel") == kernel and rec.get("source_hash") == cur:
                return int(rec["fetch_bytes"] + rec["write_bytes"])
    return None


def _gen_range(args):
    shm_name, nb, b0, b1 = args
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        arr = np.ndarray((nb, C, T, 2), dtype=np.int8, buffer=shm.buf)
        for b in range(b0, b1):
            arr[b] = synth.config1_block(b)
        del arr
    finally:
        shm.close()
    return b1 - b0


def make_config1(nb: int, workers: int, start_method: str = "fork"):
    """All blocks of the 48-station second, generated in parallel; returns
    (array view, shared-memory handle).  Use start_method="spawn" once the GPU
    runtime is initialised in this process."""
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(create=True, size=nb * C * T * 2)
    chunks = []
    step = max(1, nb // (workers * 8))
    for b0 in range(0, nb, step):
        chunks.append((shm.name, nb, b0, min(nb, b0 + step)))
    ctx = mp.get_context(start_method)
    with ctx.Pool(workers) as pool:
        for _ in pool.imap_unordered(_gen_range, chunks):
            pass
    arr = np.ndarray((nb, C, T, 2), dtype=np.int8, buffer=shm.buf)
    return arr, shm


def _oracle_one(b):
    import oracle.lof_oracle as O
    x = synth.config1_block(b)
    t0 = time.perf_counter()
    h = O.History(O.Params())
    O.flag_block(x, O.CI8, O.Params(), history=h, stream_id=0)
    return time.perf_counter() - t0


def cpu_baseline(cores: int, target_cpu_s: float):
    """The CPU reference (never tuned) on a bounded sample of config blocks,
    one block per task on `cores` processes; generation is outside the timing."""
    import oracle.lof_oracle as O
    x = synth.config1_block(0)
    t0 = time.perf_counter()
    O.flag_block(x, O.CI8, O.Params(), history=O.History(O.Params()), stream_id=0)
    t1 = time.perf_counter() - t0
    n = max(cores, int(round(target_cpu_s / max(t1, 1e-3) / cores)) * cores)
    blocks = list(range(1, 1 + n))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_one, blocks[:cores])              # warm the workers
        w0 = time.perf_counter()
        cpu = pool.map(_oracle_one, blocks)
        wall = time.perf_counter() - w0
    # generation runs inside the tasks: count only the reference's own time,
    # spread over the cores that ran it
    busy = sum(cpu) / cores
    samples = n * C * T
    return {"value": samples / busy / 1e9, "unit": "Gsamples/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} of the 6144 blocks (64 x 3072 complex int8, full path incl. history), "
                      f"{sum(cpu):.1f} s of CPU in {wall:.1f} s wall on {cores} processes"}


# ------------------------------------------------------------------ config 2
def _gen_cfg2(args):
    b, C, T = args
    return b, synth.f32_power_block(synth.rng_for(2, b), C, T)


def run_batched(args, cores):
    """4096 uneven float32 blocks: one launch per block vs one batched call
    (default tuning, autotuned, and hipGraph replay of the tuned call)."""
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as NAT
    nb = args.blocks2
    shapes = synth.config2_shapes()[:nb]
    # rows padded to 16 elements so every row starts 16-byte aligned
    offs, strides, tot, samples = [], [], 0, 0
    for C_, T_ in shapes:
        st_ = (T_ + 15) // 16 * 16
        offs.append(tot)
        strides.append(st_)
        tot += C_ * st_
        samples += C_ * T_
    data = torch.empty(tot, dtype=torch.float32, device="cuda")
    flags = torch.empty(tot, dtype=torch.uint8, device="cuda")
    t_gen = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        for b, x in pool.imap_unordered(_gen_cfg2, [(b, C_, T_) for b, (C_, T_) in enumerate(shapes)], chunksize=4):
            C_, T_ = x.shape
            data[offs[b]:offs[b] + C_ * strides[b]].view(C_, strides[b])[:, :T_].copy_(torch.from_numpy(x))
    t_gen = time.perf_counter() - t_gen
    arr = (NAT.LofBlock * nb)()
    for b, (C_, T_) in enumerate(shapes):
        blk = arr[b]
        blk.data = data[offs[b]:].data_ptr()
        blk.flags = flags[offs[b]:].data_ptr()
        blk.data_row_stride = strides[b]
        blk.flag_row_stride = strides[b]
        blk.n_channels = C_
        blk.n_times = T_
        blk.dtype = NAT.LOF_F32
        blk.stream_id = b
    base = dict(max_streams=nb, max_channels=256, max_blocks_per_call=nb, max_samples_per_call=tot)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    fl = P.Flagger(P.default_params(**base))
    one = (NAT.LofBlock * 1)()

    def per_block():
        for b in range(nb):
            one[0] = arr[b]
            if fl.flag_blocks_raw(one, 1, sh) != 0:
                raise RuntimeError("flag failed")
    t_pb = timed(per_block, 1)
    t_batch = timed(lambda: fl.flag_blocks_raw(arr, nb, sh), args.steps)
    tune = fl.autotune(list(arr), stream=sh, reps=1)
    t_tuned = timed(lambda: fl.flag_blocks_raw(arr, nb, sh), args.steps)
    fl.close()
    fg = P.Flagger(P.default_params(options=P.LOF_OPT_GRAPH, **base))
    fg.set_tuning(tune)
    t_graph = timed(lambda: fg.flag_blocks_raw(arr, nb, sh), args.steps)
    fg.close()
    gs = lambda t: round(samples / t / 1e9, 3)
    return {"metric": "flagged Gsamples/s, batched uneven blocks", "workload": "4096 float32 power blocks, "
            "C in {16,64,256}, T uniform in [768,12288], 1/f bandpass drift + RFI mix",
            "blocks": nb, "samples": samples, "unit": "Gsamples/s",
            "per_block_launches": gs(t_pb), "batched_default": gs(t_batch), "batched_autotuned": gs(t_tuned),
            "graph_replay_autotuned": gs(t_graph),
            "alg_GBps_graph": round(samples * 5 / t_graph / 1e9, 1),
            "tuning": {"time_lanes": [list(tune.time_lanes[0]), list(tune.time_lanes[1])],
                       "persistent": tune.persistent},
            "gen_s": round(t_gen, 1)}


# ------------------------------------------------------------------ config 4
def _gen_cfg4(args):
    st, sb = args
    return st, sb, synth.config4_block(st, 0, sb)


def run_serve(args, cores):
    """48 stations, 16-64 subbands each, Poisson arrivals (mean 1 s per station),
    continuous batching over a fixed device arena; sweep of arrival speed-ups."""
    import torch
    from paper_1701_08197_amd.serve import Service, latency_summary
    subs = synth.config4_subbands()
    pool = {}
    ctx = mp.get_context("fork")
    jobs = [(st, sb) for st, n in enumerate(subs) for sb in range(n)]
    with ctx.Pool(cores) as p:
        for st, sb, x in p.imap_unordered(_gen_cfg4, jobs, chunksize=8):
            pool[(st, sb)] = torch.from_numpy(x).cuda()
    points = []
    for speedup in [float(v) for v in args.speedups.split(",")]:
        obs = max(8.0, args.serve_wall * speedup)
        arrivals = [(t, st, k) for (t, st, k) in synth.config4_arrivals(obs)]
        svc = Service(len(subs), 64, n_slots=args.slots, C=C, T=T)
        t0 = time.perf_counter()
        done = svc.run(arrivals, lambda st, k: [pool[(st, sb)] for sb in range(subs[st])], speedup=speedup)
        wall = time.perf_counter() - t0
        warm = sorted(done, key=lambda r: r.arrival)[len(done) // 4:]
        summ = latency_summary(warm, C, T, wall, DEADLINE_S)
        summ["admitted_gsamples_per_s"] = round(sum(len(r.slots) for r in done) * C * T / wall / 1e9, 3)
        summ.update({"speedup": speedup, "observation_s": obs})
        points.append({k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()})
        svc.close()
    ok = [p for p in points if p["p99_ms"] <= DEADLINE_S * 1e3]
    return {"metric": "streaming: admitted Gsamples/s and p50/p99 block latency vs real-time deadline",
            "workload": "48 stations x 16-64 subbands x 64 ch x 3072 t complex int8, Poisson arrivals (1 s)",
            "arena_slots": args.slots, "points": points,
            "max_speedup_meeting_deadline": max((p["speedup"] for p in ok), default=None)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--blocks", type=int, default=synth.CONFIG1_BLOCKS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workers", type=int, default=0)
    ap.add_argument("--workload", choices=["second", "batched", "serve"], default="second",
                    help="second: the 48-station second (default); batched: 4096 uneven float blocks; "
                         "serve: streaming service sweep")
    ap.add_argument("--blocks2", type=int, default=4096)
    ap.add_argument("--slots", type=int, default=4096)
    ap.add_argument("--speedups", default="10,50,100,200,300")
    ap.add_argument("--serve-wall", type=float, default=3.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the blocks are independent and "
              f"shard by stream across GPUs, but multi-GPU runs are not part of this build.", file=sys.stderr)
        sys.exit(2)

    cores = len(os.sched_getaffinity(0))
    cores = min(cores, 16)
    workers = args.workers or cores
    if args.workload == "batched":
        print(json.dumps(run_batched(args, workers)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args, workers)), flush=True)
        return
    nb = args.blocks
    t_gen = time.perf_counter()
    host, shm = make_config1(nb, workers)
    t_gen = time.perf_counter() - t_gen

    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as NAT

    dev = torch.device("cuda:0")
    data = torch.from_numpy(host).to(dev)
    del host
    shm.close()
    shm.unlink()
    flags = torch.empty((nb, C, T), dtype=torch.uint8, device=dev)
    prm = P.default_params(max_streams=nb, max_channels=C, max_blocks_per_call=nb,
                           max_samples_per_call=nb * C * T, options=P.LOF_OPT_PHASE_TIMING)
    fl = P.Flagger(prm)
    arr = (NAT.LofBlock * nb)()
    for b in range(nb):
        blk = arr[b]
        blk.data = data[b].data_ptr()
        blk.flags = flags[b].data_ptr()
        blk.data_row_stride = T
        blk.flag_row_stride = T
        blk.n_channels = C
        blk.n_times = T
        blk.dtype = NAT.LOF_CI8
        blk.stream_id = b
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def step(e0=None, e1=None):
        if e0 is not None:
            e0.record(stream)
        rc = fl.flag_blocks_raw(arr, nb, sh)
        if e1 is not None:
            e1.record(stream)
        if rc != 0:
            raise RuntimeError(f"lof_flag_blocks failed: {rc}")
        fl.history_update(None, sh)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fl.phase_times()          # drop the warm-up calls from the phase totals
    K = args.steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(K):
        step(*evs[k])
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phase_tot, phase_calls = fl.phase_times()
    phase_ms = {k: v / max(1, phase_calls) for k, v in phase_tot.items()}
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    # per-step latency: time from the step's launch to its completion
    step_ms = [evs[k][0].elapsed_time(ends[k]) for k in range(K)]
    ms_per_step = wall * 1e3 / K
    samples = nb * C * T
    value = samples / (ms_per_step * 1e-3) / 1e9

    # algorithmic bytes per launch: 2 B input + 1 B flag per sample, plus the
    # history ring read (committed entries, once warm-up is over) and the staged write
    H, Hmin = prm.history_len, prm.history_min
    hist_bytes = []
    for k in range(K):
        L = min(args.warmup + k, H)
        rd = nb * C * L * 8 if L >= Hmin else 0
        hist_bytes.append(rd + nb * C * 8)
    alg_bytes = samples * 3 + statistics.mean(hist_bytes)
    kmean = statistics.mean(kern_ms)
    path_achieved = alg_bytes / (kmean * 1e-3) / 1e9
    # dominant kernel: the phase with the largest share of the call
    dom = max(phase_ms, key=phase_ms.get)
    dom_ms = phase_ms[dom]
    dom_bytes = samples * DOMINANT_BYTES_PER_SAMPLE[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(DOMINANT_KERNEL[dom])
    lat = sorted(step_ms)
    p50 = lat[len(lat) // 2]
    p99 = lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]

    fl.close()
    out = {
        "metric": "flagged Gsamples/s + % HBM roofline; p99 block latency vs real-time deadline",
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "LOFAR-like second of pre-beamformer voltages: 48 stations x 2 pols x 64 "
                               "subbands = 6144 blocks of 64 channels x 3072 times, complex int8 "
                               "(sigma 16, RFI mix, weak dispersed pulse)",
                   "blocks": nb, "channels": C, "times": T, "input": "complex int8",
                   "n_levels": prm.n_levels, "sir_eta": [prm.sir_eta_num, prm.sir_eta_den],
                   "history_len": H, "launch": "one lof_flag_blocks + one lof_history_update per step"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": DOMINANT_KERNEL[dom], "kernel_ms": round(dom_ms, 4),
                     "alg_bytes_per_launch": int(dom_bytes),
                     "alg_bytes_per_sample": DOMINANT_BYTES_PER_SAMPLE[dom]},
        "path_roofline": {"bound": "hbm", "achieved": round(path_achieved, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(path_achieved / HBM_PEAK_GBS, 4),
                          "call_ms": round(kmean, 4), "alg_bytes_per_call": int(alg_bytes),
                          "phases_ms": {k: round(v, 4) for k, v in phase_ms.items()}},
        "latency": {"p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
                    "deadline_ms": round(DEADLINE_S * 1e3, 2), "unit": "ms per 6144-block second"},
        "gen_s": round(t_gen, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cores, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
