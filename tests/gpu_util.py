"""Helpers shared by the GPU tests: run blocks through the HIP library (C ABI)
and the CPU reference on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle.lof_oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.cuda()


def oracle_params(fp) -> O.Params:
    """CPU-reference parameters equal to a LofParams."""
    return O.Params(start_threshold=fp.start_threshold, p=fp.p, sensitivity=fp.sensitivity,
                    n_levels=fp.n_levels, n_levels_freq=fp.n_levels_freq,
                    sir_eta_num=fp.sir_eta_num, sir_eta_den=fp.sir_eta_den,
                    history_sensitivity=fp.history_sensitivity, history_len=fp.history_len,
                    history_min=fp.history_min,
                    literal_history_tie=bool(fp.options & 0x2))


def run_gpu(flagger, items, stream=None):
    """items: list of (x numpy, dtype, stream_id).  Returns (flags list, stats list)."""
    import torch
    from paper_1701_08197_amd import Block, STATS_BYTES, decode_stats
    blocks, outs, keep = [], [], []
    for x, dt, sid in items:
        d = to_dev(x, dt)
        C, T = (x.shape[0], x.shape[1])
        f = torch.full((C, T), 7, dtype=torch.uint8, device="cuda")
        keep.append(d)
        outs.append(f)
        blocks.append(Block(d, f, dt, sid))
    stats = torch.zeros(len(items) * STATS_BYTES, dtype=torch.uint8, device="cuda")
    flagger.flag_blocks(blocks, stream=stream, stats=stats)
    torch.cuda.synchronize()
    flags = [o.cpu().numpy() for o in outs]
    st = decode_stats(stats.cpu().numpy().tobytes())
    return flags, st


def mismatch(a, b):
    return int(np.count_nonzero(a.astype(bool) != b.astype(bool)))
