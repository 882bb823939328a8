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
                    literal_history_tie=bool(fp.options & 0x2),
                    sir_prose=bool(fp.options & 0x10),
                    robust_sigma=bool(fp.options & 0x40),
                    history_winsor=fp.history_winsor)


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


# ---------------------------------------------------------------- float criterion
REL = 1e-6


def level_windows(p, m, T, I):
    """float64 window sums S and counts c of level I on mask m (rows)."""
    R, n = p.shape
    nw = n - I + 1
    unfl = ~m
    v = np.where(unfl, p, 0.0)
    S = np.zeros((R, nw))
    c = np.zeros((R, nw), dtype=np.int64)
    for d in range(I):
        S += v[:, d:d + nw]
        c += unfl[:, d:d + nw]
    return S, c


def replay_check(p, m_prev, m_next, T, I):
    """Windows flagged by the reference from m_prev vs the GPU's m_next."""
    S, c = level_windows(p, m_prev, T, I)
    hit = (c > 0) & (S > c * T)
    border = (c > 0) & (np.abs(S - c * T) <= REL * c * T)
    nw = S.shape[1]
    exp = m_prev.copy()
    cover_border = np.zeros_like(m_prev)
    for d in range(I):
        exp[:, d:d + nw] |= hit
        cover_border[:, d:d + nw] |= border
    diff = exp != m_next
    return int(diff.sum()), bool((~diff | cover_border).all())


def gpu_mask(x, dt, **kw):
    """The GPU's mask of one block flagged alone, SIR off (levels from kw)."""
    import paper_1701_08197_amd as P
    fl = P.Flagger(P.default_params(max_streams=1, max_channels=256, max_blocks_per_call=1,
                                    max_samples_per_call=1 << 22, sir_eta_num=0, **kw))
    flags, st = run_gpu(fl, [(x, dt, -1)])
    fl.close()
    return flags[0].astype(bool), st[0]



def level_local_replay(x, dt, name=""):
    """Level-local replay of one float block (the SumThreshold float criterion):
    the GPU runs stopped after each level (time levels, then frequency levels);
    the reference re-decides the next level from the GPU's own mask in float64;
    every disagreement must lie in a window whose unflagged mean is within REL
    of the level's threshold.  Returns the number of level-local disagreements."""
    p = O.power(x, dt)
    prm = O.Params()
    med, sd = O.block_median(p), O.block_stddev(p, False)
    Ts = O.thresholds(med, sd, prm)
    prev = np.zeros(p.shape, dtype=bool)
    total_diff = 0
    for k in range(7):
        I = 1 << k
        if I > p.shape[1]:
            break
        nxt, _ = gpu_mask(x, dt, n_levels=k + 1, n_levels_freq=0)
        nd, ok = replay_check(p, prev, nxt, Ts[k], I)
        total_diff += nd
        assert ok, (name, "time", k, nd)
        prev = nxt
    for k in range(1, 7):
        I = 1 << k
        if I > p.shape[0]:
            break
        nxt, _ = gpu_mask(x, dt, n_levels=7, n_levels_freq=k + 1)
        nd, ok = replay_check(p.T, prev.T, nxt.T, Ts[k], I)
        total_diff += nd
        assert ok, (name, "freq", k, nd)
        prev = nxt
    return total_diff
