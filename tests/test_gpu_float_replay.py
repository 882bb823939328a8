"""Float input: level-local replay.  The GPU runs SumThreshold stopped after
each level (time levels, then frequency levels); the CPU reference re-decides
the next level from the GPU's own mask in float64.  Every disagreement must lie
in a window whose unflagged mean is within 1e-6 (relative) of the level's
threshold.  The end-to-end mismatch rate is reported."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import run_gpu, say

pytestmark = pytest.mark.gpu
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
    import paper_1701_08197_amd as P
    fl = P.Flagger(P.default_params(max_streams=1, max_channels=256, max_blocks_per_call=1,
                                    max_samples_per_call=1 << 22, sir_eta_num=0, **kw))
    flags, st = run_gpu(fl, [(x, dt, -1)])
    fl.close()
    return flags[0].astype(bool), st[0]


CASES = [("config0", None), ("f32_drift", (O.F32, 64, 3000)), ("stokes", (O.F32, 16, 768)),
         ("vis_amp", (O.C64_AMP, 256, 1024))]


@pytest.mark.parametrize("name,spec", CASES)
def test_level_local_replay(name, spec):
    say(f"[level_local_replay] {name}")
    if spec is None:
        x, dt = synth.config0()
    elif name == "stokes":
        x, dt = synth.config3a_block(0), O.F32
    elif name == "vis_amp":
        x, dt = synth.config3b_block(0), O.C64_AMP
    else:
        dt, C, T = spec
        x = synth.f32_power_block(np.random.default_rng(5), C, T)
    p = O.power(x, dt)
    prm = O.Params()
    med, sd = O.block_median(p), O.block_stddev(p, False)
    Ts = O.thresholds(med, sd, prm)
    # time levels
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
    # frequency levels, starting from the GPU's full time mask
    for k in range(1, 7):
        I = 1 << k
        if I > p.shape[0]:
            break
        nxt, _ = gpu_mask(x, dt, n_levels=7, n_levels_freq=k + 1)
        nd, ok = replay_check(p.T, prev.T, nxt.T, Ts[k], I)
        total_diff += nd
        assert ok, (name, "freq", k, nd)
        prev = nxt
    full, _ = gpu_mask(x, dt)
    ref = O.flag_block(x, dt, O.Params(sir_eta_num=0))
    rate = float((full != ref.flags).mean())
    say(f"    {name}: level-local disagreements {total_diff}, end-to-end mismatch rate {rate:.3g}")
    assert rate < 1e-3
