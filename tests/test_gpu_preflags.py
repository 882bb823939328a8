"""GPU: caller-supplied pre-flags (LOF_OPT_PREFLAGGED: the flag bytes hold a
mask on entry; Sec. 4.2 statistics of the unflagged samples, Sec. 2.1 flagged
samples leave the window sums) through the C ABI, against the oracle's
flag_block(..., preflags=...).  Complex int8 input is exact: median, stddev,
thresholds, flags, history rows and rings bit for bit, for pre-flag densities
from none to every sample, long rows, blocks past 64 channels, the MAD, the
histogram-wrap path and unaligned flag rows; float input within the float
bound."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, say

pytestmark = pytest.mark.gpu


def make(**kw):
    import paper_1701_08197_amd as P
    opts = kw.pop("options", 0) | P.LOF_OPT_PREFLAGGED
    base = dict(max_streams=8, max_channels=1024, max_blocks_per_call=16, max_samples_per_call=1 << 22,
                options=opts)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


def run_pre(fl, items, pad=0):
    """items: (x, dtype, stream_id, pre).  The flag tensors start as the pre-flag
    masks (rows offset by `pad` bytes inside a wider buffer when pad > 0)."""
    import torch
    from paper_1701_08197_amd import Block, STATS_BYTES, decode_stats
    blocks, outs, keep = [], [], []
    for x, dt, sid, pre in items:
        d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        C, T = x.shape[0], x.shape[1]
        if pad:
            big = torch.zeros((C, T + pad + 3), dtype=torch.uint8, device="cuda")
            f = big[:, pad:pad + T]
        else:
            f = torch.empty((C, T), dtype=torch.uint8, device="cuda")
        f.copy_(torch.from_numpy(pre.astype(np.uint8) * np.uint8(5)))   # any nonzero byte flags
        keep.append(d)
        outs.append(f)
        blocks.append(Block(d, f, dt, sid))
    stats = torch.zeros(len(items) * STATS_BYTES, dtype=torch.uint8, device="cuda")
    fl.flag_blocks(blocks, stats=stats)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], decode_stats(stats.cpu().numpy().tobytes())


def check_exact(s, f, r, params):
    nT = max(params.n_levels, params.n_levels_freq if params.n_levels_freq >= 0 else 0)
    assert s["median"] == r.median
    assert s["stddev"] == r.stddev
    assert s["threshold"][:nT] == r.thresholds[:nT]
    assert mismatch(f, r.flags) == 0
    assert set(np.unique(f)) <= {0, 1}
    assert s["n_flagged"] == int(r.flags.sum())


SHAPES = [(1, 1), (3, 7), (16, 768), (64, 3072), (7, 1000), (2, 9001), (70, 300), (256, 64), (33, 129)]


@pytest.mark.parametrize("density", [0.0, 0.02, 0.3, 1.0])
def test_preflags_ci8_exact(density):
    say(f"[preflags_ci8_exact] density={density}")
    fl = make()
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(7000 + int(density * 100))
    items = []
    for C, T in SHAPES:
        x = synth.ci8_block(rng, C, T)
        pre = rng.random((C, T)) < density
        pre[C // 2, T // 3:T // 3 + min(T, 40)] = density > 0      # a pre-flagged stretch
        items.append((x, O.CI8, -1, pre))
    flags, st = run_pre(fl, items)
    for (x, _, _, pre), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.CI8, prm, preflags=pre)
        check_exact(s, f, r, fl.params)
        assert f[pre].all()
    fl.close()


@pytest.mark.parametrize("opts", [0, 0x10, 0x40])
def test_preflags_ci8_options_and_unaligned_rows(opts):
    """With the prose SIR reading or the MAD, and with flag rows that are not
    16-byte aligned (the byte paths of the pre-flag reads)."""
    say(f"[preflags_ci8_options_and_unaligned_rows] options={opts}")
    fl = make(options=opts)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(7100 + opts)
    items = []
    for C, T in [(16, 768), (64, 3072), (5, 4500), (100, 200)]:
        x = synth.ci8_block(rng, C, T)
        items.append((x, O.CI8, -1, rng.random((C, T)) < 0.1))
    for pad in (0, 1):
        flags, st = run_pre(fl, items, pad=pad)
        for (x, _, _, pre), f, s in zip(items, flags, st):
            check_exact(s, f, O.flag_block(x, O.CI8, prm, preflags=pre), fl.params)
    fl.close()


@pytest.mark.parametrize("variant", ["const", "ternary"])
def test_preflags_histogram_wrap(variant):
    """A power value occurring 2^16 times or more (the radix-select path over the
    samples, which must skip the pre-flagged ones too)."""
    say(f"[preflags_histogram_wrap] {variant}")
    fl = make(options=0x40)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(7200)
    C, T = 64, 3072
    x = (np.full((C, T, 2), 5, dtype=np.int8) if variant == "const"
         else rng.integers(-1, 2, size=(C, T, 2)).astype(np.int8))
    x[3, 100:140, 0] = 90
    pre = rng.random((C, T)) < 0.2
    flags, st = run_pre(fl, [(x, O.CI8, -1, pre)])
    check_exact(st[0], flags[0], O.flag_block(x, O.CI8, prm, preflags=pre), fl.params)
    fl.close()


def test_preflags_history_sequence():
    say("[preflags_history_sequence]")
    fl = make(history_len=4, history_min=2, history_sensitivity=2.0)
    prm = oracle_params(fl.params)
    h = O.History(prm)
    rng = np.random.default_rng(7300)
    shapes = [(64, 3072), (30, 1000), (80, 500)]
    for sec in range(4):
        items = []
        for sid, (C, T) in enumerate(shapes):
            pre = np.zeros((C, T), dtype=bool)
            pre[sid::7] = True                          # whole channels known bad
            pre[:, (sec * 97) % T:(sec * 97) % T + 20] = True
            items.append((synth.ci8_block(rng, C, T), O.CI8, sid, pre))
        flags, st = run_pre(fl, items)
        for (x, _, sid, pre), f, s in zip(items, flags, st):
            r = O.flag_block(x, O.CI8, prm, history=h, stream_id=sid, preflags=pre)
            check_exact(s, f, r, fl.params)
            assert s["history_flagged_rows"] == int(r.history_rows.sum())
        fl.history_update(None)
        h.commit()
    exp = fl.history_export()
    for sid, (C, T) in enumerate(shapes):
        for c in range(C):
            ring = h.ring(sid, c)
            assert exp["counts"][sid, c] == len(ring)
            assert list(exp["values"][sid, c, :len(ring)]) == ring
    fl.close()


@pytest.mark.parametrize("dt", [O.F32, O.C64, O.C64_AMP])
def test_preflags_float(dt):
    say(f"[preflags_float] dtype={dt}")
    fl = make()
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(7400 + dt)
    items = []
    for C, T in [(64, 4096), (16, 768), (7, 6000), (256, 300)]:
        x = synth.f32_power_block(rng, C, T) if dt == O.F32 else synth.c64_block(rng, C, T)
        items.append((x, dt, -1, rng.random((C, T)) < 0.15))
    flags, st = run_pre(fl, items)
    for (x, _, _, pre), f, s in zip(items, flags, st):
        r = O.flag_block(x, dt, prm, preflags=pre)
        assert s["median"] == pytest.approx(r.median, rel=2e-7)
        assert s["stddev"] == pytest.approx(r.stddev, rel=1e-6)
        assert f[pre].all()
        assert mismatch(f, r.flags) / f.size <= 1e-3
    fl.close()


def test_preflags_argument_checks():
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as N
    say("[preflags_argument_checks]")
    with pytest.raises(RuntimeError):
        make(options=P.LOF_OPT_INTEGRATED)
    with pytest.raises(RuntimeError):
        make(partial_time=8)
    fl = make()
    x = synth.ci8_block(np.random.default_rng(1), 8, 256)
    d = torch.from_numpy(x).cuda()
    f = torch.zeros((8, 256), dtype=torch.uint8, device="cuda")
    arr = (N.LofBlock * 1)(P.Block(d, f, P.LOF_CI8, -1).to_c())
    assert fl._L.lof_autotune(fl._h, arr, 1, None, 1, None) == N.LOF_ERR_INVALID
    fl.close()
