"""GPU: the integrated pre-correlation mode (LOF_OPT_INTEGRATED, Sec. 4:
spectrum flagged along frequency first, then the time series of the unflagged
channels along time, flags broadcast back), through the C ABI, against the
oracle's integrated_block: bit-exact flags and series statistics on complex
int8 input (shapes from 1 x 1 to 1024 channels and 16384 times, SIR on, off
and the prose reading, history), float input within the float bound, and the
argument limit."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 100), (3, 7), (64, 3072), (16, 768), (7, 1000), (2, 5000), (70, 300), (256, 64),
          (33, 129), (1024, 40), (5, 16384), (64, 4097)]


def make(**kw):
    import paper_1701_08197_amd as P
    opts = kw.pop("options", 0) | P.LOF_OPT_INTEGRATED
    base = dict(max_streams=8, max_channels=1024, max_blocks_per_call=16, max_samples_per_call=1 << 22,
                options=opts)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


# float input: the series are float64 sums in another order; complex64 voltages
# also have their power formed in float32 on the GPU (2^-22 relative per
# sample), which the series' stddev (a difference of moments) can amplify
SERIES_REL = {O.F32: (1e-12, 1e-9), O.C64: (1e-5, 1e-4), O.C64_AMP: (1e-5, 1e-4)}


def check_stats(st, r, prm, C, T, dt=O.CI8):
    exact = dt == O.CI8
    med, sd, th = O.series_thresholds(r.series, prm, exact, min(prm.n_levels, 7))
    if exact:
        assert st["median"] == med and st["stddev"] == sd, (C, T)
        assert st["threshold"][:len(th)] == th
    else:
        rm, rs = SERIES_REL[dt]
        assert st["median"] == pytest.approx(med, rel=rm, abs=1e-300)
        assert st["stddev"] == pytest.approx(sd, rel=rs, abs=1e-12)


@pytest.mark.parametrize("kw", [dict(), dict(sir_eta_num=0), dict(options=0x10), dict(n_levels=3, n_levels_freq=2),
                                dict(sir_eta_num=1, sir_eta_den=2)])
def test_integrated_ci8_exact(kw):
    say(f"[integrated_ci8_exact] {kw}")
    fl = make(**kw)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(4000 + len(str(kw)))
    items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in SHAPES]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.integrated_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0, x.shape
        assert s["n_flagged"] == int(r.flags.sum())
        check_stats(s, r, prm, x.shape[0], x.shape[1])
    fl.close()


def test_integrated_structured_cases():
    """Blocks whose flags the oracle's pins fix: constant, broadband impulse,
    bursty tone removed before the time series, every channel flagged."""
    say("[integrated_structured_cases]")
    fl = make(sir_eta_num=0)
    prm = oracle_params(fl.params)

    def ci8(pw):
        re = np.sqrt(pw).astype(np.int64)
        x = np.zeros(pw.shape + (2,), dtype=np.int8)
        x[..., 0] = re
        return x
    imp = np.zeros((8, 64), dtype=np.int64)
    imp[:, 32] = 25
    tone = np.ones((40, 128), dtype=np.int64)
    tone[3] = 100
    tone[3, [20, 90]] = 10000
    loud = np.full((4, 50), 16, dtype=np.int64)
    loud[:, ::7] = 0
    items = [(ci8(np.full((16, 200), 49, dtype=np.int64)), O.CI8, -1), (ci8(imp), O.CI8, -1),
             (ci8(tone), O.CI8, -1), (ci8(loud), O.CI8, -1)]
    flags, _ = run_gpu(fl, items)
    for (x, _, _), f in zip(items, flags):
        r = O.integrated_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0
    assert not flags[0].any()
    assert (flags[1].astype(bool) == (np.arange(64) == 32)[None, :]).all()
    assert (flags[2].astype(bool) == (np.arange(40) == 3)[:, None]).all()
    fl.close()


def test_integrated_with_history_exact():
    say("[integrated_with_history_exact]")
    fl = make(history_len=5, history_min=2, history_sensitivity=2.0)
    prm = oracle_params(fl.params)
    h = O.History(prm)
    for sec in range(6):
        items = [(synth.config4_block(k, sec, k), O.CI8, k) for k in range(3)]
        if sec == 4:
            items[1] = (np.clip(items[1][0].astype(np.int16) * 3, -127, 127).astype(np.int8), O.CI8, 1)
        flags, st = run_gpu(fl, items)
        for k in range(3):
            r = O.integrated_block(items[k][0], O.CI8, prm, history=h, stream_id=k)
            assert mismatch(flags[k], r.flags) == 0, (sec, k)
            assert st[k]["history_flagged_rows"] == int(r.history_rows.sum())
        exp = fl.history_export()
        for k in range(3):
            for c in range(64):
                pv = h.pending.get((k, c))
                assert bool(exp["staged_valid"][k, c]) == (pv is not None)
                if pv is not None:
                    assert exp["staged"][k, c] == pv
        fl.history_update(None)
        h.commit()
    fl.close()


@pytest.mark.parametrize("dt,C,T", [(O.F32, 64, 4096), (O.C64, 64, 4096), (O.C64_AMP, 256, 1024),
                                    (O.F32, 16, 768), (O.F32, 1, 300)])
def test_integrated_float(dt, C, T):
    say(f"[integrated_float] dtype={dt} C={C} T={T}")
    fl = make()
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(C + T + dt)
    x = synth.f32_power_block(rng, C, T) if dt == O.F32 else synth.c64_block(rng, C, T)
    flags, st = run_gpu(fl, [(x, dt, -1)])
    r = O.integrated_block(x, dt, prm)
    mm = mismatch(flags[0], r.flags)
    say(f"    mismatch {mm} of {C * T}")
    assert mm / (C * T) <= 1e-3
    check_stats(st[0], r, prm, C, T, dt)
    fl.close()


def test_integrated_rejects_long_blocks():
    say("[integrated_rejects_long_blocks]")
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as N
    fl = make()
    x = torch.zeros((2, 16385, 2), dtype=torch.int8, device="cuda")
    f = torch.zeros((2, 16385), dtype=torch.uint8, device="cuda")
    arr = (N.LofBlock * 1)(P.Block(x, f, P.LOF_CI8, -1).to_c())
    assert fl.flag_blocks_raw(arr, 1) == N.LOF_ERR_INVALID
    fl.close()


@pytest.mark.parametrize("kw", [dict(), dict(options=0x10), dict(sir_eta_num=4, sir_eta_den=4),
                                dict(options=0x10, sir_eta_num=3, sir_eta_den=3), dict(options=0x40),
                                dict(sir_eta_num=2, sir_eta_den=3, n_levels_freq=4)])
def test_integrated_spectrum_rfi(kw):
    """Spectra with many RFI channels (single, adjacent groups, weak and strong)
    at channel counts on both sides of 64 (one wave or the whole group flags the
    spectrum): flags and series statistics bit for bit."""
    say(f"[integrated_spectrum_rfi] {kw}")
    fl = make(**kw)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(4500 + len(str(kw)))
    items = []
    for C in (1, 2, 3, 5, 31, 63, 64, 65, 100, 128):
        T = int(rng.integers(50, 400))
        x = synth.ci8_block(rng, C, T).astype(np.int16)
        for _ in range(int(rng.integers(0, max(1, C // 4) + 1))):
            c0 = int(rng.integers(0, C))
            w = int(rng.integers(1, 4))
            x[c0:c0 + w] *= int(rng.integers(2, 6))
        items.append((np.clip(x, -127, 127).astype(np.int8), O.CI8, -1))
    flags, st = run_gpu(fl, items)
    nfl = 0
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.integrated_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0, x.shape
        assert s["n_flagged"] == int(r.flags.sum())
        check_stats(s, r, prm, x.shape[0], x.shape[1])
        nfl += int(r.flags.any(axis=1).sum())
    say(f"    flagged channels {nfl}")
    fl.close()


@pytest.mark.parametrize("kw", [dict(), dict(options=0x40), dict(options=0x10, sir_eta_num=2, sir_eta_den=5)])
def test_integrated_every_channel_count(kw):
    """Every channel count from 1 to 66 (the spectrum flagged by one wave up to
    64 channels, odd and even counts for the two middle ranks, then by the whole
    group): flags and series statistics bit for bit."""
    say(f"[integrated_every_channel_count] {kw}")
    fl = make(max_blocks_per_call=70, **kw)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(4700 + len(str(kw)))
    items = []
    for C in range(1, 67):
        T = int(rng.integers(20, 120))
        x = synth.ci8_block(rng, C, T).astype(np.int16)
        for _ in range(int(rng.integers(0, C // 5 + 1))):
            c0 = int(rng.integers(0, C))
            x[c0:c0 + int(rng.integers(1, 3))] *= int(rng.integers(2, 5))
        items.append((np.clip(x, -127, 127).astype(np.int8), O.CI8, -1))
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.integrated_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0, x.shape
        assert s["n_flagged"] == int(r.flags.sum())
        check_stats(s, r, prm, x.shape[0], x.shape[1])
    fl.close()
