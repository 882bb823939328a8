"""GPU: the robust stddev (LOF_OPT_ROBUST_SIGMA, Sec. 4.2 lists the MAD among the
statistics: stddev := 1.4826 * median(|x - median(x)|)) through the C ABI,
against the oracle's block_mad_sigma.  Complex int8 input is exact: median,
stddev, every threshold and the flags match bit for bit, on the packed histogram
and on the radix-select path taken when a histogram counter wraps.  Float input
within the float bound.  The integrated mode's series use the same statistic."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu


def make(**kw):
    import paper_1701_08197_amd as P
    opts = kw.pop("options", 0) | P.LOF_OPT_ROBUST_SIGMA
    base = dict(max_streams=8, max_channels=1024, max_blocks_per_call=32, max_samples_per_call=1 << 22,
                options=opts)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


@pytest.fixture(scope="module")
def lof():
    import torch  # noqa: F401
    fl = make()
    yield fl
    fl.close()


SHAPES = [(1, 1), (1, 2), (3, 7), (1, 64), (2, 65), (16, 768), (7, 1000), (64, 3072), (2, 5000), (70, 300),
          (256, 64), (33, 129), (64, 4096)]


def check_exact(st, r, params):
    nT = max(params.n_levels, params.n_levels_freq if params.n_levels_freq >= 0 else 0)
    assert st["median"] == r.median
    assert st["stddev"] == r.stddev
    assert st["threshold"][:nT] == r.thresholds[:nT]


def test_robust_ci8_exact(lof):
    say("[robust_ci8_exact]")
    prm = oracle_params(lof.params)
    assert prm.robust_sigma
    rng = np.random.default_rng(5100)
    items = [(synth.ci8_block(rng, C, T, sigma=16.0), O.CI8, -1) for C, T in SHAPES]
    flags, st = run_gpu(lof, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.CI8, prm)
        check_exact(s, r, lof.params)
        assert mismatch(f, r.flags) == 0, x.shape
        assert s["n_flagged"] == int(r.flags.sum())
    # the statistic differs from the plain stddev on RFI-contaminated blocks
    x = items[7][0]
    assert st[7]["stddev"] != O.block_stddev(O.power(x, O.CI8), True)


@pytest.mark.parametrize("variant", ["const", "ternary", "mostly_zero", "two_level", "extreme"])
def test_robust_ci8_special(lof, variant):
    """Blocks with a zero MAD, power values that occur 2^16 times or more (the
    packed histogram wraps: deviations by radix select over the samples), and
    the extreme deviations 0 and 2^16."""
    say(f"[robust_ci8_special] {variant}")
    C, T = 64, 3072
    rng = np.random.default_rng(4243)
    if variant == "const":
        x = np.full((C, T, 2), 5, dtype=np.int8)
    elif variant == "ternary":
        x = rng.integers(-1, 2, size=(C, T, 2)).astype(np.int8)
    elif variant == "mostly_zero":
        x = np.zeros((C, T, 2), dtype=np.int8)
        x[:, ::7, 0] = rng.integers(-128, 128, size=(C, len(range(0, T, 7)))).astype(np.int8)
    elif variant == "two_level":
        C, T = 8, 500        # half the samples at 0, half at 2^15: MAD = 2^14
        x = np.zeros((C, T, 2), dtype=np.int8)
        x[:, ::2] = -128
    else:
        C, T = 9, 333        # most samples 0, some at the largest power 2^15
        x = np.zeros((C, T, 2), dtype=np.int8)
        x[:, ::5] = -128
    flags, st = run_gpu(lof, [(x, O.CI8, -1)])
    r = O.flag_block(x, O.CI8, oracle_params(lof.params))
    check_exact(st[0], r, lof.params)
    assert mismatch(flags[0], r.flags) == 0


def test_robust_ci8_with_history_and_sir_variants():
    """The robust statistic with the fused SIR / history pass, the separate SIR
    kernels (blocks past 64 channels) and the prose SIR reading."""
    import paper_1701_08197_amd as P
    say("[robust_ci8_with_history_and_sir_variants]")
    for opts in (0, P.LOF_OPT_SIR_PROSE):
        fl = make(options=opts, history_len=4, history_min=1)
        prm = oracle_params(fl.params)
        rng = np.random.default_rng(5200 + opts)
        hist = O.History(prm)
        for sec in range(3):
            items = [(synth.ci8_block(rng, C, T, sigma=16.0), O.CI8, sid)
                     for sid, (C, T) in enumerate([(16, 768), (100, 300), (64, 4096)])]
            flags, st = run_gpu(fl, items)
            for (x, _, sid), f, s in zip(items, flags, st):
                r = O.flag_block(x, O.CI8, prm, history=hist, stream_id=sid)
                check_exact(s, r, fl.params)
                assert mismatch(f, r.flags) == 0, (opts, sec, x.shape)
                assert s["history_flagged_rows"] == int(r.history_rows.sum())
            fl.history_update(None)
            hist.commit()
        fl.close()


FLOAT_CASES = [(O.F32, 1, 100), (O.F32, 16, 768), (O.F32, 64, 4096), (O.F32, 7, 6000), (O.C64, 64, 4096),
               (O.C64, 3, 333), (O.C64_AMP, 256, 1024)]


@pytest.mark.parametrize("dt,C,T", FLOAT_CASES)
def test_robust_float(lof, dt, C, T):
    say(f"[robust_float] dtype={dt} C={C} T={T}")
    rng = np.random.default_rng(5300 + C + T)
    x = synth.f32_power_block(rng, C, T) if dt == O.F32 else synth.c64_block(rng, C, T)
    flags, st = run_gpu(lof, [(x, dt, -1)])
    r = O.flag_block(x, dt, oracle_params(lof.params))
    # the deviations are rounded to float32 on both sides (from the exact and
    # from the float32-rounded median): the MAD agrees to a few float32 ulps
    assert st[0]["median"] == pytest.approx(r.median, rel=2e-7)
    assert st[0]["stddev"] == pytest.approx(r.stddev, rel=1e-6)
    mm = mismatch(flags[0], r.flags)
    say(f"    mismatch {mm} / {flags[0].size}")
    assert mm / flags[0].size <= 1e-3


INTEG_SHAPES = [(1, 1), (3, 7), (64, 3072), (16, 768), (2, 5000), (70, 300), (1024, 40), (5, 16384)]


@pytest.mark.parametrize("opts", [0, 0x10])
def test_robust_integrated_ci8_exact(opts):
    import paper_1701_08197_amd as P
    say(f"[robust_integrated_ci8_exact] options={opts}")
    fl = make(options=opts | P.LOF_OPT_INTEGRATED, max_blocks_per_call=16)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(5400 + opts)
    items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in INTEG_SHAPES]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.integrated_block(x, O.CI8, prm)
        med, sd, th = O.series_thresholds(r.series, prm, True, min(prm.n_levels, 7))
        assert s["median"] == med and s["stddev"] == sd, x.shape
        assert s["threshold"][:len(th)] == th
        assert mismatch(f, r.flags) == 0, x.shape
    fl.close()


def test_robust_integrated_float():
    import paper_1701_08197_amd as P
    say("[robust_integrated_float]")
    fl = make(options=P.LOF_OPT_INTEGRATED, max_blocks_per_call=16)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(5500)
    items = [(synth.f32_power_block(rng, C, T), O.F32, -1) for C, T in [(64, 3072), (16, 768), (3, 5000)]]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.integrated_block(x, O.F32, prm)
        med, sd, _ = O.series_thresholds(r.series, prm, False, min(prm.n_levels, 7))
        assert s["median"] == pytest.approx(med, rel=1e-12)
        assert s["stddev"] == pytest.approx(sd, rel=1e-9)
        assert mismatch(f, r.flags) / x.size <= 1e-3, x.shape
    fl.close()
