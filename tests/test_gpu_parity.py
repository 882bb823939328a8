"""GPU parity: the HIP library (through the C ABI) against the CPU reference on
the same seeded inputs.  Integer (complex int8) input must match bit for bit:
flags, median, stddev and every threshold.  Float input: flags may differ only
where a window's unflagged mean lies within 1e-6 (relative) of its threshold;
the end-to-end mismatch rate is bounded and reported."""
import math

import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[1, 2], ids=["fused_post", "chunked_post"])
def lof(request):
    """Blocks of at most 64 channels and 4096 times take either the one-kernel
    SIR/history/bytes pass (fuse_post = 1) or the row- and column-chunked kernels
    (fuse_post = 2): every test runs on both."""
    import torch  # noqa: F401
    import paper_1701_08197_amd as P
    fl = P.Flagger(P.default_params(max_streams=64, max_channels=1024, max_blocks_per_call=64,
                                    max_samples_per_call=1 << 24))
    t = fl.get_tuning()
    t.fuse_post = request.param
    fl.set_tuning(t)
    yield fl
    fl.close()


def ci8_case(seed, C, T, rfi=True):
    rng = np.random.default_rng(seed)
    return synth.ci8_block(rng, C, T, sigma=16.0, rfi=rfi)


CI8_SHAPES = [(1, 1), (1, 5), (3, 7), (1, 34), (1, 35), (1, 64), (2, 65), (5, 100), (16, 768),
              (7, 1000), (3, 2049), (64, 3072), (4, 4096), (2, 4097), (2, 5000), (1, 9001),
              (70, 300), (130, 200), (256, 64), (33, 129), (17, 3000), (64, 64)]


@pytest.mark.parametrize("C,T", CI8_SHAPES)
def test_ci8_exact(lof, C, T):
    say(f"[ci8_exact] C={C} T={T}")
    x = ci8_case(1000 + C * 7 + T, C, T)
    flags, st = run_gpu(lof, [(x, O.CI8, -1)])
    r = O.flag_block(x, O.CI8, oracle_params(lof.params))
    assert st[0]["median"] == r.median
    assert st[0]["stddev"] == r.stddev
    nT = max(lof.params.n_levels, lof.params.n_levels_freq if lof.params.n_levels_freq >= 0 else 0)
    assert st[0]["threshold"][:nT] == r.thresholds[:nT]
    assert mismatch(flags[0], r.flags) == 0
    assert set(np.unique(flags[0])) <= {0, 1}
    assert st[0]["n_flagged"] == int(r.flags.sum())


@pytest.mark.parametrize("variant", ["const", "zeros", "one_hot", "dense_rfi", "max_power"])
def test_ci8_degenerate(lof, variant):
    say(f"[ci8_degenerate] {variant}")
    C, T = 8, 512
    x = np.zeros((C, T, 2), dtype=np.int8)
    if variant == "const":
        x[..., 0] = 3
        x[..., 1] = -4
    elif variant == "one_hot":
        x[2, 100, 0] = 120
    elif variant == "dense_rfi":
        x = ci8_case(5, C, T)
        x[:, ::3, 0] = 127
    elif variant == "max_power":
        x[...] = -128
    flags, st = run_gpu(lof, [(x, O.CI8, -1)])
    r = O.flag_block(x, O.CI8, oracle_params(lof.params))
    assert mismatch(flags[0], r.flags) == 0
    assert st[0]["median"] == r.median and st[0]["stddev"] == r.stddev


@pytest.mark.parametrize("variant", ["const", "ternary", "mostly_zero"])
def test_ci8_histogram_wrap(lof, variant):
    """Blocks where one power value occurs 2^16 times or more: the packed 16-bit
    histogram counters wrap, so the median comes from the radix select and the
    power sums from the samples."""
    say(f"[ci8_histogram_wrap] {variant}")
    C, T = 64, 3072
    rng = np.random.default_rng(4242)
    if variant == "const":
        x = np.full((C, T, 2), 5, dtype=np.int8)
    elif variant == "ternary":
        x = rng.integers(-1, 2, size=(C, T, 2)).astype(np.int8)
    else:
        x = np.zeros((C, T, 2), dtype=np.int8)
        x[:, ::7, 0] = rng.integers(-128, 128, size=(C, len(range(0, T, 7)))).astype(np.int8)
    flags, st = run_gpu(lof, [(x, O.CI8, -1)])
    r = O.flag_block(x, O.CI8, oracle_params(lof.params))
    assert st[0]["median"] == r.median and st[0]["stddev"] == r.stddev
    assert mismatch(flags[0], r.flags) == 0


@pytest.mark.parametrize("sens", [-1.0, 0.0, 1e-3, 0.3, 40.0, 1e12])
def test_ci8_threshold_extremes(sens):
    """Thresholds below zero, at the median and above any window sum: the clamps of
    the packed window-threshold table and its entry shared by counts 0 and 64."""
    import torch  # noqa: F401
    import paper_1701_08197_amd as P
    say(f"[ci8_threshold_extremes] sensitivity={sens}")
    fl = P.Flagger(P.default_params(max_streams=8, max_channels=64, max_blocks_per_call=4,
                                    max_samples_per_call=1 << 20, sensitivity=sens))
    try:
        items = [(ci8_case(321, 64, 3072), O.CI8, -1), (ci8_case(322, 16, 300), O.CI8, -1),
                 (np.full((8, 200, 2), -128, dtype=np.int8), O.CI8, -1)]   # p = 2^15 everywhere, sigma 0
        flags, st = run_gpu(fl, items)
        prm = oracle_params(fl.params)
        for (x, _, _), f, s in zip(items, flags, st):
            r = O.flag_block(x, O.CI8, prm)
            assert mismatch(f, r.flags) == 0
            assert s["threshold"][:7] == r.thresholds[:7]
    finally:
        fl.close()


def test_ci8_batch_mixed_shapes(lof):
    say("[ci8_batch_mixed_shapes]")
    shapes = [(64, 3072), (16, 768), (3, 5000), (256, 100), (1, 1), (64, 4096), (40, 2100)]
    items = [(ci8_case(77 + i, C, T), O.CI8, -1) for i, (C, T) in enumerate(shapes)]
    flags, st = run_gpu(lof, items)
    prm = oracle_params(lof.params)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0
        assert s["median"] == r.median and s["stddev"] == r.stddev


def test_strided_and_unaligned_rows(lof):
    say("[strided_and_unaligned_rows]")
    import torch
    from paper_1701_08197_amd import Block, LOF_CI8
    C, T = 12, 999
    x = ci8_case(9, C, T)
    big = np.zeros((C, T + 37, 2), dtype=np.int8)
    big[:, 3:3 + T] = x
    d = torch.from_numpy(big).cuda()[:, 3:3 + T]          # row stride T+37, 6-byte offset
    fbig = torch.full((C, T + 11), 9, dtype=torch.uint8, device="cuda")
    f = fbig[:, 1:1 + T]
    lof.flag_blocks([Block(d, f, LOF_CI8, -1)])
    torch.cuda.synchronize()
    r = O.flag_block(x, O.CI8, oracle_params(lof.params))
    assert mismatch(f.cpu().numpy(), r.flags) == 0
    fb = fbig.cpu().numpy()
    assert (fb[:, 0] == 9).all() and (fb[:, 1 + T:] == 9).all()   # nothing written outside


FLOAT_CASES = [(O.F32, 1, 100), (O.F32, 16, 768), (O.F32, 64, 4096), (O.F32, 256, 1024),
               (O.F32, 7, 6000), (O.C64, 64, 4096), (O.C64, 3, 333), (O.C64_AMP, 256, 1024),
               (O.C64_AMP, 32, 2500)]


def float_block(dt, C, T, seed):
    rng = np.random.default_rng(seed)
    if dt == O.F32:
        return synth.f32_power_block(rng, C, T)
    return synth.c64_block(rng, C, T)


@pytest.mark.parametrize("dt,C,T", FLOAT_CASES)
def test_float_parity(lof, dt, C, T):
    say(f"[float_parity] dtype={dt} C={C} T={T}")
    x = float_block(dt, C, T, 31 + C + T)
    flags, st = run_gpu(lof, [(x, dt, -1)])
    r = O.flag_block(x, dt, oracle_params(lof.params))
    assert st[0]["median"] == pytest.approx(r.median, rel=2e-7)
    assert st[0]["stddev"] == pytest.approx(r.stddev, rel=1e-6)
    for a, b in zip(st[0]["threshold"][:7], r.thresholds[:7]):
        assert a == pytest.approx(b, rel=1e-6)
    mm = mismatch(flags[0], r.flags)
    rate = mm / flags[0].size
    say(f"    mismatch {mm} / {flags[0].size} = {rate:.3g}")
    assert rate <= 1e-3


def test_config0_block(lof):
    say("[config0_block]")
    x, dt = synth.config0()
    flags, st = run_gpu(lof, [(x, dt, -1)])
    r = O.flag_block(x, dt, oracle_params(lof.params))
    mm = mismatch(flags[0], r.flags)
    say(f"    config0 mismatch {mm} / {x.size}")
    assert mm / x.size <= 1e-4
