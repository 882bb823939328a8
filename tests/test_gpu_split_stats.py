"""GPU: block statistics split over workgroups (calls of at most 64 blocks of a
kind, the largest of at least 65536 samples: each block's samples cut into parts,
the median and the MAD by radix passes over a shared histogram, one launch per
pass; Sec. 2.1 thresholds, Sec. 4.2 O(N) median and MAD) through the C ABI.

Complex int8 input is exact on both paths: median, stddev, thresholds and flags
bit for bit against the oracle and against the one-workgroup-per-block kernel
(the same blocks in a call padded past 64 blocks).  Float input: the same
median, and stddev and thresholds within 1e-12 relative of the one-workgroup
kernel (float64 part sums added in another order), flags within the float
criterion of the oracle.  Edge cases: one long row, every sample pre-flagged,
a constant block, both input kinds in one call, calls in a row and graph
replays (the split state clears itself)."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu

NPAD = 66   # tiny blocks that push a call past the split limit of 64 blocks per kind


def make(**kw):
    import paper_1701_08197_amd as P
    base = dict(max_streams=8, max_channels=1024, max_blocks_per_call=128, max_samples_per_call=1 << 23)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


def pad(items, dt):
    rng = np.random.default_rng(99)
    tiny = synth.ci8_block(rng, 1, 8) if dt == O.CI8 else synth.f32_power_block(rng, 1, 8)
    return items + [(tiny, dt, -1)] * NPAD


def exact_stats(s, r, nT):
    assert s["median"] == r.median
    assert s["stddev"] == r.stddev
    assert s["threshold"][:nT] == r.thresholds[:nT]


CI8_SHAPES = [(64, 3072), (256, 1024), (1, 70000), (7, 9999), (3, 7), (33, 2049)]


@pytest.mark.parametrize("opts", [0, 0x40, 0x10])
def test_split_ci8_exact_both_paths(opts):
    say(f"[split_ci8_exact_both_paths] options={opts}")
    fl = make(options=opts)
    prm = oracle_params(fl.params)
    nT = max(prm.n_levels, 7)
    rng = np.random.default_rng(8000 + opts)
    items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in CI8_SHAPES]
    f_split, st_split = run_gpu(fl, items)
    f_one, st_one = run_gpu(fl, pad(items, O.CI8))
    for (x, _, _), fs, ss, fo, so in zip(items, f_split, st_split, f_one, st_one):
        r = O.flag_block(x, O.CI8, prm)
        exact_stats(ss, r, nT)
        exact_stats(so, r, nT)
        assert mismatch(fs, r.flags) == 0, x.shape
        assert mismatch(fo, r.flags) == 0, x.shape
        assert ss["n_flagged"] == so["n_flagged"] == int(r.flags.sum())
    fl.close()


@pytest.mark.parametrize("dt", [O.F32, O.C64, O.C64_AMP])
@pytest.mark.parametrize("opts", [0, 0x40])
def test_split_float_against_one_workgroup(dt, opts):
    say(f"[split_float_against_one_workgroup] dtype={dt} options={opts}")
    fl = make(options=opts)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8100 + dt + opts)
    shapes = [(64, 4096), (256, 1024), (1, 66000), (5, 333)]
    gen = (lambda C, T: synth.f32_power_block(rng, C, T)) if dt == O.F32 else (lambda C, T: synth.c64_block(rng, C, T))
    items = [(gen(C, T), dt, -1) for C, T in shapes]
    f_split, st_split = run_gpu(fl, items)
    f_one, st_one = run_gpu(fl, pad(items, dt))
    for (x, _, _), fs, ss, fo, so in zip(items, f_split, st_split, f_one, st_one):
        assert ss["median"] == so["median"]
        assert ss["stddev"] == pytest.approx(so["stddev"], rel=1e-12, abs=0.0)
        for a, b in zip(ss["threshold"][:7], so["threshold"][:7]):
            assert a == pytest.approx(b, rel=1e-12)
        r = O.flag_block(x, dt, prm)
        assert ss["median"] == pytest.approx(r.median, rel=2e-7)
        assert ss["stddev"] == pytest.approx(r.stddev, rel=1e-6)
        assert mismatch(fs, r.flags) / fs.size <= 1e-3
        assert mismatch(fs, fo) / fs.size <= 1e-3
    fl.close()


def test_split_edge_cases():
    """One long row, a constant block (every key equal), a two-valued block, and
    a block of both kinds in the same call."""
    say("[split_edge_cases]")
    fl = make(options=0x40)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8200)
    const = np.full((32, 4096, 2), 5, dtype=np.int8)
    const[4, 100:140, 0] = 90
    two = rng.integers(0, 2, size=(64, 2048, 2)).astype(np.int8)
    items = [(synth.ci8_block(rng, 1, 131072), O.CI8, -1), (const, O.CI8, -1), (two, O.CI8, -1),
             (synth.f32_power_block(rng, 16, 8192), O.F32, -1)]
    flags, st = run_gpu(fl, items)
    for (x, dt, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, dt, prm)
        if dt == O.CI8:
            exact_stats(s, r, 7)
            assert mismatch(f, r.flags) == 0, x.shape
        else:
            assert s["median"] == pytest.approx(r.median, rel=2e-7)
            assert mismatch(f, r.flags) / f.size <= 1e-3
    fl.close()


def test_split_preflags_including_all_flagged():
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import Block, STATS_BYTES, decode_stats
    say("[split_preflags_including_all_flagged]")
    for opts in (0, 0x40):
        fl = make(options=P.LOF_OPT_PREFLAGGED | opts)
        prm = oracle_params(fl.params)
        rng = np.random.default_rng(8300 + opts)
        xs = [synth.ci8_block(rng, 64, 3072), synth.ci8_block(rng, 20, 4000), synth.ci8_block(rng, 128, 1024)]
        pres = [rng.random((64, 3072)) < 0.2, np.ones((20, 4000), dtype=bool), rng.random((128, 1024)) < 0.9]
        blocks, outs, keep = [], [], []
        for x, pre in zip(xs, pres):
            d = torch.from_numpy(x).cuda()
            f = torch.from_numpy(pre.astype(np.uint8)).cuda()
            keep.append(d)
            outs.append(f)
            blocks.append(Block(d, f, P.LOF_CI8, -1))
        stats = torch.zeros(len(xs) * STATS_BYTES, dtype=torch.uint8, device="cuda")
        fl.flag_blocks(blocks, stats=stats)
        torch.cuda.synchronize()
        st = decode_stats(stats.cpu().numpy().tobytes())
        for x, pre, f, s in zip(xs, pres, outs, st):
            r = O.flag_block(x, O.CI8, prm, preflags=pre)
            exact_stats(s, r, 7)
            assert mismatch(f.cpu().numpy(), r.flags) == 0
        assert st[1]["median"] == 0.0 and st[1]["stddev"] == 0.0
        fl.close()


def test_split_state_clears_between_calls_and_graph_replays():
    """Calls in a row on the same slots, with other data and other shapes, then
    one block table replayed as a graph with new data each time and the
    device's own work in between: every result is the oracle's."""
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import Block, STATS_BYTES, decode_stats
    say("[split_state_clears_between_calls_and_graph_replays]")
    fl = make(call_slots=2)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8400)
    for rep in range(5):
        shapes = [(64, 3072), (16, 8192)] if rep % 2 == 0 else [(200, 1000)]
        items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in shapes]
        flags, st = run_gpu(fl, items)
        for (x, _, _), f, s in zip(items, flags, st):
            r = O.flag_block(x, O.CI8, prm)
            exact_stats(s, r, 7)
            assert mismatch(f, r.flags) == 0, (rep, x.shape)
    fl.close()
    fg = make(options=P.LOF_OPT_GRAPH)
    shapes = [(64, 3072), (16, 8192), (3, 7)]
    ds = [torch.zeros((C, T, 2), dtype=torch.int8, device="cuda") for C, T in shapes]
    fs = [torch.zeros((C, T), dtype=torch.uint8, device="cuda") for C, T in shapes]
    blocks = [Block(d, f, P.LOF_CI8, -1) for d, f in zip(ds, fs)]
    stats = torch.zeros(len(shapes) * STATS_BYTES, dtype=torch.uint8, device="cuda")
    for rep in range(4):
        xs = [synth.ci8_block(rng, C, T) for C, T in shapes]
        for d, x in zip(ds, xs):
            d.copy_(torch.from_numpy(x))
        torch.cuda.synchronize()
        fg.flag_blocks(blocks, stats=stats)
        torch.cuda.synchronize()
        st = decode_stats(stats.cpu().numpy().tobytes())
        for x, f, s in zip(xs, fs, st):
            r = O.flag_block(x, O.CI8, prm)
            exact_stats(s, r, 7)
            assert mismatch(f.cpu().numpy(), r.flags) == 0, (rep, x.shape)
    fg.close()


def test_split_at_the_block_limit():
    """64 blocks of a kind (the most a split launch takes) with one large block
    among small ones of many shapes, in a context whose call limit is 64: every
    block exact against the oracle."""
    say("[split_at_the_block_limit]")
    fl = make(max_blocks_per_call=64)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8500)
    shapes = [(64, 3072)] + [(int(rng.integers(1, 40)), int(rng.integers(1, 700))) for _ in range(63)]
    items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in shapes]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.CI8, prm)
        exact_stats(s, r, 7)
        assert mismatch(f, r.flags) == 0, x.shape
    fl.close()
