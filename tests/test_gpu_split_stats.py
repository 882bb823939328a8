"""GPU: statistics of large float blocks split over workgroups (calls with at
most 4 float blocks whose largest has at least 65536 samples, or at most 16 with
the largest at least 2^20: each block's samples cut into parts, the median and
the MAD by radix passes over a shared histogram, one launch per pass; Sec. 2.1
thresholds, Sec. 4.2 O(N) median and MAD) through the C ABI.

Against the one-workgroup-per-block kernel (the same blocks in a call padded
past 16 float blocks): the same median, stddev and thresholds within 1e-12
relative (float64 part sums added in another order), flags within the float
criterion.  Against the oracle: float32 input has the oracle's median exactly,
stddev and thresholds within 1e-9 (1e-6 with the MAD, an order statistic of
float32 deviations on the GPU); complex64 input (powers formed in float32)
within 2e-7 / 1e-6; flags within the float criterion.  Edge cases: one long
row, a constant block (every key equal), a two-valued block, complex int8
blocks in the same call (one workgroup each, exact), every sample pre-flagged,
calls in a row and graph replays (the split state clears itself), the 16-block
limit."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu

NPAD = 17   # tiny float blocks that push a call past the split limit of 16 float blocks


def make(**kw):
    import paper_1701_08197_amd as P
    base = dict(max_streams=8, max_channels=1024, max_blocks_per_call=64, max_samples_per_call=1 << 24)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


def pad(items):
    tiny = synth.f32_power_block(np.random.default_rng(99), 1, 8)
    return items + [(tiny, O.F32, -1)] * NPAD


def gen(rng, dt, C, T):
    return synth.f32_power_block(rng, C, T) if dt == O.F32 else synth.c64_block(rng, C, T)


def check_oracle(s, f, r, dt, robust=False):
    if dt == O.F32:
        # the MAD is an order statistic of float32 deviations on the GPU (float64
        # in the oracle): float32 rounding of the stddev
        rel = 1e-6 if robust else 1e-9
        assert s["median"] == r.median
        assert s["stddev"] == pytest.approx(r.stddev, rel=rel, abs=1e-300)
        for a, b in zip(s["threshold"][:7], r.thresholds[:7]):
            assert a == pytest.approx(b, rel=rel, abs=1e-300)
    else:
        assert s["median"] == pytest.approx(r.median, rel=2e-7)
        assert s["stddev"] == pytest.approx(r.stddev, rel=1e-6)
    assert mismatch(f, r.flags) / f.size <= 1e-3


def exact_stats(s, r, nT):
    assert s["median"] == r.median
    assert s["stddev"] == r.stddev
    assert s["threshold"][:nT] == r.thresholds[:nT]


@pytest.mark.parametrize("dt", [O.F32, O.C64, O.C64_AMP])
@pytest.mark.parametrize("opts", [0, 0x40])
def test_split_float_against_one_workgroup_and_oracle(dt, opts):
    say(f"[split_float_against_one_workgroup_and_oracle] dtype={dt} options={opts}")
    fl = make(options=opts)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8100 + dt + opts)
    shapes = [(64, 4096), (256, 1024), (1, 66000), (5, 333)]
    items = [(gen(rng, dt, C, T), dt, -1) for C, T in shapes]
    f_split, st_split = run_gpu(fl, items)
    f_one, st_one = run_gpu(fl, pad(items))
    for (x, _, _), fs, ss, fo, so in zip(items, f_split, st_split, f_one, st_one):
        assert ss["median"] == so["median"]
        assert ss["stddev"] == pytest.approx(so["stddev"], rel=1e-12, abs=0.0)
        for a, b in zip(ss["threshold"][:7], so["threshold"][:7]):
            assert a == pytest.approx(b, rel=1e-12)
        assert mismatch(fs, fo) / fs.size <= 1e-3
        check_oracle(ss, fs, O.flag_block(x, dt, prm), dt, robust=opts == 0x40)
    fl.close()


def test_split_edge_cases():
    """One long row, a constant block, a two-valued block, and complex int8
    blocks in the same call."""
    say("[split_edge_cases]")
    fl = make(options=0x40)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8200)
    const = np.full((32, 4096), 5.0, dtype=np.float32)
    const[4, 100:140] = 90.0
    two = rng.integers(1, 3, size=(64, 2048)).astype(np.float32)
    items = [(synth.f32_power_block(rng, 1, 131072), O.F32, -1), (const, O.F32, -1), (two, O.F32, -1),
             (synth.ci8_block(rng, 64, 3072), O.CI8, -1), (synth.ci8_block(rng, 1, 70000), O.CI8, -1)]
    flags, st = run_gpu(fl, items)
    for (x, dt, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, dt, prm)
        if dt == O.CI8:
            exact_stats(s, r, 7)
            assert mismatch(f, r.flags) == 0, x.shape
        else:
            check_oracle(s, f, r, dt, robust=True)
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
        xs = [synth.f32_power_block(rng, 64, 3072), synth.f32_power_block(rng, 20, 4000),
              synth.f32_power_block(rng, 128, 1024)]
        pres = [rng.random((64, 3072)) < 0.2, np.ones((20, 4000), dtype=bool), rng.random((128, 1024)) < 0.9]
        blocks, outs, keep = [], [], []
        for x, pre in zip(xs, pres):
            d = torch.from_numpy(x).cuda()
            f = torch.from_numpy(pre.astype(np.uint8)).cuda()
            keep.append(d)
            outs.append(f)
            blocks.append(Block(d, f, P.LOF_F32, -1))
        stats = torch.zeros(len(xs) * STATS_BYTES, dtype=torch.uint8, device="cuda")
        fl.flag_blocks(blocks, stats=stats)
        torch.cuda.synchronize()
        st = decode_stats(stats.cpu().numpy().tobytes())
        for x, pre, f, s in zip(xs, pres, outs, st):
            r = O.flag_block(x, O.F32, prm, preflags=pre)
            check_oracle(s, f.cpu().numpy(), r, O.F32, robust=opts == 0x40)
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
        items = [(synth.f32_power_block(rng, C, T), O.F32, -1) for C, T in shapes]
        flags, st = run_gpu(fl, items)
        for (x, _, _), f, s in zip(items, flags, st):
            check_oracle(s, f, O.flag_block(x, O.F32, prm), O.F32)
    fl.close()
    fg = make(options=P.LOF_OPT_GRAPH)
    shapes = [(64, 3072), (16, 8192), (3, 7)]
    ds = [torch.zeros((C, T), dtype=torch.float32, device="cuda") for C, T in shapes]
    fs = [torch.zeros((C, T), dtype=torch.uint8, device="cuda") for C, T in shapes]
    blocks = [Block(d, f, P.LOF_F32, -1) for d, f in zip(ds, fs)]
    stats = torch.zeros(len(shapes) * STATS_BYTES, dtype=torch.uint8, device="cuda")
    for rep in range(4):
        xs = [synth.f32_power_block(rng, C, T) for C, T in shapes]
        for d, x in zip(ds, xs):
            d.copy_(torch.from_numpy(x))
        torch.cuda.synchronize()
        fg.flag_blocks(blocks, stats=stats)
        torch.cuda.synchronize()
        st = decode_stats(stats.cpu().numpy().tobytes())
        for x, f, s in zip(xs, fs, st):
            check_oracle(s, f.cpu().numpy(), O.flag_block(x, O.F32, prm), O.F32)
    fg.close()


def test_split_at_the_block_limit():
    """16 float blocks (the most a split launch takes), the largest of 2^20
    samples, among small ones of many shapes, in a context whose call limit is
    16: every block against the oracle."""
    say("[split_at_the_block_limit]")
    fl = make(max_blocks_per_call=16)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(8500)
    shapes = [(256, 4096)] + [(int(rng.integers(1, 40)), int(rng.integers(1, 700))) for _ in range(15)]
    items = [(synth.f32_power_block(rng, C, T), O.F32, -1) for C, T in shapes]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        check_oracle(s, f, O.flag_block(x, O.F32, prm), O.F32)
    fl.close()
