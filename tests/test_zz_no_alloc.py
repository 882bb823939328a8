"""GPU: the allocation-free entry point (lof_flag_blocks_static) against
lof_flag_blocks on the same blocks, through the C ABI: two calls in a row, the
second smaller; every flag byte equal, every statistic of a complex int8 block
equal, and of a float block the same median, flag counts and stddev and
thresholds within 1e-12 relative (lof_flag_blocks may split a large block's
statistics over workgroups, which adds the float64 moment sums in another
order); its capacity limits and argument checks."""
import numpy as np
import pytest

import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _blocks(rng, shapes, dtypes):
    out = []
    for (C, T), dt in zip(shapes, dtypes):
        if dt == 0:
            out.append((synth.ci8_block(rng, C, T), dt))
        elif dt == 2:
            out.append((synth.f32_power_block(rng, C, T), dt))
        else:
            out.append((synth.c64_block(rng, C, T), dt))
    return out


def _run(items, use_static, params):
    import torch
    import paper_1701_08197_amd as P
    blocks, flags, keep = [], [], []
    for x, dt in items:
        d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        f = torch.full((x.shape[0], x.shape[1]), 7, dtype=torch.uint8, device="cuda")
        keep.append(d)
        flags.append(f)
        blocks.append(P.Block(d, f, dt, -1))
    stats = torch.zeros(len(items) * P.STATS_BYTES, dtype=torch.uint8, device="cuda")
    if use_static:
        P.flag_blocks_static(params, blocks, stats=stats)
    else:
        fl = P.Flagger(params)
        fl.flag_blocks(blocks, stats=stats)
        torch.cuda.synchronize()
        fl.close()
    torch.cuda.synchronize()
    return [f.cpu().numpy() for f in flags], stats.cpu().numpy()


def test_static_equals_flag_blocks_two_calls():
    import paper_1701_08197_amd as P
    rng = np.random.default_rng(555)
    prm = P.default_params(max_streams=1, max_channels=256, max_blocks_per_call=64, max_samples_per_call=1 << 24)
    first = _blocks(rng, [(64, 3072)] * 6 + [(16, 768), (7, 1000), (256, 1024), (3, 5000), (1, 1)],
                    [0] * 6 + [2, 0, 3, 1, 0])
    second = _blocks(rng, [(64, 3072), (5, 100), (33, 129)], [0, 2, 0])
    for k, items in enumerate([first, second]):
        say(f"[static_equals_flag_blocks] call {k}: {len(items)} blocks")
        fs, ss = _run(items, True, prm)
        fr, sr = _run(items, False, prm)
        for i, (a, b) in enumerate(zip(fs, fr)):
            assert np.array_equal(a, b), (k, i)
        ds, dr = P.decode_stats(ss.tobytes()), P.decode_stats(sr.tobytes())
        for i, ((_, dt), a, b) in enumerate(zip(items, ds, dr)):
            if dt == 0:
                assert a == b, (k, i)
                continue
            assert a["median"] == b["median"], (k, i)
            assert a["n_flagged"] == b["n_flagged"] and a["history_flagged_rows"] == b["history_flagged_rows"]
            assert a["stddev"] == pytest.approx(b["stddev"], rel=1e-12, abs=0.0), (k, i)
            for x, y in zip(a["threshold"], b["threshold"]):
                assert x == pytest.approx(y, rel=1e-12, abs=0.0), (k, i)


def test_static_limits_and_errors():
    say("[static_limits_and_errors]")
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as N
    L = N.load()
    prm = P.default_params()
    x = torch.zeros((8, 128, 2), dtype=torch.int8, device="cuda")
    f = torch.full((8, 128), 5, dtype=torch.uint8, device="cuda")
    good = P.Block(x, f, P.LOF_CI8, -1).to_c()
    hist = P.Block(x, f, P.LOF_CI8, 0).to_c()
    arr = (N.LofBlock * 1)(hist)
    assert L.lof_flag_blocks_static(prm, 0, arr, 1, None, None) == N.LOF_ERR_INVALID
    assert b"stream_id" in L.lof_last_error(None)
    big = torch.zeros((64, 262144, 2), dtype=torch.int8, device="cuda")
    fb = torch.zeros((64, 262144), dtype=torch.uint8, device="cuda")
    too_big = [P.Block(big[:, :131072], fb[:, :131072], P.LOF_CI8, -1).to_c() for _ in range(40)]
    arr = (N.LofBlock * 40)(*too_big)
    assert L.lof_flag_blocks_static(prm, 0, arr, 40, None, None) == N.LOF_ERR_CAPACITY
    arr = (N.LofBlock * 1)(good)
    assert L.lof_flag_blocks_static(prm, 99, arr, 1, None, None) == N.LOF_ERR_INVALID
    torch.cuda.synchronize()
    assert (f.cpu().numpy() == 5).all()
    assert L.lof_flag_blocks_static(prm, 0, arr, 0, None, None) == N.LOF_OK
