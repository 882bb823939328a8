"""GPU: history flagger across calls, parameter/option variants, argument
validation and the full-size 48-station workload, all through the C ABI and
compared with the CPU reference."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu


def make(**kw):
    import paper_1701_08197_amd as P
    base = dict(max_streams=16, max_channels=256, max_blocks_per_call=16, max_samples_per_call=1 << 22)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


def history_case(seed, steps, C, T, n_streams, level_jump_step=None):
    rng = np.random.default_rng(seed)
    blocks = []
    for s in range(steps):
        row = []
        for st in range(n_streams):
            x = synth.ci8_block(rng, C, T, rfi=(s % 3 == 0))
            if level_jump_step is not None and s == level_jump_step and st == 0:
                x = np.clip(x.astype(np.int16) * 3, -127, 127).astype(np.int8)
            row.append(x)
        blocks.append(row)
    return blocks


@pytest.mark.parametrize("literal,winsor", [(False, 0), (True, 0), (False, 2)])
def test_history_sequence_exact(literal, winsor):
    """Flags, staged values and rings over 10 steps; with winsor = 2 the ring's
    statistics are those of the winsorized ring (k = 1 or 2 as it fills)."""
    say(f"[history_sequence_exact] literal={literal} winsor={winsor}")
    opts = 0x2 if literal else 0
    fl = make(history_len=6, history_min=3, history_sensitivity=2.0, options=opts, history_winsor=winsor)
    prm = oracle_params(fl.params)
    h = O.History(prm)
    steps, C, T, ns = 10, 24, 500, 3
    data = history_case(7, steps, C, T, ns, level_jump_step=7)
    for s in range(steps):
        items = [(data[s][st], O.CI8, st) for st in range(ns)]
        flags, st = run_gpu(fl, items)
        for k in range(ns):
            r = O.flag_block(data[s][k], O.CI8, prm, history=h, stream_id=k)
            assert mismatch(flags[k], r.flags) == 0, (s, k)
            assert st[k]["history_flagged_rows"] == int(r.history_rows.sum())
        exp = fl.history_export()
        for k in range(ns):
            for c in range(C):
                pv = h.pending.get((k, c))
                assert bool(exp["staged_valid"][k, c]) == (pv is not None)
                if pv is not None:
                    assert exp["staged"][k, c] == pv
        fl.history_update(list(range(ns)))
        h.commit()
        exp = fl.history_export()
        for k in range(ns):
            for c in range(C):
                ring = h.ring(k, c)
                assert exp["counts"][k, c] == len(ring)
                assert list(exp["values"][k, c, :len(ring)]) == ring
    fl.close()


def test_history_commit_selected_streams_and_autocommit():
    say("[history_commit_selected_streams_and_autocommit]")
    import paper_1701_08197_amd as P
    fl = make(history_len=4, history_min=1)
    x = synth.ci8_block(np.random.default_rng(3), 8, 256)
    run_gpu(fl, [(x, O.CI8, 0), (x, O.CI8, 1)])
    fl.history_update([1])                         # only stream 1 commits
    exp = fl.history_export()
    assert (exp["counts"][0, :8] == 0).all() and (exp["counts"][1, :8] == 1).all()
    assert (exp["staged_valid"][0, :8] == 1).all() and (exp["staged_valid"][1, :8] == 0).all()
    fl.history_update(None)                        # everything pending
    exp = fl.history_export()
    assert (exp["counts"][0, :8] == 1).all()
    fl.close()
    fa = make(history_len=4, history_min=1, options=P.LOF_OPT_AUTOCOMMIT)
    run_gpu(fa, [(x, O.CI8, 5)])
    exp = fa.history_export()
    assert (exp["counts"][5, :8] == 1).all() and (exp["staged_valid"][5, :8] == 0).all()
    fa.close()


@pytest.mark.parametrize("kw", [dict(n_levels=1), dict(n_levels=3), dict(n_levels_freq=0),
                                dict(n_levels_freq=2), dict(sir_eta_num=0), dict(sir_eta_num=1, sir_eta_den=2),
                                dict(sir_eta_num=3, sir_eta_den=3), dict(start_threshold=3.0, p=1.3),
                                dict(sensitivity=0.7)])
def test_parameter_variants_exact(kw):
    say(f"[parameter_variants_exact] {kw}")
    fl = make(**kw)
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(11)
    items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in [(64, 3072), (16, 768), (5, 5000), (100, 300)]]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0
        assert s["median"] == r.median and s["stddev"] == r.stddev
    fl.close()


def test_invalid_calls_change_nothing():
    say("[invalid_calls_change_nothing]")
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as N
    fl = make(max_streams=4, max_channels=64, max_blocks_per_call=4, max_samples_per_call=64 * 4096)
    x = torch.from_numpy(synth.ci8_block(np.random.default_rng(1), 8, 128)).cuda()
    f = torch.full((8, 128), 5, dtype=torch.uint8, device="cuda")
    good = P.Block(x, f, P.LOF_CI8, 0)
    bad_cases = []
    b1 = good.to_c(); b1.stream_id = 9; bad_cases.append(([good.to_c(), b1], N.LOF_ERR_INVALID))
    b2 = good.to_c(); bad_cases.append(([good.to_c(), b2], N.LOF_ERR_INVALID))          # repeated id
    b3 = good.to_c(); b3.dtype = 7; bad_cases.append(([b3], N.LOF_ERR_INVALID))
    b4 = good.to_c(); b4.data_row_stride = 10; bad_cases.append(([b4], N.LOF_ERR_INVALID))
    b5 = good.to_c(); b5.n_channels = 65; bad_cases.append(([b5], N.LOF_ERR_CAPACITY))
    b6 = good.to_c(); b6.n_times = 0; bad_cases.append(([b6], N.LOF_ERR_INVALID))
    b7 = good.to_c(); b7.data = None; bad_cases.append(([b7], N.LOF_ERR_INVALID))
    bad_cases.append(([good.to_c()] * 5, N.LOF_ERR_CAPACITY))
    for blocks, code in bad_cases:
        arr = (N.LofBlock * len(blocks))(*blocks)
        assert fl.flag_blocks_raw(arr, len(blocks)) == code
    torch.cuda.synchronize()
    assert (f.cpu().numpy() == 5).all()                 # nothing was written
    exp = fl.history_export()
    assert (exp["staged_valid"] == 0).all() and (exp["counts"] == 0).all()
    assert fl.flag_blocks_raw((N.LofBlock * 1)(), 0) == 0  # empty call
    with pytest.raises(P.LofError):
        fl.history_update([17])
    fl.close()


def test_config1_full_second_sampled():
    """All 6144 blocks of the 48-station second in one call (the benchmark's
    launch), then sampled blocks against the reference, bit for bit."""
    say("[config1_full_second_sampled] generating")
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd import _native as N
    import bench
    nb = synth.CONFIG1_BLOCKS
    host, shm = bench.make_config1(nb, 16, start_method="spawn")
    data = torch.from_numpy(host).cuda()
    del host
    shm.close()
    shm.unlink()
    flags = torch.zeros((nb, 64, 3072), dtype=torch.uint8, device="cuda")
    fl = P.Flagger(P.default_params(max_streams=nb, max_channels=64, max_blocks_per_call=nb,
                                    max_samples_per_call=nb * 64 * 3072))
    arr = (N.LofBlock * nb)()
    for b in range(nb):
        blk = arr[b]
        blk.data = data[b].data_ptr(); blk.flags = flags[b].data_ptr()
        blk.data_row_stride = 3072; blk.flag_row_stride = 3072
        blk.n_channels = 64; blk.n_times = 3072; blk.dtype = 0; blk.stream_id = b
    stats = torch.zeros(nb * P.STATS_BYTES, dtype=torch.uint8, device="cuda")
    say("[config1_full_second_sampled] flagging")
    assert fl.flag_blocks_raw(arr, nb, None, stats.data_ptr()) == 0
    torch.cuda.synchronize()
    st = P.decode_stats(stats.cpu().numpy().tobytes())
    rng = np.random.default_rng(2024)
    sample = sorted(set([0, nb - 1] + rng.choice(nb, size=6, replace=False).tolist()))
    prm = O.Params()
    for b in sample:
        x = synth.config1_block(b)
        r = O.flag_block(x, O.CI8, prm, history=O.History(prm), stream_id=b)
        got = flags[b].cpu().numpy()
        assert mismatch(got, r.flags) == 0, b
        assert st[b]["median"] == r.median and st[b]["stddev"] == r.stddev
        assert st[b]["n_flagged"] == int(r.flags.sum())
    # properties at full size: flags are 0/1 and every block's count matches its bytes
    tot = int(flags.sum().item())
    assert tot == sum(s["n_flagged"] for s in st)
    fl.close()
