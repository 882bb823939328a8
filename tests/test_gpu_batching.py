"""GPU: batched uneven blocks.  Results must not depend on the launch tuning
(time layout per length bucket, one workgroup per work item vs persistent grid),
hipGraph replays must equal eager calls on every replay, and the autotuner must
leave results unchanged."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, say

pytestmark = pytest.mark.gpu


def uneven_items(seed, n, float_share=0.5):
    rng = np.random.default_rng(seed)
    items = []
    for i in range(n):
        C = int(rng.choice([16, 64, 256]))
        T = int(rng.integers(300, 9000))
        if C * T > 900_000:
            T = 900_000 // C
        if rng.random() < float_share:
            items.append((synth.f32_power_block(rng, C, T), O.F32, i))
        else:
            items.append((synth.ci8_block(rng, C, T), O.CI8, i))
    return items


def upload(items):
    import torch
    from paper_1701_08197_amd import Block
    blocks, outs = [], []
    for x, dt, sid in items:
        d = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        f = torch.full((x.shape[0], x.shape[1]), 9, dtype=torch.uint8, device="cuda")
        blocks.append(Block(d, f, dt, sid))
        outs.append(f)
    return blocks, outs


def flagger(**kw):
    import paper_1701_08197_amd as P
    base = dict(max_streams=64, max_channels=256, max_blocks_per_call=64, max_samples_per_call=1 << 25)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


def snapshot(outs):
    import torch
    torch.cuda.synchronize()
    return [o.cpu().numpy().copy() for o in outs]


def all_tunings():
    import paper_1701_08197_amd as P
    out = []
    for lanes in (32, 48, 64):
        for pers in (0, 1):
            t = P.LofTuning()
            for k in range(2):
                for b in range(5):
                    allowed = [32, 48, 64] if b < 2 else ([48, 64] if b == 2 else [64])
                    t.time_lanes[k][b] = lanes if lanes in allowed else 64
            t.persistent = pers
            t.fuse_post = (lanes + pers) % 3      # the fused SIR/history pass: auto, always, never
            out.append(t)
    return out


def test_tuning_does_not_change_results():
    say("[tuning_does_not_change_results]")
    items = uneven_items(1, 20)
    blocks, outs = upload(items)
    ref = None
    for t in all_tunings():
        fl = flagger()
        fl.set_tuning(t)
        for o in outs:
            o.fill_(9)
        fl.flag_blocks(blocks)
        got = snapshot(outs)
        if ref is None:
            ref = got
            prm = oracle_params(fl.params)
            for (x, dt, _), g in zip(items, got):
                if dt == O.CI8:
                    r = O.flag_block(x, dt, prm, history=O.History(prm), stream_id=0)
                    assert mismatch(g, r.flags) == 0
        else:
            for a, b in zip(ref, got):
                assert (a == b).all(), (list(t.time_lanes[0]), t.persistent)
        fl.close()


def test_graph_replays_equal_eager():
    say("[graph_replays_equal_eager]")
    import torch
    import paper_1701_08197_amd as P
    items = uneven_items(2, 12)
    blocks, outs = upload(items)
    eager = flagger(history_len=4, history_min=2)
    graph = flagger(history_len=4, history_min=2, options=P.LOF_OPT_GRAPH)
    for rep in range(4):
        for o in outs:
            o.fill_(9)
        eager.flag_blocks(blocks)
        eager.history_update()
        e = snapshot(outs)
        # some unrelated eager device work and a sync between replays
        (torch.randn(1 << 20, device="cuda") * 2).sum().item()
        for o in outs:
            o.fill_(9)
        graph.flag_blocks(blocks)
        graph.history_update()
        g = snapshot(outs)
        for a, b in zip(e, g):
            assert (a == b).all(), rep
        he, hg = eager.history_export(), graph.history_export()
        assert (he["counts"] == hg["counts"]).all()
        assert (he["values"] == hg["values"]).all()
    # a changed table rebuilds the graph: its flags are checked before the eager
    # call runs, and blocks outside the new table are left alone
    blocks2 = blocks[:5]
    for o in outs:
        o.fill_(9)
    graph.flag_blocks(blocks2)
    g2 = snapshot(outs)
    assert all((g2[i] == 9).all() for i in range(5, 12))
    for o in outs:
        o.fill_(9)
    eager.flag_blocks(blocks2)
    e2 = snapshot(outs)
    for i in range(5):
        assert (g2[i] == e2[i]).all(), i
    eager.close()
    graph.close()


def test_autotune_keeps_results():
    say("[autotune_keeps_results]")
    items = uneven_items(3, 16)
    blocks, outs = upload(items)
    fl = flagger()
    fl.flag_blocks(blocks)
    before = snapshot(outs)
    staged = fl.history_export()
    t = fl.autotune(blocks, reps=2)
    after_tune = fl.history_export()
    assert (staged["staged"] == after_tune["staged"]).all()          # tuning runs stage no history
    assert (staged["staged_valid"] == after_tune["staged_valid"]).all()
    for k in range(2):
        for b in range(5):
            assert t.time_lanes[k][b] in (32, 48, 64)
    assert t.persistent in (0, 1)
    for o in outs:
        o.fill_(9)
    fl.flag_blocks(blocks)
    after = snapshot(outs)
    for a, b in zip(before, after):
        assert (a == b).all()
    fl.close()
