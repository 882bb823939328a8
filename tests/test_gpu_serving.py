"""GPU: the continuous-batching service.  Each station's flags are the same
whether its seconds are flagged alone (one call per second, nothing else in
flight) or mixed with other stations' requests in shared, overlapping batches;
integer input, so 'the same' means bit for bit, history included."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

SUBBANDS = [3, 5, 2, 4, 6, 1]
SECONDS = 4
C, T = 64, 3072


def block(st, sec, sb):
    return synth.config4_block(st, sec, sb)


def test_alone_equals_mixed():
    say("[alone_equals_mixed] generating")
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd.serve import Service
    dev = {}
    for st, nsb in enumerate(SUBBANDS):
        for sec in range(SECONDS):
            for sb in range(nsb):
                dev[(st, sec, sb)] = torch.from_numpy(block(st, sec, sb)).cuda()
    rng = np.random.default_rng(5)
    arrivals = []
    for st in range(len(SUBBANDS)):
        t = 0.0
        for sec in range(SECONDS):
            t += rng.exponential(1.0)
            arrivals.append((t, st, sec))
    arrivals.sort()
    hp = dict(history_len=4, history_min=2, history_sensitivity=3.0)
    say("[alone_equals_mixed] serving")
    svc = Service(len(SUBBANDS), 8, n_slots=9, C=C, T=T, keep_outputs=True, **hp)
    done = svc.run(arrivals, lambda st, sec: [dev[(st, sec, sb)] for sb in range(SUBBANDS[st])],
                   speedup=200.0)
    assert len(done) == len(arrivals)
    mixed = svc.outputs
    svc.close()
    say("[alone_equals_mixed] alone")
    for st, nsb in enumerate(SUBBANDS):
        fl = P.Flagger(P.default_params(max_streams=8, max_channels=C, max_blocks_per_call=8,
                                        max_samples_per_call=8 * C * T, options=P.LOF_OPT_AUTOCOMMIT, **hp))
        h = O.History(O.Params(history_len=4, history_min=2, history_sensitivity=3.0))
        for sec in range(SECONDS):
            outs = [torch.zeros((C, T), dtype=torch.uint8, device="cuda") for _ in range(nsb)]
            fl.flag_blocks([P.Block(dev[(st, sec, sb)], outs[sb], P.LOF_CI8, sb) for sb in range(nsb)])
            torch.cuda.synchronize()
            for sb in range(nsb):
                alone = outs[sb].cpu().numpy()
                assert (alone == mixed[(st, sec, sb)]).all(), (st, sec, sb)
            if st == 1:   # and against the reference, history included
                for sb in range(nsb):
                    r = O.flag_block(block(st, sec, sb), O.CI8, h.params, history=h, stream_id=sb)
                    assert (r.flags == mixed[(st, sec, sb)].astype(bool)).all(), (st, sec, sb)
                h.commit()
        fl.close()


def test_station_order_kept_when_subband_counts_change():
    """A station whose subband count changes between seconds, with an arena
    that is nearly full: its seconds are admitted in arrival order (a smaller
    later second never overtakes a deferred earlier one), and every station's
    flags equal a sequential run, history included."""
    say("[station_order_kept_when_subband_counts_change]")
    import torch
    import paper_1701_08197_amd as P
    from paper_1701_08197_amd.serve import Request, Service
    counts = {0: [6, 1, 5, 1, 6], 1: [2, 2, 2, 2, 2], 2: [1, 6, 1, 6, 1]}
    dev = {(st, sec, sb): torch.from_numpy(block(st, sec, sb)).cuda()
           for st, per in counts.items() for sec, n in enumerate(per) for sb in range(n)}
    arrivals = sorted((0.01 * sec + 0.001 * st, st, sec) for st, per in counts.items() for sec in range(len(per)))
    hp = dict(history_len=4, history_min=2, history_sensitivity=3.0)
    svc = Service(len(counts), 8, n_slots=7, C=C, T=T, keep_outputs=True, **hp)
    with pytest.raises(ValueError):
        svc.submit(Request(0, 99, 0.0, [dev[(0, 0, 0)]] * 8))
    done = svc.run(arrivals, lambda st, sec: [dev[(st, sec, sb)] for sb in range(counts[st][sec])], speedup=1e4)
    assert len(done) == len(arrivals) and svc.shed == 0
    for st in counts:
        seq = [r.admit_seq for r in sorted((r for r in done if r.station == st), key=lambda r: r.second)]
        assert seq == sorted(seq), (st, seq)
    mixed = svc.outputs
    svc.close()
    for st, per in counts.items():
        fl = P.Flagger(P.default_params(max_streams=8, max_channels=C, max_blocks_per_call=8,
                                        max_samples_per_call=8 * C * T, options=P.LOF_OPT_AUTOCOMMIT, **hp))
        for sec, n in enumerate(per):
            outs = [torch.zeros((C, T), dtype=torch.uint8, device="cuda") for _ in range(n)]
            fl.flag_blocks([P.Block(dev[(st, sec, sb)], outs[sb], P.LOF_CI8, sb) for sb in range(n)])
            torch.cuda.synchronize()
            for sb in range(n):
                assert (outs[sb].cpu().numpy() == mixed[(st, sec, sb)]).all(), (st, sec, sb)
        fl.close()
