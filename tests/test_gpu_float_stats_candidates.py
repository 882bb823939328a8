"""GPU: the one-workgroup float statistics (Sec. 2.1 median and stddev, Sec. 4.2
MAD) keep the keys of the median's first-digit bins from the second radix pass
in a candidate list and run the third pass over it; when the list would exceed
its capacity (about N / 8: a constant or few-valued block) the third pass reads
the block again.  Both ways against the oracle on float32 input, where the
median is exact, the stddev within 1e-9 (the MAD within 1e-6, an order
statistic of float32 deviations), the flags within the float criterion; calls of
more than 16 float blocks, so no block takes the split statistics."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("opts", [0, 0x40])
def test_candidate_list_and_overflow(opts):
    import paper_1701_08197_amd as P
    say(f"[candidate_list_and_overflow] options={opts}")
    fl = P.Flagger(P.default_params(max_streams=4, max_channels=256, max_blocks_per_call=32,
                                    max_samples_per_call=1 << 23, options=opts))
    prm = oracle_params(fl.params)
    rng = np.random.default_rng(9300 + opts)
    const = np.full((64, 4096), 3.0, dtype=np.float32)
    const[7, 50:90] = 80.0
    two = rng.integers(1, 3, size=(32, 4096)).astype(np.float32)
    few = rng.choice(np.array([0.5, 1.0, 1.5, 2.0, 8.0], dtype=np.float32), size=(16, 5000))
    items = [(const, O.F32, -1), (two, O.F32, -1), (few, O.F32, -1)]
    items += [(synth.f32_power_block(rng, C, T), O.F32, -1)
              for C, T in [(64, 4096), (256, 1024), (16, 768), (7, 9001), (3, 5)] * 3]
    flags, st = run_gpu(fl, items)
    rel = 1e-6 if opts else 1e-9
    bad = tot = 0
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.F32, prm)
        assert s["median"] == r.median, x.shape
        assert s["stddev"] == pytest.approx(r.stddev, rel=rel, abs=1e-300), x.shape
        for a, b in zip(s["threshold"][:7], r.thresholds[:7]):
            assert a == pytest.approx(b, rel=rel, abs=1e-300)
        bad += mismatch(f, r.flags)
        tot += f.size
    say(f"    mismatch {bad} of {tot}")
    assert bad / tot <= 1e-3
    fl.close()
