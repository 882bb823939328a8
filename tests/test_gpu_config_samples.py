"""GPU: full-size float workloads sampled from one batched call.  Uneven float32
blocks (C in {16, 64, 256}, T in [768, 12288], gain drift + RFI) flagged together
in one lof_flag_blocks call, with the largest blocks (256 channels, T >= 12000)
among them; beam-formed Stokes I (16 x 768) and visibility amplitudes
(256 x 1024).  Each block against the CPU reference: flag mismatch rate within
the float bound (1e-3 per block), and the largest block by the level-local
replay (every disagreement inside the 1e-6 band of its level's threshold)."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import level_local_replay, mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu


def sample_uneven(n_random=14, n_largest=2, seed=8):
    shapes = synth.config2_shapes()
    largest = sorted(range(len(shapes)), key=lambda b: -(shapes[b][0] * shapes[b][1]))[:n_largest]
    rng = np.random.default_rng(seed)
    rest = [b for b in rng.choice(len(shapes), size=n_random + n_largest, replace=False).tolist()
            if b not in largest][:n_random]
    return shapes, largest + sorted(rest)


def flag_and_compare(fl, items, label):
    flags, st = run_gpu(fl, items)
    prm = oracle_params(fl.params)
    bad = tot = 0
    for (x, dt, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, dt, prm)
        mm = mismatch(f, r.flags)
        assert mm / f.size <= 1e-3, (label, x.shape, mm)
        assert s["median"] == pytest.approx(r.median, rel=2e-7)
        assert s["stddev"] == pytest.approx(r.stddev, rel=1e-6)
        bad += mm
        tot += f.size
    say(f"    {label}: {len(items)} blocks, mismatch {bad} / {tot} = {bad / tot:.3g}")
    return bad, tot


def test_uneven_float_blocks_one_call():
    import paper_1701_08197_amd as P
    shapes, sample = sample_uneven()
    say(f"[uneven_float_blocks_one_call] blocks {sample}")
    assert any(shapes[b][0] == 256 and shapes[b][1] >= 12000 for b in sample)
    items = [(synth.config2_block(b, shapes), O.F32, -1) for b in sample]
    n = sum(x.shape[0] * x.shape[1] for x, _, _ in items)
    fl = P.Flagger(P.default_params(max_streams=1, max_channels=256, max_blocks_per_call=len(items),
                                    max_samples_per_call=n))
    flag_and_compare(fl, items, "uneven float32")
    fl.close()


def test_largest_uneven_block_level_local_replay():
    shapes, sample = sample_uneven()
    b = sample[0]
    say(f"[largest_uneven_block_level_local_replay] block {b} shape {shapes[b]}")
    x = synth.config2_block(b, shapes)
    nd = level_local_replay(x, O.F32, f"uneven block {b}")
    say(f"    level-local disagreements {nd}")


def test_stokes_and_visibility_blocks_one_call():
    import paper_1701_08197_amd as P
    say("[stokes_and_visibility_blocks_one_call]")
    items = [(synth.config3a_block(b), O.F32, -1) for b in (0, 1, 977, 61975)]
    items += [(synth.config3b_block(b), O.C64_AMP, -1) for b in (0, 4511)]
    fl = P.Flagger(P.default_params(max_streams=1, max_channels=256, max_blocks_per_call=len(items),
                                    max_samples_per_call=1 << 20))
    flag_and_compare(fl, items, "stokes + visibility amplitude")
    fl.close()
