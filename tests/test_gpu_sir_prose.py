"""GPU: the prose reading of the SIR step (LOF_OPT_SIR_PROSE, Sec. 2.2: every
range of L consecutive flagged samples gains floor(eta L) samples on each side),
through the C ABI, against the CPU reference: exact on complex int8 input, with
history, for several eta, and within the float criterion on float input."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import mismatch, oracle_params, run_gpu, say

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 300), (3, 7), (64, 3072), (16, 768), (7, 1000), (2, 5000), (70, 300), (130, 200),
          (256, 64), (33, 129), (1, 9001)]


def make(**kw):
    import paper_1701_08197_amd as P
    base = dict(max_streams=8, max_channels=256, max_blocks_per_call=16, max_samples_per_call=1 << 22,
                options=P.LOF_OPT_SIR_PROSE)
    base.update(kw)
    return P.Flagger(P.default_params(**base))


@pytest.mark.parametrize("num,den", [(1, 5), (1, 2), (3, 7), (1, 1)])
def test_prose_ci8_exact(num, den):
    say(f"[prose_ci8_exact] eta={num}/{den}")
    fl = make(sir_eta_num=num, sir_eta_den=den)
    prm = oracle_params(fl.params)
    assert prm.sir_prose
    rng = np.random.default_rng(900 + num * 10 + den)
    items = [(synth.ci8_block(rng, C, T), O.CI8, -1) for C, T in SHAPES]
    flags, st = run_gpu(fl, items)
    for (x, _, _), f, s in zip(items, flags, st):
        r = O.flag_block(x, O.CI8, prm)
        assert mismatch(f, r.flags) == 0, x.shape
        assert s["n_flagged"] == int(r.flags.sum())
    fl.close()


def test_prose_with_history_exact():
    say("[prose_with_history_exact]")
    fl = make(history_len=5, history_min=2, history_sensitivity=2.0)
    prm = oracle_params(fl.params)
    h = O.History(prm)
    rng = np.random.default_rng(4321)
    for step in range(5):
        items = [(synth.ci8_block(rng, 32, 1024, rfi=(step % 2 == 0)), O.CI8, k) for k in range(3)]
        flags, st = run_gpu(fl, items)
        for k, ((x, _, _), f) in enumerate(zip(items, flags)):
            r = O.flag_block(x, O.CI8, prm, history=h, stream_id=k)
            assert mismatch(f, r.flags) == 0, (step, k)
            assert st[k]["history_flagged_rows"] == int(r.history_rows.sum())
        fl.history_update(None)
        h.commit()
    fl.close()


@pytest.mark.parametrize("dt,C,T", [(O.F32, 64, 4096), (O.C64, 16, 768), (O.C64_AMP, 256, 1024)])
def test_prose_float(dt, C, T):
    say(f"[prose_float] dtype={dt} C={C} T={T}")
    fl = make()
    rng = np.random.default_rng(77 + C)
    x = synth.f32_power_block(rng, C, T) if dt == O.F32 else synth.c64_block(rng, C, T)
    flags, _ = run_gpu(fl, [(x, dt, -1)])
    r = O.flag_block(x, dt, oracle_params(fl.params))
    rate = mismatch(flags[0], r.flags) / x[..., 0].size if dt == O.CI8 else mismatch(flags[0], r.flags) / (C * T)
    say(f"    mismatch rate {rate:.3g}")
    assert rate <= 1e-3
    fl.close()
