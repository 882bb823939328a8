"""Float input: level-local replay.  The GPU runs SumThreshold stopped after
each level (time levels, then frequency levels); the CPU reference re-decides
the next level from the GPU's own mask in float64.  Every disagreement must lie
in a window whose unflagged mean is within 1e-6 (relative) of the level's
threshold.  The end-to-end mismatch rate is reported."""
import numpy as np
import pytest

import oracle.lof_oracle as O
import synth
from tests.gpu_util import gpu_mask, level_local_replay, say

pytestmark = pytest.mark.gpu


CASES = [("config0", None), ("f32_drift", (O.F32, 64, 3000)), ("stokes", (O.F32, 16, 768)),
         ("vis_amp", (O.C64_AMP, 256, 1024))]


@pytest.mark.parametrize("name,spec", CASES)
def test_level_local_replay(name, spec):
    say(f"[level_local_replay] {name}")
    if spec is None:
        x, dt = synth.config0()
    elif name == "stokes":
        x, dt = synth.config3a_block(0), O.F32
    elif name == "vis_amp":
        x, dt = synth.config3b_block(0), O.C64_AMP
    else:
        dt, C, T = spec
        x = synth.f32_power_block(np.random.default_rng(5), C, T)
    total_diff = level_local_replay(x, dt, name)
    full, _ = gpu_mask(x, dt)
    ref = O.flag_block(x, dt, O.Params(sir_eta_num=0))
    rate = float((full != ref.flags).mean())
    say(f"    {name}: level-local disagreements {total_diff}, end-to-end mismatch rate {rate:.3g}")
    assert rate < 1e-3
