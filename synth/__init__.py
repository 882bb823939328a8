"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws input data (noise, injected interference, a weak dispersed
pulse, bandpass drift) and returns raw sample arrays in the layouts the flagger
takes.  It holds none of the flagging method's arithmetic; both the HIP library's
tests/benchmarks and the CPU reference are fed from here.

Every block is generated from ``numpy.random.SeedSequence([1701, 8197, cfg, index])``
so any block of any workload can be regenerated on its own.

Workloads (shapes follow the paper: 16-channel beams at 12 kHz / 82 us for the
pulsar observation, stations x polarisations x subbands x channels x times for the
pre-correlation flagger; Sec. 4 complexity, Sec. 5.1):

* cfg 0: one complex64 block, 64 channels x 4096 times, unit complex noise + RFI mix.
* cfg 1: 48 stations x 2 pols x 64 subbands, each 64 x 3072 complex int8
  (sigma 16 per component, clipped to +-127) + RFI mix + a weak dispersed pulse.
* cfg 2: 4096 float32 power blocks, C in {16, 64, 256}, T in [768, 12288],
  with 1/f bandpass gain drift (0.5x .. 2x) and the RFI mix.
* cfg 3a: 127 beams x 488 subbands of 16 x 768 float32 Stokes I (chi^2, 4 dof, mean 1).
* cfg 3b: 1128 baselines x 4 correlations of 256 x 1024 complex64 visibilities.
* cfg 4: streaming: 48 stations with 16..64 subbands each of 64 x 3072 complex int8.
"""
from __future__ import annotations

import numpy as np

CI8, C64, F32, C64_AMP = 0, 1, 2, 3
SEED_ROOT = (1701, 8197)

# RFI mix in units of the noise power's standard deviation (for complex Gaussian
# noise that equals the mean noise power).
RFI_TONE_K = 8.0
RFI_IMPULSE_K = 10.0
RFI_BURST_K = 3.0

CFG1_STATIONS, CFG1_POLS, CFG1_SUBBANDS = 48, 2, 64
CFG1_C, CFG1_T = 64, 3072
CFG1_SIGMA = 16.0


def rng_for(cfg: int, index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT[0], SEED_ROOT[1], cfg, index]))


# ---------------------------------------------------------------- interference plan
def rfi_plan(rng: np.random.Generator, C: int, T: int):
    """3 narrowband channels for all times, 5 broadband impulses 1..16 samples wide,
    one 32-channel x 256-sample burst, all clipped to the block."""
    plan = []
    tones = rng.choice(C, size=min(3, C), replace=False)
    for ch in tones:
        plan.append(("tone", int(ch), int(ch) + 1, 0, T, RFI_TONE_K, float(rng.uniform(0.01, 0.49))))
    for _ in range(5):
        w = int(rng.integers(1, 17))
        t0 = int(rng.integers(0, max(1, T - w + 1)))
        plan.append(("impulse", 0, C, t0, min(T, t0 + w), RFI_IMPULSE_K, 0.0))
    bc, bt = min(32, C), min(256, T)
    c0 = int(rng.integers(0, C - bc + 1))
    t0 = int(rng.integers(0, T - bt + 1))
    plan.append(("burst", c0, c0 + bc, t0, t0 + bt, RFI_BURST_K, 0.0))
    return plan


def _add_rfi_voltage(rng, re, im, plan, noise_power):
    """Add each interferer as a complex signal of power k * noise_power."""
    T = re.shape[1]
    for kind, c0, c1, t0, t1, k, nu in plan:
        amp = np.float32(np.sqrt(k * noise_power))
        n = t1 - t0
        if kind == "tone":
            ph = (2.0 * np.pi * nu * np.arange(t0, t1) + rng.uniform(0, 2 * np.pi)).astype(np.float32)
            ph = np.broadcast_to(ph, (c1 - c0, n))
        else:
            ph = rng.uniform(0, 2 * np.pi, size=(c1 - c0, n)).astype(np.float32)
        re[c0:c1, t0:t1] += amp * np.cos(ph)
        im[c0:c1, t0:t1] += amp * np.sin(ph)
    return re, im


def _add_rfi_power(power, plan, gain=None):
    for kind, c0, c1, t0, t1, k, _ in plan:
        add = np.float32(k)
        if gain is not None:
            power[c0:c1, t0:t1] += add * gain[c0:c1, t0:t1]
        else:
            power[c0:c1, t0:t1] += add
    return power


# ------------------------------------------------------------------------ cfg 0
def c64_block(rng: np.random.Generator, C: int, T: int, rfi: bool = True) -> np.ndarray:
    """Unit complex Gaussian noise (E|n|^2 = 1) plus the RFI mix, complex64 [C, T]."""
    s = np.float32(np.sqrt(0.5))
    re = rng.standard_normal((C, T), dtype=np.float32) * s
    im = rng.standard_normal((C, T), dtype=np.float32) * s
    if rfi:
        _add_rfi_voltage(rng, re, im, rfi_plan(rng, C, T), 1.0)
    out = np.empty((C, T), dtype=np.complex64)
    out.real = re
    out.imag = im
    return out


def config0():
    return c64_block(rng_for(0, 0), 64, 4096), C64


# ------------------------------------------------------------------------ cfg 1
def _pulse_profile(subband: int, C: int, T: int, n_subbands: int = 64, t_start: float = 0.0):
    """Weak dispersed periodic pulse (DM 30, period 0.714 s, 10 ms wide) over 64
    contiguous 195.3125 kHz subbands centred at 150 MHz, 64 channels each,
    327.68 us samples, for the block starting t_start seconds into the
    observation.  Returns a bool [C, T] on-pulse mask."""
    df_sb = 195.3125e3
    df_ch = df_sb / C
    tsamp = 1.0 / df_ch
    f_lo = 150e6 - (n_subbands / 2) * df_sb
    f_top = f_lo + n_subbands * df_sb
    f = f_lo + subband * df_sb + (np.arange(C) + 0.5) * df_ch
    dm, period, width, t_first = 30.0, 0.714, 10e-3, 0.05
    delay = 4.1488e-3 * dm * ((f / 1e9) ** -2 - (f_top / 1e9) ** -2)
    t = t_start + np.arange(T) * tsamp
    on = np.zeros((C, T), dtype=bool)
    for c in range(C):
        ph = np.mod(t - t_first - delay[c], period)
        on[c] = ph < width
    return on


def ci8_block(rng: np.random.Generator, C: int, T: int, sigma: float = CFG1_SIGMA,
              rfi: bool = True, pulse_subband: int | None = None,
              pulse_k: float = 0.2, pulse_t0: float = 0.0) -> np.ndarray:
    """Complex int8 voltages [C, T, 2] (re, im): Gaussian with per-component sigma,
    the RFI mix and an optional weak pulse added before rounding half-to-even and
    clipping to +-127."""
    re = rng.standard_normal((C, T), dtype=np.float32) * np.float32(sigma)
    im = rng.standard_normal((C, T), dtype=np.float32) * np.float32(sigma)
    noise_power = 2.0 * sigma * sigma
    if rfi:
        _add_rfi_voltage(rng, re, im, rfi_plan(rng, C, T), noise_power)
    if pulse_subband is not None:
        on = _pulse_profile(pulse_subband, C, T, t_start=pulse_t0)
        amp = np.float32(np.sqrt(pulse_k * noise_power))
        ph = rng.uniform(0, 2 * np.pi, size=int(on.sum())).astype(np.float32)
        re[on] += amp * np.cos(ph)
        im[on] += amp * np.sin(ph)
    out = np.empty((C, T, 2), dtype=np.int8)
    out[..., 0] = np.clip(np.rint(re), -127, 127)
    out[..., 1] = np.clip(np.rint(im), -127, 127)
    return out


def plan_mask(plan, C: int, T: int) -> dict:
    """Boolean [C, T] masks of where each kind of interferer of an RFI plan was
    injected (ground truth for quality reports)."""
    out = {k: np.zeros((C, T), dtype=bool) for k in ("tone", "impulse", "burst")}
    for kind, c0, c1, t0, t1, _, _ in plan:
        out[kind][c0:c1, t0:t1] = True
    return out


def config1_truth(b: int, second: int = 0):
    """(block, interferer masks, pulse mask) of config1_block(b, second): the same
    draws, with the plan kept."""
    subband = b % CFG1_SUBBANDS
    idx = b if second == 0 else second * CFG1_STATIONS * CFG1_POLS * CFG1_SUBBANDS + b
    rng = rng_for(1, idx)
    C, T, sigma = CFG1_C, CFG1_T, CFG1_SIGMA
    re = rng.standard_normal((C, T), dtype=np.float32) * np.float32(sigma)
    im = rng.standard_normal((C, T), dtype=np.float32) * np.float32(sigma)
    plan = rfi_plan(rng, C, T)
    x = config1_block(b, second)
    return x, plan_mask(plan, C, T), _pulse_profile(subband, C, T, t_start=second * CFG1_SECOND_S)


def config1_index(station: int, pol: int, subband: int) -> int:
    return (station * CFG1_POLS + pol) * CFG1_SUBBANDS + subband


CFG1_SECOND_S = CFG1_T * CFG1_C / 195.3125e3   # 3072 samples of 327.68 us


def config1_block(b: int, second: int = 0) -> np.ndarray:
    """Block b = (station * 2 + pol) * 64 + subband of second `second` of the
    48-station observation (each second has its own noise, RFI and pulse phase)."""
    subband = b % CFG1_SUBBANDS
    idx = b if second == 0 else second * CFG1_STATIONS * CFG1_POLS * CFG1_SUBBANDS + b
    return ci8_block(rng_for(1, idx), CFG1_C, CFG1_T, pulse_subband=subband,
                     pulse_t0=second * CFG1_SECOND_S)


CONFIG1_BLOCKS = CFG1_STATIONS * CFG1_POLS * CFG1_SUBBANDS   # 6144


# ------------------------------------------------------------------------ cfg 2
def config2_shapes(n_blocks: int = 4096):
    rng = rng_for(2, 1 << 30)
    Cs = rng.choice(np.array([16, 64, 256]), size=n_blocks)
    Ts = rng.integers(768, 12288 + 1, size=n_blocks)
    return [(int(c), int(t)) for c, t in zip(Cs, Ts)]


def _one_over_f(rng, C, T):
    """Per-channel 1/f process normalised to [-1, 1]."""
    nf = T // 2 + 1
    freqs = np.arange(nf, dtype=np.float64)
    freqs[0] = 1.0
    spec = (rng.standard_normal((C, nf)) + 1j * rng.standard_normal((C, nf))) / np.sqrt(freqs)
    spec[:, 0] = 0.0
    u = np.fft.irfft(spec, n=T, axis=1)
    lo = u.min(axis=1, keepdims=True)
    hi = u.max(axis=1, keepdims=True)
    return (2.0 * (u - lo) / np.maximum(hi - lo, 1e-30) - 1.0).astype(np.float32)


def f32_power_block(rng: np.random.Generator, C: int, T: int, drift: bool = True) -> np.ndarray:
    """Float32 power of unit complex noise (exponential, mean 1) times a drifting
    per-channel gain 2^u, u a 1/f process in [-1, 1], plus the RFI mix."""
    pw = rng.exponential(1.0, size=(C, T)).astype(np.float32)
    gain = np.exp2(_one_over_f(rng, C, T)) if drift else None
    if gain is not None:
        pw *= gain
    _add_rfi_power(pw, rfi_plan(rng, C, T), gain)
    return pw


def config2_block(b: int, shapes=None) -> np.ndarray:
    shapes = shapes or config2_shapes()
    C, T = shapes[b]
    return f32_power_block(rng_for(2, b), C, T)


# ------------------------------------------------------------------------ cfg 3
CFG3A_BLOCKS = 127 * 488
CFG3B_BLOCKS = 1128 * 4


def config3a_block(b: int) -> np.ndarray:
    """Stokes I of two unit complex polarisations: chi^2 with 4 dof, mean 1, + RFI."""
    rng = rng_for(3, b)
    si = rng.gamma(2.0, 0.5, size=(16, 768)).astype(np.float32)
    _add_rfi_power(si, rfi_plan(rng, 16, 768))
    return si


def config3b_block(b: int) -> np.ndarray:
    """Complex64 visibilities, unit complex noise + RFI mix, 256 x 1024."""
    return c64_block(rng_for(33, b), 256, 1024)


# ------------------------------------------------------------------------ cfg 4
CFG4_STATIONS = 48


def config4_subbands():
    rng = rng_for(4, 1 << 30)
    return [int(s) for s in rng.integers(16, 65, size=CFG4_STATIONS)]


def config4_block(station: int, second: int, subband: int) -> np.ndarray:
    idx = (second * CFG4_STATIONS + station) * 64 + subband
    return ci8_block(rng_for(4, idx), CFG1_C, CFG1_T, pulse_subband=subband)


def config4_arrivals(seconds: float, rate: float = 1.0, seed_index: int = 0):
    """Poisson arrival times (mean interval 1/rate seconds) per station."""
    rng = rng_for(4, (1 << 29) + seed_index)
    out = []
    for s in range(CFG4_STATIONS):
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t > seconds:
                break
            out.append((t, s, k))
            k += 1
    out.sort()
    return out
