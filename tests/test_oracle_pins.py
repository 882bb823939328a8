"""Pins of the CPU reference against what the paper and mathematics fix.

Each test ties a reference function to something other than itself: values the
paper prints (tests/golden/paper_values.json), closed forms, invariants, library
routines it must reduce to, or an independent brute force on tiny inputs.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle.lof_oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def f32(a):
    return np.asarray(a, dtype=np.float32)


def run(x, dtype=O.F32, **kw):
    return O.flag_block(x, dtype, O.Params(**kw))


# ------------------------------------------------------------------ thresholds
def test_factor_worked_values_from_paper():
    g = golden()
    prm = O.Params(p=g["default_p"]["value"], sensitivity=g["default_sensitivity"]["value"])
    f = O.level_factors(prm, 2)
    # Sec. 2.1: 6 sigma at window 1, 4.5 sigma at window 2.
    assert f[0] * prm.sensitivity == g["first_iteration_sigma"]["value"]
    assert f[1] * prm.sensitivity == g["second_iteration_sigma"]["value"]


def test_factor_closed_form():
    # startThreshold * p^log2(I) / I with p = 1.5 is 6 * 0.75^k exactly in binary.
    f = O.level_factors(O.Params(), 10)
    for k, v in enumerate(f):
        assert v == 6.0 * 0.75 ** k
        assert Fraction(v) == Fraction(6) * Fraction(3, 4) ** k
    assert f[:7] == [6, 4.5, 3.375, 2.53125, 1.8984375, 1.423828125, 1.06787109375]


def test_threshold_is_median_plus_scaled_sigma():
    T = O.thresholds(3.0, 2.0, O.Params(sensitivity=0.5), 3)
    assert T == [3.0 + 2.0 * 6.0 * 0.5, 3.0 + 2.0 * 4.5 * 0.5, 3.0 + 2.0 * 3.375 * 0.5]


# --------------------------------------------------------------- median, stddev
@pytest.mark.parametrize("n", [1, 2, 3, 10, 11, 1000, 1001])
def test_median_matches_numpy(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, 50, size=n)
    assert O.block_median(a) == float(np.median(a))
    b = rng.standard_normal(n).astype(np.float64)
    assert O.block_median(b) == float(np.median(b))


@pytest.mark.parametrize("n", [1, 7, 64, 4096])
def test_stddev_matches_numpy_and_exact(n):
    rng = np.random.default_rng(100 + n)
    a = rng.integers(0, 32769, size=n).astype(np.int64)
    sd = O.block_stddev(a, exact=True)
    s1, s2 = sum(int(v) for v in a), sum(int(v) * int(v) for v in a)
    var_exact = Fraction(s2, n) - Fraction(s1, n) ** 2
    ref = math.sqrt(float(var_exact))
    assert sd == pytest.approx(ref, rel=1e-14, abs=1e-300)
    assert sd == pytest.approx(float(np.std(a.astype(np.float64))), rel=1e-12, abs=1e-300)
    b = rng.exponential(1.0, size=n)
    assert O.block_stddev(b, exact=False) == pytest.approx(float(np.std(b)), rel=1e-12, abs=1e-300)


def test_power_definitions():
    x = np.array([[[3, 4], [-128, -128], [0, 0]]], dtype=np.int8)
    assert O.power(x, O.CI8).tolist() == [[25, 32768, 0]]
    z = np.array([[3 + 4j, 1 - 1j]], dtype=np.complex64)
    assert O.power(z, O.C64).tolist() == [[25.0, 2.0]]
    assert O.power(z, O.C64_AMP).tolist() == [[5.0, math.sqrt(2.0)]]


# ------------------------------------------------------------- SumThreshold pins
@pytest.mark.parametrize("dtype", [O.F32, O.CI8])
def test_constant_input_gives_no_flags(dtype):
    if dtype == O.F32:
        x = np.full((8, 300), 7.25, dtype=np.float32)
    else:
        x = np.zeros((8, 300, 2), dtype=np.int8)
        x[..., 0] = 5
        x[..., 1] = -3
    r = O.flag_block(x, dtype, O.Params())
    assert r.stddev == 0.0
    assert not r.flags.any()


@pytest.mark.parametrize("N", list(range(28, 44)) + [64, 100])
def test_single_impulse_flagged_iff_N_at_least_35(N):
    # Zero background, one impulse: sigma = A sqrt(N-1)/N, so A > 6 sigma iff N >= 35.
    for A in (1.0, 37.5):
        x = np.zeros((1, N), dtype=np.float32)
        x[0, N // 3] = A
        r = run(x)
        expect = np.zeros((1, N), dtype=bool)
        if N >= 35:
            expect[0, N // 3] = True
        assert (r.flags == expect).all(), (N, A)


def test_single_impulse_exact_path():
    for N in (34, 35):
        x = np.zeros((1, N, 2), dtype=np.int8)
        x[0, 5, 0] = 100
        r = O.flag_block(x, O.CI8, O.Params())
        assert r.flags[0, 5] == (N >= 35)
        assert r.flags.sum() == (1 if N >= 35 else 0)


def _box_closed_form(N, w, A=1.0, prm=O.Params()):
    """Independent derivation for a 1-D box on a zero background: the first level
    k* with a window whose mean exceeds T_k flags the union of all such windows
    of that level (windows are judged on the unflagged data)."""
    b0 = (N - w) // 2
    frac = w / N
    sigma = A * math.sqrt(frac * (1 - frac))
    med = 0.0
    for k in range(prm.n_levels):
        I = 1 << k
        T = med + sigma * prm.start_threshold * 0.75 ** k
        flagged = np.zeros(N, dtype=bool)
        for s in range(N - I + 1):
            ov = max(0, min(s + I, b0 + w) - max(s, b0))
            if A * ov > I * T:
                flagged[s:s + I] = True
        if flagged.any():
            return k, flagged
    return None, np.zeros(N, dtype=bool)


# (width, first level k*, extra samples flagged on each side) worked on paper.
BOX_TABLE = [(1, 0, 0), (8, 0, 0), (29, 0, 0), (30, 1, 0), (53, 1, 0), (54, 2, 0),
             (100, 3, 1), (200, 4, 3), (300, 4, 2)]


@pytest.mark.parametrize("w,kstar,ext", BOX_TABLE)
def test_box_closed_form(w, kstar, ext):
    N = 1024
    x = np.zeros((1, N), dtype=np.float32)
    b0 = (N - w) // 2
    x[0, b0:b0 + w] = 1.0
    r = run(x, sir_eta_num=0)
    k, cf = _box_closed_form(N, w)
    assert k == kstar
    expect = np.zeros(N, dtype=bool)
    expect[max(0, b0 - ext):b0 + w + ext] = True
    assert (cf == expect).all()
    assert (r.flags[0] == expect).all()
    # same on the exact integer path (re = 1 -> power 1)
    xi = np.zeros((1, N, 2), dtype=np.int8)
    xi[0, b0:b0 + w, 0] = 1
    ri = O.flag_block(xi, O.CI8, O.Params(sir_eta_num=0))
    assert (ri.flags[0] == expect).all()


def test_box_2d_detected_per_row():
    # A w x h box detected by the time pass: each row behaves as the 1-D box.
    C, N, w, h = 16, 512, 100, 4
    x = np.zeros((C, N), dtype=np.float32)
    x[5:5 + h, 200:200 + w] = 1.0
    r = run(x, sir_eta_num=0)
    frac = (w * h) / (C * N)
    sigma = math.sqrt(frac * (1 - frac))
    rowflag = np.zeros(N, dtype=bool)
    for k in range(7):
        I = 1 << k
        T = sigma * 6 * 0.75 ** k
        for s in range(N - I + 1):
            ov = max(0, min(s + I, 300) - max(s, 200))
            if ov > I * T:
                rowflag[s:s + I] = True
        if rowflag.any():
            break
    for c in range(C):
        if 5 <= c < 5 + h:
            assert (r.st_mask[c] == rowflag).all()
        else:
            assert not r.st_mask[c].any()


def test_n_levels_one_is_plain_thresholder():
    rng = np.random.default_rng(5)
    x = rng.exponential(1.0, size=(16, 700)).astype(np.float32)
    x[3, 100] = 40.0
    r = run(x, n_levels=1, sir_eta_num=0)
    p = x.astype(np.float64)
    T0 = O.block_median(p) + 6.0 * O.block_stddev(p, False)
    assert (r.flags == (p > T0)).all()


def test_flags_only_accumulate_over_levels():
    rng = np.random.default_rng(6)
    p = rng.exponential(1.0, size=(12, 600))
    p[:, 300:340] += 2.0
    med, sd = O.block_median(p), O.block_stddev(p, False)
    T = O.thresholds(med, sd, O.Params())
    prev = np.zeros(p.shape, dtype=bool)
    for n in range(1, 8):
        m = O.sumthreshold_rows(p, np.zeros(p.shape, dtype=bool), T, n, False)
        assert (m >= prev).all()
        prev = m


@pytest.mark.parametrize("seed", range(6))
def test_time_and_frequency_reversal_symmetry(seed):
    rng = np.random.default_rng(seed)
    x = rng.exponential(1.0, size=(24, 400)).astype(np.float32)
    x[rng.integers(0, 24), :] += 5.0
    x[:, rng.integers(0, 380):][:, :10] += 8.0
    x[4:12, 50:90] += 1.5
    r = run(x)
    rt = run(x[:, ::-1].copy())
    rf = run(x[::-1, :].copy())
    assert (rt.flags == r.flags[:, ::-1]).all()
    assert (rf.flags == r.flags[::-1, :]).all()


def test_power_of_two_scaling_invariance():
    rng = np.random.default_rng(9)
    x = rng.exponential(1.0, size=(32, 512)).astype(np.float32)
    x[7, :] += 6.0
    x[:, 100:104] += 9.0
    r1 = run(x)
    for s in (0.25, 4.0, 1024.0):
        r2 = run((x * np.float32(s)).astype(np.float32))
        assert (r1.flags == r2.flags).all()


def test_pure_noise_level0_rate():
    # Exponential power (unit complex noise): P(p > ln2 + 6) = e^{-6}/2 = 1.239e-3.
    rng = np.random.default_rng(11)
    p = rng.exponential(1.0, size=(64, 16384))
    med, sd = O.block_median(p), O.block_stddev(p, False)
    T = O.thresholds(med, sd, O.Params(), 1)
    m = O.sumthreshold_rows(p, np.zeros(p.shape, dtype=bool), T, 1, False)
    rate = m.mean()
    expect = 0.5 * math.exp(-6.0)
    n = p.size
    assert abs(rate - expect) < 5 * math.sqrt(expect / n) + 2e-4


def test_frequency_level_one_is_noop_after_time():
    rng = np.random.default_rng(12)
    p = rng.exponential(1.0, size=(20, 300))
    p[3, 7] = 30
    T = O.thresholds(O.block_median(p), O.block_stddev(p, False), O.Params())
    m = O.sumthreshold_rows(p, np.zeros(p.shape, dtype=bool), T, 7, False)
    m1 = O.sumthreshold_rows(p.T, m.T, T, 1, False).T
    assert (m1 == m).all()


def _st_bruteforce_fraction(p_rows, T, n_levels):
    """Pure-Python per-window SumThreshold with exact rationals (independent loops)."""
    out = []
    for row in p_rows:
        n = len(row)
        m = [False] * n
        for k in range(n_levels):
            I = 1 << k
            if I > n:
                break
            nm = list(m)
            for s in range(n - I + 1):
                vals = [row[j] for j in range(s, s + I) if not m[j]]
                if vals and Fraction(sum(vals)) > len(vals) * Fraction(T[k]):
                    for j in range(s, s + I):
                        nm[j] = True
            m = nm
        out.append(m)
    return np.array(out, dtype=bool)


@pytest.mark.parametrize("seed", range(40))
def test_tiny_exhaustive_vs_rational_bruteforce(seed):
    rng = np.random.default_rng(1000 + seed)
    C, T = int(rng.integers(1, 7)), int(rng.integers(1, 9))
    x = rng.integers(-6, 7, size=(C, T, 2)).astype(np.int8)
    if seed % 3 == 0:
        x[rng.integers(0, C), :, 0] = 60
    prm = O.Params(start_threshold=float(rng.choice([0.5, 1.0, 2.0, 6.0])), sir_eta_num=0)
    r = O.flag_block(x, O.CI8, prm)
    p = O.power(x, O.CI8)
    th = r.thresholds
    m = _st_bruteforce_fraction([list(map(int, row)) for row in p], th, prm.n_levels)
    mt = _st_bruteforce_fraction([list(map(int, col)) for col in p.T], th, prm.n_levels)
    # frequency pass starts from the time mask: run it column by column
    cols = []
    for t in range(T):
        col = [int(v) for v in p[:, t]]
        mcol = [bool(v) for v in m[:, t]]
        n = len(col)
        for k in range(prm.n_levels):
            I = 1 << k
            if I > n:
                break
            nm = list(mcol)
            for s in range(n - I + 1):
                vals = [col[j] for j in range(s, s + I) if not mcol[j]]
                if vals and Fraction(sum(vals)) > len(vals) * Fraction(th[k]):
                    for j in range(s, s + I):
                        nm[j] = True
            mcol = nm
        cols.append(mcol)
    expect = np.array(cols, dtype=bool).T
    assert (r.st_mask == expect).all()
    del mt


# ------------------------------------------------------------------------- SIR
@pytest.mark.parametrize("num,den", [(1, 5), (1, 2), (2, 5), (0, 1), (1, 1)])
def test_sir_linear_equals_bruteforce(num, den):
    rng = np.random.default_rng(num * 10 + den)
    for _ in range(150):
        n = int(rng.integers(1, 40))
        m = rng.random(n) < rng.uniform(0.05, 0.7)
        lin = O.sir_rows(m[None, :], num, den)[0]
        bf = O.sir_row_bruteforce(m, num, den)
        assert (lin == bf).all(), (m.astype(int), num, den)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 7, 8, 12, 20, 40, 41])
def test_sir_isolated_run_closed_form(L):
    # eta = 0.2: a run of L grows by floor(eta L / (1 - eta)) = floor(L / 4) per side.
    n = 200
    m = np.zeros(n, dtype=bool)
    m[80:80 + L] = True
    out = O.sir_rows(m[None, :], 1, 5)[0]
    e = L // 4
    expect = np.zeros(n, dtype=bool)
    expect[80 - e:80 + L + e] = True
    assert (out == expect).all()


def test_sir_properties():
    rng = np.random.default_rng(3)
    for _ in range(100):
        n = int(rng.integers(1, 80))
        a = rng.random(n) < 0.3
        b = a | (rng.random(n) < 0.1)
        sa = O.sir_rows(a[None], 1, 5)[0]
        sb = O.sir_rows(b[None], 1, 5)[0]
        assert (sa >= a).all()                       # extensive
        assert (sb >= sa).all()                      # monotone
        assert (O.sir_rows(a[None], 0, 5)[0] == a).all()   # eta = 0: identity


def test_sir_block_is_time_then_frequency():
    rng = np.random.default_rng(4)
    m = rng.random((9, 30)) < 0.25
    got = O.sir_block(m, O.Params())
    rows = np.array([O.sir_row_bruteforce(r, 1, 5) for r in m])
    expect = np.array([O.sir_row_bruteforce(c, 1, 5) for c in rows.T]).T
    assert (got == expect).all()


# The prose reading of Sec. 2.2 (LOF_OPT_SIR_PROSE): every maximal range of
# consecutive flagged samples, of length L, gains floor(eta L) samples before and
# after it.  Pinned by hand-worked rows and by an independent per-position check
# of that sentence.
@pytest.mark.parametrize("L,ext", [(1, 0), (4, 0), (5, 1), (9, 1), (10, 2), (14, 2), (15, 3), (40, 8)])
def test_sir_prose_isolated_run(L, ext):
    n = 120
    m = np.zeros(n, dtype=bool)
    m[50:50 + L] = True
    out = O.sir_prose_rows(m[None, :], 1, 5)[0]
    expect = np.zeros(n, dtype=bool)
    expect[50 - ext:50 + L + ext] = True
    assert (out == expect).all()


def test_sir_prose_hand_worked_rows():
    def row(txt):
        return np.array([c == "1" for c in txt])
    cases = [
        # a run of 10 at the start is clipped on the left, grows 2 on the right
        ("111111111100000000", "111111111111000000"),
        # runs of 10 and 5 three apart: [0, 12) and [12, 19) join
        ("11111111110001111100000", "11111111111111111110000"),
        # short runs (L < 5) do not grow, whatever their neighbours
        ("0011101101110000", "0011101101110000"),
        # a run of 5 at the end grows by 1 on the left only
        ("0000000011111", "0000000111111"),
    ]
    for src, want in cases:
        got = O.sir_prose_rows(row(src)[None, :], 1, 5)[0]
        assert "".join("1" if v else "0" for v in got) == want, src


def _prose_by_definition(m, num, den):
    # y is flagged iff it lies in [s - floor(eta L), e + floor(eta L)) of some
    # maximal flagged range [s, e) of length L = e - s
    n = len(m)
    edges = np.diff(np.concatenate([[0], m.astype(np.int8), [0]]))
    starts = np.flatnonzero(edges == 1)
    ends = np.flatnonzero(edges == -1)
    y = np.arange(n)
    out = np.zeros(n, dtype=bool)
    for s_, e_ in zip(starts, ends):
        ext = (num * (e_ - s_)) // den
        out |= (y >= s_ - ext) & (y < e_ + ext)
    return out


@pytest.mark.parametrize("num,den", [(1, 5), (1, 2), (3, 7), (0, 1), (1, 1)])
def test_sir_prose_equals_definition(num, den):
    rng = np.random.default_rng(100 + num * 10 + den)
    for _ in range(200):
        n = int(rng.integers(1, 90))
        m = rng.random(n) < rng.uniform(0.05, 0.9)
        got = O.sir_prose_rows(m[None, :], num, den)[0]
        assert (got == _prose_by_definition(m, num, den)).all(), (m.astype(int), num, den)


def test_sir_prose_differs_from_operator_and_orders_directions():
    # L = 20: the operator grows floor(L/4) = 5 per side, the prose reading floor(L/5) = 4
    m = np.zeros(60, dtype=bool)
    m[20:40] = True
    assert O.sir_rows(m[None], 1, 5)[0].sum() == 30
    assert O.sir_prose_rows(m[None], 1, 5)[0].sum() == 28
    rng = np.random.default_rng(8)
    blk = rng.random((11, 37)) < 0.3
    got = O.sir_block(blk, O.Params(sir_prose=True))
    rows = np.array([_prose_by_definition(r, 1, 5) for r in blk])
    expect = np.array([_prose_by_definition(c, 1, 5) for c in rows.T]).T
    assert (got == expect).all()
    assert (O.sir_block(blk, O.Params(sir_prose=True, sir_eta_num=0)) == blk).all()


def test_sir_percentage_from_paper():
    g = golden()
    prm = O.Params()
    assert prm.sir_eta_num / prm.sir_eta_den == g["sir_percentage"]["value"]


# --------------------------------------------------------------------- history
def test_history_worked_sequences():
    prm = O.Params(history_sensitivity=6.0)
    ring = [10.0, 10.0, 10.0, 10.0]
    assert O.history_row(40, 4, ring, prm) == (False, 10.0)      # cur = thr: not flagged
    assert O.history_row(42, 4, ring, prm) == (True, 10.0)       # cur > thr: push thr
    lit = O.Params(literal_history_tie=True)
    assert O.history_row(40, 4, ring, lit) == (True, 10.0)
    # ring [1,2,3,4]: mean 2.5, population var 1.25
    prm1 = O.Params(history_sensitivity=1.0)
    thr = 2.5 + math.sqrt(1.25)
    assert O.history_row(3.6, 1, [1.0, 2.0, 3.0, 4.0], prm1) == (False, 3.6)
    f, v = O.history_row(3.7, 1, [1.0, 2.0, 3.0, 4.0], prm1)
    assert f and v == thr
    # warm-up: fewer than history_min entries -> never flags, pushes cur
    assert O.history_row(1e9, 1, [1.0, 1.0, 1.0], prm) == (False, 1e9)
    # fully flagged channel: no flag, no push
    assert O.history_row(0, 0, ring, prm) == (False, None)


def test_history_ring_and_constant_stream():
    prm = O.Params(history_len=5, history_min=2)
    h = O.History(prm)
    x = np.full((3, 64), 2.0, dtype=np.float32)
    for i in range(12):
        r = O.flag_block(x, O.F32, prm, history=h, stream_id=7)
        assert not r.flags.any()
        h.commit()
    assert len(h.ring(7, 0)) == 5 and h.ring(7, 0) == [2.0] * 5
    lit = O.Params(history_len=5, history_min=2, literal_history_tie=True)
    h2 = O.History(lit)
    got = []
    for i in range(5):
        r = O.flag_block(x, O.F32, lit, history=h2, stream_id=0)
        got.append(bool(r.history_rows.all()))
        h2.commit()
    assert got == [False, False, True, True, True]


def test_history_flags_broadband_step():
    prm = O.Params(history_len=8, history_min=4)
    h = O.History(prm)
    rng = np.random.default_rng(21)
    flagged = []
    for i in range(10):
        x = rng.exponential(1.0, size=(4, 256)).astype(np.float32)
        if i == 8:
            x *= 3.0   # a broadband level change longer than the block
        r = O.flag_block(x, O.F32, prm, history=h, stream_id=0)
        flagged.append(bool(r.history_rows.all()))
        h.commit()
    assert flagged[8] and not any(flagged[:8])


def test_history_sizing_from_paper():
    g = golden()
    a = g["history_precorrelation"]
    per_s = O.history_bytes_per_second(a["stations"], a["subbands"], a["channels"], a["bytes"])
    assert round(per_s / 2 ** 20, 1) == a["mbyte_per_s"]
    assert round(per_s * a["entries_5min"] / 2 ** 30, 1) == a["gbyte_5min"]
    b = g["history_postcorrelation"]
    per_s = O.history_bytes_per_second(b["baselines"], b["subbands"], b["channels"], b["bytes"])
    assert round(per_s / 2 ** 20) == b["mbyte_per_s"]
    assert round(per_s * b["entries_5min"] / 2 ** 30) == b["gbyte_5min"]


# ---------------------------------------------------------------- end to end
def test_injected_rfi_is_found_config0_shape():
    import synth
    x, dt = synth.config0()
    r = O.flag_block(x, dt, O.Params())
    rng = synth.rng_for(0, 0)
    # regenerate the plan exactly as the generator drew it
    rng.standard_normal((64, 4096), dtype=np.float32)
    rng.standard_normal((64, 4096), dtype=np.float32)
    plan = synth.rfi_plan(rng, 64, 4096)
    for kind, c0, c1, t0, t1, k, _ in plan:
        frac = r.flags[c0:c1, t0:t1].mean()
        if kind in ("tone", "impulse"):
            assert frac > 0.9, (kind, frac)
    assert r.flags.mean() < 0.2


# ------------------------------------------------------------ integrated mode
# Sec. 4 (integration paragraph): the spectrum (time fully integrated) is
# flagged along frequency first, then the time series of the unflagged channels
# (frequency fully integrated) along time; flags are broadcast back.
def _ci8_from_power(pw):
    """complex int8 block whose power re^2 + im^2 is exactly `pw` (pw = re^2,
    values that are squares of 0..127)."""
    re = np.sqrt(pw).astype(np.int64)
    assert (re * re == pw).all()
    x = np.zeros(pw.shape + (2,), dtype=np.int8)
    x[..., 0] = re
    return x


def test_integrated_constant_block_flags_nothing():
    x = _ci8_from_power(np.full((16, 200), 49, dtype=np.int64))
    r = O.integrated_block(x, O.CI8)
    assert not r.flags.any()
    assert (r.spectrum == 49 * 200).all() and (r.series == 49 * 16).all()


@pytest.mark.parametrize("T,flagged", [(34, False), (35, True), (64, True)])
def test_integrated_broadband_impulse_closed_form(T, flagged):
    # zero background, one time column of power 25 in every channel: the spectrum
    # is constant (no channel flags) and the time series is a single impulse on a
    # zero background, flagged iff its length is at least 35 (N/sqrt(N-1) > 6)
    pw = np.zeros((8, T), dtype=np.int64)
    pw[:, T // 2] = 25
    r = O.integrated_block(_ci8_from_power(pw), O.CI8, O.Params(sir_eta_num=0))
    assert not r.channel_flags.any()
    expect = np.zeros(T, dtype=bool)
    expect[T // 2] = flagged
    assert (r.time_flags == expect).all()
    assert (r.flags == expect[None, :]).all()


def test_integrated_removes_narrowband_rfi_before_the_time_series():
    # background power 1; channel 3 carries a tone of power 100 with two bursts of
    # 10000.  The spectrum flags channel 3; the time series of the other channels
    # is then constant and nothing else is flagged.  Left in, the tone's bursts
    # would flag their two times in every channel.
    C, T = 40, 128
    pw = np.ones((C, T), dtype=np.int64)
    pw[3] = 100
    pw[3, [20, 90]] = 10000
    x = _ci8_from_power(pw)
    prm = O.Params(sir_eta_num=0)
    r = O.integrated_block(x, O.CI8, prm)
    assert r.channel_flags.nonzero()[0].tolist() == [3]
    assert not r.time_flags.any()
    assert (r.flags == (np.arange(C) == 3)[:, None]).all()
    assert O.flag_series(pw.sum(axis=0), prm, True, 7).nonzero()[0].tolist() == [20, 90]


def test_integrated_finds_a_weak_tone_full_rate_misses():
    # a +0.25 sigma narrowband tone in unit complex noise: below the full-rate
    # thresholds at every window size, but 2048 integrated samples lift it clear
    # of the spectrum's noise
    rng = np.random.default_rng(17)
    C, T = 128, 2048
    s = np.float32(np.sqrt(0.5))
    z = (rng.standard_normal((C, T), dtype=np.float32) * s
         + 1j * rng.standard_normal((C, T), dtype=np.float32) * s).astype(np.complex64)
    z[11] += np.complex64(0.5) * np.exp(1j * rng.uniform(0, 2 * np.pi, T)).astype(np.complex64)
    prm = O.Params(sir_eta_num=0)
    full = O.flag_block(z, O.C64, prm)
    assert full.flags[11].mean() < 0.01
    r = O.integrated_block(z, O.C64, prm)
    assert r.channel_flags.nonzero()[0].tolist() == [11]


def test_integrated_int_and_float_agree_on_integer_power():
    rng = np.random.default_rng(5)
    x = synth.ci8_block(rng, 24, 700)
    p = O.power(x, O.CI8)
    a = O.integrated_block(x, O.CI8)
    b = O.integrated_block(p.astype(np.float32), O.F32)
    assert (a.flags == b.flags).all()


def test_series_stddev_exact_beyond_64_bits():
    v = np.array([2 ** 33 - 1, 2 ** 33 - 5, 3, 2 ** 32], dtype=np.int64)
    vals = [int(a) for a in v]
    mu = Fraction(sum(vals), 4)
    var = Fraction(sum(a * a for a in vals), 4) - mu * mu
    assert O.series_stddev(v, True) == pytest.approx(math.sqrt(float(var)), rel=1e-15)


# ------------------------------------------------------------ robust stddev (MAD)
# Sec. 4.2 lists the MAD among the statistics; 1.4826 * MAD estimates the stddev
# of normal noise without the RFI it is meant to find.
def test_mad_sigma_hand_worked():
    p = np.array([[1, 2, 3, 4, 100]], dtype=np.int64)          # median 3, |p - 3| = 2 1 0 1 97
    assert O.block_mad_sigma(p, True) == 1.4826 * 1.0
    q = np.array([[1, 2, 4, 7]], dtype=np.int64)                # median 3, |q - 3| = 2 1 1 4 -> 1.5
    assert O.block_mad_sigma(q, True) == 1.4826 * 1.5
    r = np.array([[1, 2, 3, 6]], dtype=np.int64)                # median 2.5, |r - 2.5| = 1.5 .5 .5 3.5 -> 1
    assert O.block_mad_sigma(r, True) == 1.4826 * 1.0
    assert O.block_mad_sigma(p.astype(np.float64), False) == 1.4826 * 1.0


def test_mad_sigma_ignores_outlier_size():
    rng = np.random.default_rng(3)
    p = rng.integers(0, 1000, size=(8, 125))
    base = O.block_mad_sigma(p, True)
    q = p.copy()
    q[p > 900] = 10 ** 6                                       # far beyond median + MAD already
    assert O.block_mad_sigma(q, True) == base
    assert O.block_stddev(q, True) > 10 * O.block_stddev(p, True)


def test_mad_sigma_estimates_normal_stddev():
    rng = np.random.default_rng(4)
    x = rng.normal(10.0, 2.0, size=200_000)
    assert O.block_mad_sigma(x, False) == pytest.approx(2.0, rel=0.01)


def test_mad_sigma_int_equals_float_on_integers():
    rng = np.random.default_rng(6)
    for n in (1, 2, 3, 10, 101, 1000):
        p = rng.integers(0, 5000, size=n)
        assert O.block_mad_sigma(p, True) == O.block_mad_sigma(p.astype(np.float64), False)


def test_robust_sigma_finds_tones_the_classic_stddev_hides():
    # three strong tone channels among 64 inflate the spectrum's stddev so much
    # that 6 sigma misses them; the MAD-based stddev does not
    rng = np.random.default_rng(9)
    C, T = 64, 512
    pw = rng.integers(90, 111, size=(C, T)).astype(np.int64)
    for ch in (5, 21, 40):
        pw[ch] = 900
    sq = np.rint(np.sqrt(pw)).astype(np.int64)
    x = np.zeros((C, T, 2), dtype=np.int8)
    x[..., 0] = sq
    prm = O.Params(sir_eta_num=0)
    assert not O.integrated_block(x, O.CI8, prm).channel_flags.any()
    r = O.integrated_block(x, O.CI8, O.Params(sir_eta_num=0, robust_sigma=True))
    assert r.channel_flags.nonzero()[0].tolist() == [5, 21, 40]


# ------------------------------------------------- 2-D partial integration pins
def test_partial_unit_tiles_equal_full_rate():
    # tiles of one sample: the grid of means is the block itself (float32 power),
    # so the result is the full-rate path's, history included
    rng = np.random.default_rng(31)
    x = synth.f32_power_block(rng, 24, 500)
    prm = O.Params(history_min=1, history_len=4)
    h1, h2 = O.History(prm), O.History(prm)
    for _ in range(3):
        r = O.partial_block(x, O.F32, prm, 1, 1, h1, 0)
        f = O.flag_block(x, O.F32, prm, h2, 0)
        assert (r.flags == f.flags).all()
        assert h1.pending == h2.pending
        h1.commit()
        h2.commit()
        x = x * np.float32(1.5)


def test_partial_full_time_integration_is_the_integrated_spectrum_step():
    # one tile per channel (f_time = T, T a power of two so the means are the exact
    # spectrum / T): the 1 x C grid is flagged at level 1 along time and levels
    # 2..64 along frequency, which is the integrated mode's spectrum flagging
    # (Sec. 4) on a scaled spectrum, SIR included
    rng = np.random.default_rng(5)
    x = synth.ci8_block(rng, 64, 64, rfi=False)
    x[11, :, 0] = np.clip(x[11, :, 0].astype(np.int64) + 60, -127, 127)   # a strong tone
    prm = O.Params()
    r = O.partial_block(x, O.CI8, prm, f_time=64, f_freq=1)
    ri = O.integrated_block(x, O.CI8, prm)
    assert ri.channel_flags.any()
    assert (r.coarse[:, 0].astype(np.float64) * 64 == ri.spectrum).all()
    assert (r.flags == ri.channel_flags[:, None]).all()


def test_partial_full_frequency_integration_is_the_integrated_time_series_step():
    # one tile per time (f_freq = C = 64): the grid is the all-channel time series
    # / 64; when the integrated mode flags no channel its time series is the same
    # sum, so the time flags agree
    rng = np.random.default_rng(8)
    x = synth.ci8_block(rng, 64, 1000, rfi=False)
    x[:, 300:304, 0] = 60            # a broadband impulse, 4 samples wide
    prm = O.Params()
    ri = O.integrated_block(x, O.CI8, prm)
    assert not ri.channel_flags.any() and ri.time_flags[300:304].all()
    r = O.partial_block(x, O.CI8, prm, f_time=1, f_freq=64)
    assert (r.coarse[0].astype(np.float64) * 64 == ri.series).all()
    assert (r.flags == ri.time_flags[None, :]).all()


def test_partial_tile_constant_block_with_ragged_tiles():
    # power constant on every tile, edge tiles narrower (30 channels in tiles of 4,
    # 50 times in tiles of 8): each tile mean is that constant whatever the tile's
    # size, so the flags are the full-rate flags of the 8 x 7 grid of constants,
    # spread over the tiles; the one strong tile is the ragged corner (2 x 2
    # samples), flagged alone among 56 (a single impulse needs N >= 35)
    rng = np.random.default_rng(12)
    vals = rng.integers(1, 12, size=(8, 7)) ** 2
    vals[7, 6] = 120 * 120
    rows, cols = np.arange(30) // 4, np.arange(50) // 8
    x = _ci8_from_power(vals[rows][:, cols])
    prm = O.Params(sir_eta_num=0)
    r = O.partial_block(x, O.CI8, prm, f_time=8, f_freq=4)
    assert (r.coarse == vals.astype(np.float32)).all()
    g = O.flag_block(vals.astype(np.float32), O.F32, prm)
    assert g.flags[7, 6]
    assert (r.flags == g.flags[rows][:, cols]).all()
    assert r.flags[28:, 48:].all()


@pytest.mark.parametrize("T,j0", [(128, 5), (125, 15)])
def test_partial_broadband_impulse_hand_worked(T, j0):
    # background power 1, power 400 in every channel over the times of tile column
    # j0 (the last, 5 samples wide, when T = 125): the grid column of 400s is
    # flagged along frequency (window of 4 tiles: mean 400 > 1 + 3.375 sigma,
    # sigma = 399 * sqrt(15) / 16 ~ 96.6), a single flagged tile per row does not
    # grow under SIR (floor(1/4) = 0), so exactly the impulse's times are flagged
    C = 8
    pw = np.ones((C, T), dtype=np.int64)
    t = np.arange(T)
    pw[:, t // 8 == j0] = 400
    r = O.partial_block(_ci8_from_power(pw), O.CI8, O.Params(), f_time=8, f_freq=2)
    assert r.coarse.shape == (4, 16)
    assert (r.flags == (t // 8 == j0)[None, :]).all()


# --------------------------------------------------------- caller-supplied pre-flags
def test_preflags_none_equal_no_preflags():
    x = synth.ci8_block(np.random.default_rng(40), 16, 300)
    a = O.flag_block(x, O.CI8)
    b = O.flag_block(x, O.CI8, preflags=np.zeros((16, 300), dtype=bool))
    assert (a.flags == b.flags).all() and a.median == b.median and a.stddev == b.stddev


@pytest.mark.parametrize("robust", [False, True])
def test_preflags_leave_the_statistics(robust):
    rng = np.random.default_rng(41)
    x = synth.ci8_block(rng, 12, 500)
    pre = rng.random((12, 500)) < 0.3
    r = O.flag_block(x, O.CI8, O.Params(robust_sigma=robust), preflags=pre)
    live = O.power(x, O.CI8)[~pre].astype(np.float64)
    assert r.median == np.median(live)
    sd = 1.4826 * np.median(np.abs(live - np.median(live))) if robust else np.std(live)
    assert r.stddev == pytest.approx(sd, rel=1e-12)
    assert r.flags[pre].all()


def test_preflagged_rows_are_removed_rows():
    # frequency levels and SIR off: rows are independent along time, so
    # pre-flagging whole rows is the same as flagging the block without them
    rng = np.random.default_rng(42)
    x = synth.ci8_block(rng, 20, 700)
    rows = np.zeros(20, dtype=bool)
    rows[[1, 5, 6, 17]] = True
    prm = O.Params(n_levels_freq=0, sir_eta_num=0)
    r = O.flag_block(x, O.CI8, prm, preflags=np.repeat(rows[:, None], 700, axis=1))
    q = O.flag_block(x[~rows], O.CI8, prm)
    assert r.flags[rows].all()
    assert (r.flags[~rows] == q.flags).all() and r.thresholds == q.thresholds


def test_preflagging_a_strong_burst_reveals_a_weak_outlier():
    # power 1 everywhere, a burst of 10^4 over 10 % of the block and one sample of
    # power 16: the burst's share of the stddev hides the outlier; with the burst
    # pre-flagged the remaining samples have median 1 and stddev 15/sqrt(N), and
    # the lone outlier is flagged (N >= 35)
    C, T = 10, 100
    pw = np.ones((C, T), dtype=np.int64)
    pw[:, 40:50] = 100 * 100
    pw[3, 80] = 16
    x = _ci8_from_power(pw)
    prm = O.Params(sir_eta_num=0)
    plain = O.flag_block(x, O.CI8, prm)
    assert not plain.flags[3, 80]
    pre = np.zeros((C, T), dtype=bool)
    pre[:, 40:50] = True
    r = O.flag_block(x, O.CI8, prm, preflags=pre)
    n = C * T - pre.sum()
    assert r.median == 1.0 and r.stddev == pytest.approx(15 * np.sqrt(n - 1) / n, rel=1e-12)
    expect = pre.copy()
    expect[3, 80] = True
    assert (r.flags == expect).all()


@pytest.mark.parametrize("seed", range(12))
def test_preflags_tiny_exhaustive_vs_rational_bruteforce(seed):
    # SumThreshold from a random initial mask, window by window in exact
    # rational arithmetic, with the thresholds of the unflagged samples
    rng = np.random.default_rng(2000 + seed)
    C, T = int(rng.integers(1, 6)), int(rng.integers(2, 9))
    x = rng.integers(-6, 7, size=(C, T, 2)).astype(np.int8)
    x[rng.integers(0, C), rng.integers(0, T), 0] = 50
    pre = rng.random((C, T)) < 0.25
    prm = O.Params(start_threshold=float(rng.choice([0.5, 1.0, 2.0])), sir_eta_num=0)
    r = O.flag_block(x, O.CI8, prm, preflags=pre)
    p = O.power(x, O.CI8)
    live = sorted(int(v) for v in p[~pre])
    if live:
        n = len(live)
        med = Fraction(live[n // 2]) if n % 2 else Fraction(live[n // 2 - 1] + live[n // 2], 2)
        assert r.median == float(med)
    th = r.thresholds

    def run(rows, masks):
        out = []
        for vals, m in zip(rows, masks):
            m = list(m)
            for k in range(prm.n_levels):
                I = 1 << k
                if I > len(vals):
                    break
                nm = list(m)
                for s in range(len(vals) - I + 1):
                    live_w = [vals[j] for j in range(s, s + I) if not m[j]]
                    if live_w and Fraction(sum(live_w)) > len(live_w) * Fraction(th[k]):
                        for j in range(s, s + I):
                            nm[j] = True
                m = nm
            out.append(m)
        return np.array(out, dtype=bool)
    mt = run([[int(v) for v in row] for row in p], pre.tolist())
    mf = run([[int(v) for v in col] for col in p.T], mt.T.tolist()).T
    assert (r.st_mask == mf).all()


# ------------------------------------------------------ winsorized history statistics
def test_winsorize_ring_hand_worked():
    assert O.winsorize_ring([1.0, 2.0, 3.0, 4.0, 100.0], 1) == [2.0, 2.0, 3.0, 4.0, 4.0]
    assert O.winsorize_ring([5.0, -7.0, 5.0, 9.0], 1) == [5.0, 5.0, 5.0, 5.0]   # k = 1: 2nd smallest, 2nd largest
    assert O.winsorize_ring([3.0, 1.0], 5) == [3.0, 1.0]                      # k capped at (L-1)//2 = 0


@pytest.mark.parametrize("L,k", [(5, 1), (8, 2), (32, 3), (33, 16), (7, 0)])
def test_winsorize_ring_equals_scipy(L, k):
    from scipy.stats import mstats
    rng = np.random.default_rng(L * 10 + k)
    ring = rng.standard_normal(L).tolist()
    ring[3 % L] = 50.0
    want = np.asarray(mstats.winsorize(np.array(ring), limits=((k + 0.5) / L, (k + 0.5) / L))).tolist()
    assert O.winsorize_ring(ring, k) == want


def test_winsorized_history_threshold_closed_form():
    # ring [1, 2, 3, 4, 100], k = 1 -> [2, 2, 3, 4, 4]: mean 3, variance 0.8
    # (threshold 3 + 2 sqrt(0.8) = 4.79: a current mean of 10 is flagged and the
    # threshold is pushed)
    prm = O.Params(history_min=1, history_winsor=1, history_sensitivity=2.0)
    f, pv = O.history_row(100, 10, [1.0, 2.0, 3.0, 4.0, 100.0], prm)
    thr = 3.0 + 2.0 * np.sqrt(0.8)
    assert f and pv == pytest.approx(thr, rel=1e-15)
    # without winsorizing the outlier inflates the threshold (mean 22, stddev 39)
    # far above the current mean
    f0, pv0 = O.history_row(100, 10, [1.0, 2.0, 3.0, 4.0, 100.0], O.Params(history_min=1, history_sensitivity=2.0))
    assert not f0 and pv0 == 10.0


def test_winsorized_history_ignores_an_outlier_second():
    # one second of strong broadband RFI committed into the ring does not move the
    # winsorized threshold, whatever its size
    prm = O.Params(history_min=1, history_winsor=1)
    base = [10.0, 10.5, 9.5, 10.2, 9.8, 10.1]
    t1 = O.history_row(0, 1, base + [1e3], prm)
    t2 = O.history_row(0, 1, base + [1e9], prm)
    assert t1 == t2
