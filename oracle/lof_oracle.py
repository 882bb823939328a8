"""Plain CPU reference ("oracle") for the LOFAR Online Flagger (LOF) hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  The product
path (the HIP library behind ``include/lof.h``) never calls it, shares no code,
tables or constants with it, and does not import it.

Everything here is written from van Nieuwpoort, "Towards exascale real-time RFI
mitigation" (arXiv 1701.08197), in float64 (exact Python/NumPy integers where
the input is integer), favouring obviousness over speed:

* power formation ............................ Sec. 4 (first paragraph)
* block median and standard deviation ......... Sec. 2.1 threshold definition, Sec. 4.2
* SumThreshold thresholds and levels .......... Sec. 2.1 (threshold_I, factor_I, worked
                                                 values 6 sigma at I=1, 4.5 sigma at I=2)
* SumThreshold in time then frequency ......... Sec. 2.1 (one-dimensional mode, both
                                                 directions)
* scale-invariant rank (SIR) operator ......... Sec. 2.2 (and its cited linear algorithm,
                                                 van de Gronde et al. 2016)
* history flagger ............................. Sec. 4.1 (pseudocode and Fig. "history")
* integrated pre-correlation mode ............. Sec. 4 (integration paragraph, Fig. "integrate")
* robust stddev from the MAD .................. Sec. 4.2 (statistics list)
* 2-D flagging with partial integration ....... Sec. 4 (integration paragraph, the
                                                 alternative method)
* winsorized history statistics ............... Sec. 4.2 (statistics list)
* caller-supplied pre-flags ................... Sec. 4.2 (statistics of the unflagged
                                                 samples), Sec. 2.1 (flagged samples
                                                 leave the window sums)

Where the paper is silent or garbled, each function states the reading it
implements.  Window sums are brute force
(a direct sum over each window), the median is a full sort, and integer-input
comparisons are exact rational comparisons (``fractions.Fraction``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

# Input sample types (Sec. 4: voltages need power/amplitude first; visibilities
# are flagged on amplitude; beam-formed data is Stokes I as given).
CI8 = 0      # complex int8 voltages (interleaved re, im) -> exact integer power
C64 = 1      # complex64 voltages -> power re^2 + im^2
F32 = 2      # float32 power / Stokes I, flagged as given
C64_AMP = 3  # complex64 visibilities -> amplitude sqrt(re^2 + im^2)


@dataclass(frozen=True)
class Params:
    """Flagger parameters.  Defaults: Sec. 2.1 (p = 1.5, sensitivity = 1.0, a 6 sigma
    first threshold, 7 iterations -> I = 1..64), Sec. 2.2 (SIR 20 %), Sec. 4.1
    (history)."""
    start_threshold: float = 6.0
    p: float = 1.5
    sensitivity: float = 1.0
    n_levels: int = 7
    n_levels_freq: int = -1          # -1: same as n_levels
    sir_eta_num: int = 1             # eta = num / den = 0.2; num = 0 disables SIR
    sir_eta_den: int = 5
    history_sensitivity: float = 6.0
    history_len: int = 32
    history_min: int = 4
    literal_history_tie: bool = False  # True: flag when cur >= thr (listing's else-branch)
    sir_prose: bool = False            # True: the prose reading of Sec. 2.2 (sir_prose_rows)
    robust_sigma: bool = False         # True: stddev from the MAD (block_mad_sigma, Sec. 4.2)
    history_winsor: int = 0            # k > 0: the ring's mean and stddev after winsorizing k per side

    @property
    def levels_freq(self) -> int:
        return self.n_levels if self.n_levels_freq < 0 else self.n_levels_freq


# --------------------------------------------------------------------------- power
def power(x: np.ndarray, dtype: int) -> np.ndarray:
    """Per-sample flagged quantity (Sec. 4).

    CI8: ``x`` int8 [C, T, 2] -> int64 re^2 + im^2 (exact).
    C64: complex64 [C, T] -> float64 re^2 + im^2 from the float32 components.
    F32: float32 [C, T] -> float64 as given.
    C64_AMP: complex64 [C, T] -> float64 sqrt(re^2 + im^2).
    """
    if dtype == CI8:
        re = x[..., 0].astype(np.int64)
        im = x[..., 1].astype(np.int64)
        return re * re + im * im
    if dtype == F32:
        return np.asarray(x, dtype=np.float64)
    re = np.real(x).astype(np.float64)
    im = np.imag(x).astype(np.float64)
    pw = re * re + im * im
    if dtype == C64:
        return pw
    if dtype == C64_AMP:
        return np.sqrt(pw)
    raise ValueError(f"unknown dtype {dtype}")


def is_exact(dtype: int) -> bool:
    return dtype == CI8


# ---------------------------------------------------------------------- statistics
def block_median(p: np.ndarray) -> float:
    """Median of all samples of the block (Sec. 2.1 'median'), by full sort.

    Even count: mean of the two middle order statistics."""
    a = np.sort(p.ravel())
    n = a.size
    if n % 2 == 1:
        return float(a[n // 2])
    lo = float(a[n // 2 - 1])
    hi = float(a[n // 2])
    return (lo + hi) / 2.0


def block_stddev(p: np.ndarray, exact: bool) -> float:
    """Population standard deviation of all samples of the block (Sec. 2.1 'stddev').

    mu = S1/N, var = max(S2/N - mu*mu, 0), sigma = sqrt(var), evaluated in float64
    in exactly this order.  Integer input: S1 and S2 are exact integers."""
    n = p.size
    if exact:
        s1 = int(np.sum(p, dtype=np.int64))
        s2 = int(np.sum(p * p, dtype=np.int64))
        mu = s1 / n                      # correctly rounded quotient of two integers
        ex2 = s2 / n
    else:
        flat = p.ravel()
        mu = math.fsum(flat.tolist()) / n
        ex2 = math.fsum((flat * flat).tolist()) / n
    var = ex2 - mu * mu
    if var < 0.0:
        var = 0.0
    return math.sqrt(var)


MAD_TO_SIGMA = 1.4826   # stddev of a normal distribution per unit of its MAD (1 / 0.6745)


def block_mad_sigma(p: np.ndarray, exact: bool) -> float:
    """Robust stddev of the block (Sec. 4.2 lists the MAD among the statistics
    used): 1.4826 * median(|p - median(p)|), both medians with the numpy
    definition.  Integer input: |2p - 2 median| are integers, so the MAD is exact
    (an integer or a half-integer, then halved); the product is one float64
    rounding."""
    med = block_median(p)
    if exact:
        d2 = np.abs(2 * p.astype(np.int64).ravel() - int(round(2 * med)))
        mad = block_median(d2) / 2.0
    else:
        mad = block_median(np.abs(p.ravel() - med))
    return MAD_TO_SIGMA * mad


def level_factors(params: Params, n: int) -> list[float]:
    """factor_I for I = 2^k, k < n (Sec. 2.1): startThreshold * p^(log2 I) / I,
    with p^k by repeated multiplication."""
    out = []
    pk = 1.0
    for k in range(n):
        out.append(params.start_threshold * pk / float(2 ** k))
        pk = pk * params.p
    return out


def thresholds(median: float, sigma: float, params: Params, n: int | None = None) -> list[float]:
    """threshold_I = median + stddev * factor_I * sensitivity (Sec. 2.1)."""
    n = max(params.n_levels, params.levels_freq) if n is None else n
    return [median + sigma * (f * params.sensitivity) for f in level_factors(params, n)]


# ------------------------------------------------------------------- SumThreshold
def _exceeds(S: np.ndarray, c: np.ndarray, T: float, I: int, exact: bool) -> np.ndarray:
    """Window test of Sec. 2.1: mean of the window's unflagged samples above T,
    i.e. S > c*T with c > 0.  Integer input: exact rational comparison."""
    if exact:
        tf = Fraction(T)
        table = np.array([math.floor(cc * tf) for cc in range(I + 1)], dtype=np.int64)
        return (c > 0) & (S > table[c])
    return (c > 0) & (S > c.astype(np.float64) * T)


def sumthreshold_rows(p: np.ndarray, mask: np.ndarray, T: list[float], n_levels: int,
                      exact: bool) -> np.ndarray:
    """One-dimensional SumThreshold along axis 1 of ``p`` (Sec. 2.1), every row
    independently, for I = 1, 2, 4, ... while I <= row length.

    Level-synchronous: every full window [s, s+I) of level k is judged against the
    mask left by level k-1; samples already flagged are left out of the window's sum
    and count; a window that exceeds flags all of its samples; flags only accumulate.
    """
    R, n = p.shape
    m = mask.copy()
    for k in range(n_levels):
        I = 1 << k
        if I > n:
            break
        nw = n - I + 1
        unfl = ~m
        v = np.where(unfl, p, 0)
        S = np.zeros((R, nw), dtype=v.dtype)
        c = np.zeros((R, nw), dtype=np.int64)
        for d in range(I):                      # brute force: sum every window directly
            S += v[:, d:d + nw]
            c += unfl[:, d:d + nw]
        hit = _exceeds(S, c, T[k], I, exact)
        new = m.copy()
        for d in range(I):
            new[:, d:d + nw] |= hit
        m = new
    return m


def sumthreshold_block(p: np.ndarray, T: list[float], params: Params, exact: bool,
                       mask: np.ndarray | None = None) -> np.ndarray:
    """SumThreshold over a [C, T] block: all levels along time (rows), then all levels
    along frequency (columns) starting from the time result (Sec. 2.1)."""
    m = np.zeros(p.shape, dtype=bool) if mask is None else mask.copy()
    m = sumthreshold_rows(p, m, T, params.n_levels, exact)
    m = sumthreshold_rows(p.T, m.T, T, params.levels_freq, exact).T
    return np.ascontiguousarray(m)


# ------------------------------------------------------------------------------ SIR
def sir_row_bruteforce(mask: np.ndarray, num: int, den: int) -> np.ndarray:
    """SIR operator on one 1-D mask by enumerating all intervals (Sec. 2.2):
    y is flagged iff some interval [a, b) containing y holds at most eta*(b-a)
    unflagged samples, eta = num/den.  Pure Python; small inputs only."""
    n = len(mask)
    out = np.array(mask, dtype=bool)
    unfl = [0]
    for v in mask:
        unfl.append(unfl[-1] + (0 if v else 1))
    for a in range(n):
        for b in range(a + 1, n + 1):
            if den * (unfl[b] - unfl[a]) <= num * (b - a):
                out[a:b] = True
    return out


def sir_rows(mask: np.ndarray, num: int, den: int) -> np.ndarray:
    """Linear-time SIR operator along axis 1 (Sec. 2.2, the linear algorithm of the
    cited van de Gronde et al. paper): weights w = num (flagged) or num - den
    (unflagged), W = running sum with W[0] = 0; y is flagged iff
    max_{b > y} W[b] - min_{a <= y} W[a] >= 0."""
    R, n = mask.shape
    w = np.where(mask, num, num - den).astype(np.int64)
    W = np.zeros((R, n + 1), dtype=np.int64)
    W[:, 1:] = np.cumsum(w, axis=1)
    pmin = np.minimum.accumulate(W[:, :n], axis=1)
    smax = np.maximum.accumulate(W[:, :0:-1], axis=1)[:, ::-1]   # smax[y] = max W[y+1..n]
    return (smax - pmin) >= 0


def sir_prose_rows(mask: np.ndarray, num: int, den: int) -> np.ndarray:
    """The prose reading of Sec. 2.2 along axis 1: every maximal range of consecutive
    flagged samples in a row, of length L, is extended by floor(eta * L) samples
    before it and after it (eta = num/den: 20 % -> 1/5), clipped to the row.  The
    extensions of all ranges of the given mask are combined by OR; they are not
    applied again to the grown ranges."""
    R, n = mask.shape
    out = mask.copy()
    for r in range(R):
        y = 0
        while y < n:
            if not mask[r, y]:
                y += 1
                continue
            s = y
            while y < n and mask[r, y]:
                y += 1
            ext = (num * (y - s)) // den
            out[r, max(0, s - ext):min(n, y + ext)] = True
    return out


def sir_block(mask: np.ndarray, params: Params) -> np.ndarray:
    """SIR in time (rows) then in frequency (columns) on the time result (Sec. 2.2);
    the scale-invariant rank operator, or with ``params.sir_prose`` the range
    extension the section's prose describes."""
    if params.sir_eta_num == 0:
        return mask.copy()
    op = sir_prose_rows if params.sir_prose else sir_rows
    m = op(mask, params.sir_eta_num, params.sir_eta_den)
    m = op(m.T, params.sir_eta_num, params.sir_eta_den).T
    return np.ascontiguousarray(m)


# -------------------------------------------------------------------------- history
@dataclass
class History:
    """History flagger state (Sec. 4.1): per (stream, channel) a sliding window of the
    committed means of unflagged samples of past blocks, plus one pending value that
    the next commit pushes."""
    params: Params
    rings: dict = field(default_factory=dict)     # (stream, ch) -> list, oldest first
    pending: dict = field(default_factory=dict)   # (stream, ch) -> float

    def ring(self, stream: int, ch: int) -> list:
        return self.rings.get((stream, ch), [])

    def commit(self, streams=None) -> None:
        keys = list(self.pending.keys())
        for key in keys:
            if streams is not None and key[0] not in streams:
                continue
            r = self.rings.setdefault(key, [])
            r.append(self.pending.pop(key))
            if len(r) > self.params.history_len:
                del r[0]


def winsorize_ring(ring: list, k: int) -> list:
    """Winsorized history (Sec. 4.2 lists winsorized means among the statistics):
    the k smallest committed means are replaced by the (k+1)-th smallest and the
    k largest by the (k+1)-th largest (k at most (L-1)//2 for L values), in ring
    order."""
    L = len(ring)
    k = min(k, (L - 1) // 2)
    srt = sorted(ring)
    lo, hi = srt[k], srt[L - 1 - k]
    return [min(max(x, lo), hi) for x in ring]


def history_row(cur_sum, n_unflagged: int, ring: list, params: Params):
    """Compare one channel's current mean with its history (Sec. 4.1 listing).

    Returns (flag, pending) where pending is None when nothing is pushed.
    cur = mean of unflagged samples; with at least history_min committed means,
    thr = mean(ring) + history_sensitivity * std(ring) (population, sequential sums;
    with history_winsor = k, of the winsorized ring, winsorize_ring);
    the channel is flagged when cur > thr (or >= with the literal tie) and then the
    pushed value is thr, else cur.  During warm-up the value is pushed unflagged; a
    fully flagged channel neither flags nor pushes."""
    if n_unflagged == 0:
        return False, None
    cur = cur_sum / n_unflagged          # int/int: correctly rounded; float: float64
    L = len(ring)
    if L < params.history_min:
        return False, float(cur)
    if params.history_winsor > 0:
        ring = winsorize_ring(ring, params.history_winsor)
    acc = 0.0
    for x in ring:
        acc += x
    hm = acc / L
    acc = 0.0
    for x in ring:
        d = x - hm
        acc += d * d
    hv = acc / L
    thr = hm + params.history_sensitivity * math.sqrt(hv)
    flag = (cur >= thr) if params.literal_history_tie else (cur > thr)
    return flag, (thr if flag else float(cur))


# ------------------------------------------------------------------------- pipeline
@dataclass
class BlockResult:
    flags: np.ndarray          # bool [C, T]
    median: float
    stddev: float
    thresholds: list
    st_mask: np.ndarray        # after SumThreshold (time + frequency)
    sir_mask: np.ndarray       # after SIR
    history_rows: np.ndarray   # bool [C]
    pending: list              # per channel: float or None


def flag_block(x: np.ndarray, dtype: int, params: Params = Params(),
               history: History | None = None, stream_id: int = -1,
               preflags: np.ndarray | None = None) -> BlockResult:
    """The whole per-block hot path: power -> median, stddev -> thresholds ->
    SumThreshold time then frequency -> SIR time then frequency -> history flagger
    (pending values are staged in ``history``; call ``history.commit``).

    ``preflags`` (bool [C, T]) marks samples flagged before the flagger runs
    (Sec. 4.2: the statistics are those of the unflagged samples): they leave the
    median and stddev (with none left, both are 0), start flagged in SumThreshold
    (so they leave every window's sum and count) and stay flagged."""
    exact = is_exact(dtype)
    p = power(x, dtype)
    C, T = p.shape
    pre = None if preflags is None else np.asarray(preflags, dtype=bool)
    live = p if pre is None else p[~pre]
    if live.size == 0:
        med, sd = 0.0, 0.0
    else:
        med = block_median(live)
        sd = block_mad_sigma(live, exact) if params.robust_sigma else block_stddev(live, exact)
    th = thresholds(med, sd, params)
    st = sumthreshold_block(p, th, params, exact, mask=pre)
    sm = sir_block(st, params)
    hrows = np.zeros(C, dtype=bool)
    pend = [None] * C
    if history is not None and stream_id >= 0:
        for c in range(C):
            unfl = ~sm[c]
            n_u = int(unfl.sum())
            if exact:
                s = int(np.sum(p[c][unfl], dtype=np.int64))
            else:
                s = math.fsum(p[c][unfl].tolist())
            f, pv = history_row(s, n_u, history.ring(stream_id, c), params)
            hrows[c] = f
            pend[c] = pv
            if pv is not None:
                history.pending[(stream_id, c)] = pv
    flags = sm | hrows[:, None]
    return BlockResult(flags, med, sd, th, st, sm, hrows, pend)


# ------------------------------------------------------------- integrated mode
def series_stddev(v: np.ndarray, exact: bool) -> float:
    """Population standard deviation of a 1-D series with the formula of
    block_stddev; integer series use Python integers throughout (their squares
    can exceed 64 bits), and mu = S1/N, E[x^2] = S2/N are the correctly rounded
    quotients."""
    n = v.size
    if exact:
        s1 = sum(int(a) for a in v.tolist())
        s2 = sum(int(a) * int(a) for a in v.tolist())
        mu = s1 / n
        ex2 = s2 / n
    else:
        mu = math.fsum(v.tolist()) / n
        ex2 = math.fsum((v * v).tolist()) / n
    var = ex2 - mu * mu
    if var < 0.0:
        var = 0.0
    return math.sqrt(var)


def series_thresholds(v: np.ndarray, params: Params, exact: bool, n_levels: int):
    """(median, stddev, thresholds) of one integrated 1-D series (Sec. 2.1)."""
    med = block_median(v)
    sd = block_mad_sigma(v, exact) if params.robust_sigma else series_stddev(v, exact)
    return med, sd, thresholds(med, sd, params, max(1, n_levels))


def flag_series(v: np.ndarray, params: Params, exact: bool, n_levels: int) -> np.ndarray:
    """Flags of one integrated 1-D series: its own median and stddev, the
    thresholds of Sec. 2.1, one-dimensional SumThreshold, then the SIR step
    (Sec. 2.2) on the series' mask."""
    _, _, th = series_thresholds(v, params, exact, n_levels)
    m = sumthreshold_rows(v[None, :], np.zeros((1, v.size), dtype=bool), th, n_levels, exact)
    if params.sir_eta_num > 0:
        op = sir_prose_rows if params.sir_prose else sir_rows
        m = op(m, params.sir_eta_num, params.sir_eta_den)
    return m[0]


@dataclass
class IntegratedResult:
    flags: np.ndarray          # bool [C, T]: channel flags OR time flags (then history rows)
    channel_flags: np.ndarray  # bool [C]
    time_flags: np.ndarray     # bool [T]
    spectrum: np.ndarray       # [C] time-integrated power
    series: np.ndarray         # [T] frequency-integrated power of the unflagged channels
    history_rows: np.ndarray
    pending: list


def integrated_block(x: np.ndarray, dtype: int, params: Params = Params(),
                     history: History | None = None, stream_id: int = -1) -> IntegratedResult:
    """Integrated pre-correlation mode (Sec. 4, integration paragraph): integrate
    time fully and flag the spectrum along frequency first (this removes strong
    narrow-band RFI before the time statistics are formed), then integrate the
    unflagged channels fully and flag the time series along time; a flagged
    channel flags its whole row, a flagged time flags its whole column.  Sums are
    exact integers for complex int8 input, float64 otherwise.  The history
    flagger (Sec. 4.1) then runs on the result as in flag_block."""
    exact = is_exact(dtype)
    p = power(x, dtype)
    C, T = p.shape
    if exact:
        spec = p.sum(axis=1, dtype=np.int64)
    else:
        spec = np.array([math.fsum(r.tolist()) for r in p])
    chan = flag_series(spec, params, exact, min(params.levels_freq, ST_LEVELS_MAX))
    keep = ~chan
    if exact:
        series = p[keep].sum(axis=0, dtype=np.int64) if keep.any() else np.zeros(T, dtype=np.int64)
    else:
        series = (np.array([math.fsum(col.tolist()) for col in p[keep].T]) if keep.any()
                  else np.zeros(T))
    tim = flag_series(series, params, exact, min(params.n_levels, ST_LEVELS_MAX))
    m = chan[:, None] | tim[None, :]
    hrows = np.zeros(C, dtype=bool)
    pend = [None] * C
    if history is not None and stream_id >= 0:
        for c in range(C):
            unfl = ~m[c]
            n_u = int(unfl.sum())
            s = int(np.sum(p[c][unfl], dtype=np.int64)) if exact else math.fsum(p[c][unfl].tolist())
            f, pv = history_row(s, n_u, history.ring(stream_id, c), params)
            hrows[c] = f
            pend[c] = pv
            if pv is not None:
                history.pending[(stream_id, c)] = pv
    return IntegratedResult(m | hrows[:, None], chan, tim, spec, series, hrows, pend)


ST_LEVELS_MAX = 7   # windows up to 64 samples


# ------------------------------------------------- 2-D partial integration
@dataclass
class PartialResult:
    flags: np.ndarray          # bool [C, T]: each sample takes its tile's flag
    coarse: np.ndarray         # float32 [ceil(C/f_freq), ceil(T/f_time)] tile means
    coarse_result: BlockResult  # the 2-D path on the coarse grid


def integrate_tiles(p: np.ndarray, f_time: int, f_freq: int, exact: bool) -> np.ndarray:
    """Tile means of the power (Sec. 4: partial integration in one or both
    dimensions): tile (i, j) covers channels [i f_freq, (i+1) f_freq) and times
    [j f_time, (j+1) f_time), clipped to the block, so edge tiles may hold fewer
    samples; its value is the sum of its samples (exact integer, or an exact
    float sum) divided by their number, rounded once to float32."""
    C, T = p.shape
    Cc, Tc = -(-C // f_freq), -(-T // f_time)
    out = np.zeros((Cc, Tc), dtype=np.float32)
    for i in range(Cc):
        for j in range(Tc):
            tile = p[i * f_freq:(i + 1) * f_freq, j * f_time:(j + 1) * f_time]
            if exact:
                total = sum(int(v) for v in tile.ravel().tolist())
            else:
                total = math.fsum(tile.ravel().tolist())
            out[i, j] = np.float32(total / tile.size)
    return out


def partial_block(x: np.ndarray, dtype: int, params: Params = Params(), f_time: int = 1, f_freq: int = 1,
                  history: History | None = None, stream_id: int = -1) -> PartialResult:
    """2-D flagging with partial integration (Sec. 4, the alternative to the
    integrated mode): integrate the power over tiles of f_freq channels x f_time
    times (integrate_tiles), run the whole 2-D path of flag_block on the grid of
    tile means (statistics, SumThreshold time then frequency, SIR, history per
    row of tiles, keyed by the tile row), and give every sample its tile's flag."""
    p = power(x, dtype)
    C, T = p.shape
    coarse = integrate_tiles(p, f_time, f_freq, is_exact(dtype))
    r = flag_block(coarse, F32, params, history, stream_id)
    rows = np.arange(C) // f_freq
    cols = np.arange(T) // f_time
    return PartialResult(r.flags[rows][:, cols], coarse, r)


# ----------------------------------------------------------------------- sizing aid
def history_bytes_per_second(n_streams: int, n_subbands: int, n_channels: int,
                             bytes_per_value: int = 4) -> int:
    """History growth per second of data (Sec. 4.2): one value per stream, subband
    and channel per second."""
    return n_streams * n_subbands * n_channels * bytes_per_value
