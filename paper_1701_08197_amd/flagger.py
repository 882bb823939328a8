"""Thin Python wrapper of the LOF C ABI (names follow include/lof.h).

Torch is used for device memory and streams only: tensors hand their device
pointers to the library, which does all of the flagging on the GPU.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _native as N


class LofError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"LOF status {status}: {msg}")
        self.status = status


def default_params(**overrides) -> N.LofParams:
    """lof_default_params() with fields overridden by keyword."""
    L = N.load()
    p = N.LofParams()
    L.lof_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


@dataclass
class Block:
    """One time-frequency block: ``data`` is a device tensor of
    int8 [C, T, 2] (LOF_CI8), complex64 [C, T] (LOF_C64, LOF_C64_AMP) or float32
    [C, T] (LOF_F32); ``flags`` a uint8/bool device tensor [C, T]."""
    data: object
    flags: object
    dtype: int
    stream_id: int = -1

    def to_c(self) -> N.LofBlock:
        d, f = self.data, self.flags
        if self.dtype == N.LOF_CI8:
            if d.dim() != 3 or d.shape[2] != 2 or d.stride(2) != 1 or d.stride(1) != 2:
                raise ValueError("CI8 data must be int8 [C, T, 2] with interleaved (re, im)")
            C, T = d.shape[0], d.shape[1]
            rs = d.stride(0) // 2
        else:
            if d.dim() != 2 or d.stride(1) != 1:
                raise ValueError("data must be [C, T] with unit time stride")
            C, T = d.shape
            rs = d.stride(0)
        if f.dim() != 2 or tuple(f.shape) != (C, T) or f.stride(1) != 1 or f.element_size() != 1:
            raise ValueError("flags must be a 1-byte [C, T] tensor with unit time stride")
        b = N.LofBlock()
        b.data = d.data_ptr()
        b.flags = f.data_ptr()
        b.data_row_stride = rs
        b.flag_row_stride = f.stride(0)
        b.n_channels = C
        b.n_times = T
        b.dtype = self.dtype
        b.stream_id = self.stream_id
        return b


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Flagger:
    """Owns one lof_ctx (lof_create / lof_destroy)."""

    def __init__(self, params: N.LofParams | None = None, device: int = 0, **overrides):
        self._L = N.load()
        self.params = params if params is not None else default_params(**overrides)
        self.device = device
        h = ctypes.c_void_p()
        st = self._L.lof_create(ctypes.byref(self.params), device, ctypes.byref(h))
        if st != N.LOF_OK:
            raise LofError(st, self._L.lof_last_error(None).decode())
        self._h = h

    def _check(self, st: int):
        if st != N.LOF_OK:
            raise LofError(st, self._L.lof_last_error(self._h).decode())

    def flag_blocks(self, blocks, stream=None, stats=None) -> None:
        """lof_flag_blocks: ``blocks`` a list of Block (or LofBlock); ``stats`` an
        optional device uint8 tensor of len(blocks) * STATS_BYTES bytes."""
        n = len(blocks)
        arr = (N.LofBlock * max(1, n))()
        for i, b in enumerate(blocks):
            arr[i] = b if isinstance(b, N.LofBlock) else b.to_c()
        sp = None if stats is None else stats.data_ptr()
        self._check(self._L.lof_flag_blocks(self._h, arr, n, _stream_handle(stream), sp))

    def flag_blocks_raw(self, arr, n: int, stream=None, stats_ptr=None) -> int:
        """lof_flag_blocks on a prebuilt ctypes LofBlock array; returns the status."""
        return self._L.lof_flag_blocks(self._h, arr, n, _stream_handle(stream), stats_ptr)

    def history_update(self, stream_ids=None, stream=None) -> None:
        if stream_ids is None:
            self._check(self._L.lof_history_update(self._h, None, 0, _stream_handle(stream)))
            return
        ids = list(stream_ids)
        arr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
        self._check(self._L.lof_history_update(self._h, arr, len(ids), _stream_handle(stream)))

    def history_export(self, stream=None):
        import numpy as np
        p = self.params
        S, C, H = p.max_streams, p.max_channels, p.history_len
        vals = np.zeros((S, C, H), dtype=np.float64)
        cnt = np.zeros((S, C), dtype=np.int32)
        staged = np.zeros((S, C), dtype=np.float64)
        valid = np.zeros((S, C), dtype=np.uint8)
        self._check(self._L.lof_history_export(
            self._h, vals.ctypes.data, cnt.ctypes.data, staged.ctypes.data, valid.ctypes.data,
            _stream_handle(stream)))
        return {"values": vals, "counts": cnt, "staged": staged, "staged_valid": valid}

    def get_tuning(self) -> N.LofTuning:
        t = N.LofTuning()
        self._check(self._L.lof_get_tuning(self._h, ctypes.byref(t)))
        return t

    def set_tuning(self, t: N.LofTuning) -> None:
        self._check(self._L.lof_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, blocks, stream=None, reps: int = 3) -> N.LofTuning:
        """lof_autotune on a list of Block (or LofBlock); returns the chosen tuning."""
        n = len(blocks)
        arr = (N.LofBlock * max(1, n))()
        for i, b in enumerate(blocks):
            arr[i] = b if isinstance(b, N.LofBlock) else b.to_c()
        t = N.LofTuning()
        self._check(self._L.lof_autotune(self._h, arr, n, _stream_handle(stream), reps, ctypes.byref(t)))
        return t

    def autotune_raw(self, arr, n: int, stream=None, reps: int = 3) -> N.LofTuning:
        """lof_autotune on a ctypes lof_block array of n entries."""
        t = N.LofTuning()
        self._check(self._L.lof_autotune(self._h, arr, n, _stream_handle(stream), reps, ctypes.byref(t)))
        return t

    def phase_times(self):
        """lof_phase_times: per-phase kernel milliseconds summed over the calls
        since the previous read, and the number of calls (needs
        LOF_OPT_PHASE_TIMING in the params' options)."""
        arr = (ctypes.c_double * N.LOF_N_PHASES)()
        n = ctypes.c_int32()
        self._check(self._L.lof_phase_times(self._h, arr, ctypes.byref(n)))
        return {name: float(arr[i]) for i, name in enumerate(N.PHASES)}, int(n.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._L.lof_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flag_blocks_static(params: N.LofParams, blocks, device: int = 0, stream=None, stats=None) -> None:
    """lof_flag_blocks_static: flags ``blocks`` (Block or LofBlock, stream ids -1)
    with the library's own static scratch; nothing is allocated."""
    L = N.load()
    n = len(blocks)
    arr = (N.LofBlock * max(1, n))()
    for i, b in enumerate(blocks):
        arr[i] = b if isinstance(b, N.LofBlock) else b.to_c()
    sp = None if stats is None else stats.data_ptr()
    st = L.lof_flag_blocks_static(ctypes.byref(params), device, arr, n, _stream_handle(stream), sp)
    if st != N.LOF_OK:
        raise LofError(st, L.lof_last_error(None).decode())


def decode_stats(raw_bytes) -> list:
    """Decode a host copy of the stats buffer into dicts."""
    n = len(raw_bytes) // N.STATS_BYTES
    out = []
    buf = bytes(raw_bytes)
    for i in range(n):
        s = N.LofBlockStats.from_buffer_copy(buf[i * N.STATS_BYTES:(i + 1) * N.STATS_BYTES])
        out.append({"median": s.median, "stddev": s.stddev, "threshold": list(s.threshold),
                    "n_flagged": s.n_flagged, "history_flagged_rows": s.history_flagged_rows})
    return out
