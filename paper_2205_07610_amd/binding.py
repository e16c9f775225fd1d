"""ctypes binding of libanyseq_mi.so (argument marshalling only).

Every step of the alignment runs inside the HIP library; this module only
turns torch device tensors into pointers, the host scoring matrix into the
ABI struct, and return codes into exceptions.  It never falls back to any
other implementation: if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libanyseq_mi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "anyseq_mi.h")

GLOBAL, SEMIGLOBAL, LOCAL = 0, 1, 2

_lib = None


class Scoring(ctypes.Structure):
    _fields_ = [("alphabet_size", ctypes.c_int32),
                ("subst", ctypes.c_void_p),
                ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("classify_ms", ctypes.c_float), ("full32_ms", ctypes.c_float),
                ("full16_ms", ctypes.c_float), ("rerun32_ms", ctypes.c_float),
                ("long_ms", ctypes.c_float), ("band_ms", ctypes.c_float),
                ("reserved_ms", ctypes.c_float * 2),
                ("pairs_full32", ctypes.c_int64), ("pairs_full16", ctypes.c_int64),
                ("pairs_rerun32", ctypes.c_int64), ("pairs_long", ctypes.c_int64),
                ("pairs_fallback", ctypes.c_int64), ("cells", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved_ms"}


class BandStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("accepted", ctypes.c_int64 * 8), ("fallback", ctypes.c_int64),
                ("band_cells", ctypes.c_int64), ("cells", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"rounds": self.rounds, "accepted": list(self.accepted)[:max(self.rounds, 1)],
                "fallback": self.fallback, "band_cells": self.band_cells, "cells": self.cells}


class AlignError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"anyseq_mi error {code}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2205_07610_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.as_align_batch.restype = ctypes.c_int
    L.as_align_batch.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p]
    L.as_strerror.restype = ctypes.c_char_p
    L.as_strerror.argtypes = [ctypes.c_int]
    L.as_release_workspace.restype = ctypes.c_int
    L.as_release_workspace.argtypes = []
    L.as_build_info.restype = ctypes.c_char_p
    L.as_build_info.argtypes = []
    L.as_align_batch_band.restype = ctypes.c_int
    L.as_align_batch_band.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, i32, p,
                                      ctypes.POINTER(BandStats), p]
    L.as_band_scores.restype = ctypes.c_int
    L.as_band_scores.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p, p, p, p]
    L.as_set_i16_limit.restype = ctypes.c_int
    L.as_set_i16_limit.argtypes = [ctypes.c_int32]
    L.as_enable_timing.restype = ctypes.c_int
    L.as_enable_timing.argtypes = [ctypes.c_int]
    L.as_last_timing.restype = ctypes.c_int
    L.as_last_timing.argtypes = [ctypes.POINTER(Timing)]
    _lib = L
    return L


def declared_functions() -> list[str]:
    """Names of the functions include/anyseq_mi.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(as_[a-z_0-9]+)\s*\(", text, flags=re.M)


def strerror(code: int) -> str:
    return lib().as_strerror(code).decode()


def _check(code: int):
    if code != 0:
        raise AlignError(code, strerror(code))


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def make_scoring(subst, alpha: int, beta: int):
    s = np.ascontiguousarray(np.asarray(subst, dtype=np.int8))
    sc = Scoring(s.shape[0], s.ctypes.data_as(ctypes.c_void_p), int(alpha), int(beta))
    return sc, s  # keep s alive while sc is used


def align_batch(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                scores_out=None, stream=None):
    """Scores of every pair (device tensors in, int32 device tensor out).

    seqs_*: uint8 CUDA tensors of residue codes; offs_*: int64 CUDA tensors
    [n_pairs + 1]; subst: host [asz, asz] int8 matrix; mode: 0 global,
    1 semi-global, 2 local.  Raises AlignError on a non-zero return code."""
    import torch
    n_pairs = offs_a.numel() - 1
    if offs_b.numel() != n_pairs + 1:
        raise ValueError("offs_a and offs_b must have the same length")
    if scores_out is None:
        scores_out = torch.empty(max(n_pairs, 0), dtype=torch.int32, device=offs_a.device)
    sc, keep = make_scoring(subst, alpha, beta)
    if stream is None:
        stream = torch.cuda.current_stream(offs_a.device).cuda_stream
    # an empty uint8 tensor still needs a non-null pointer for the ABI's checks
    pa = _dev_ptr(seqs_a, torch.uint8, "seqs_a") if seqs_a.numel() else ctypes.c_void_p(offs_a.data_ptr())
    pb = _dev_ptr(seqs_b, torch.uint8, "seqs_b") if seqs_b.numel() else ctypes.c_void_p(offs_b.data_ptr())
    rc = lib().as_align_batch(pa, _dev_ptr(offs_a, torch.int64, "offs_a"),
                              pb, _dev_ptr(offs_b, torch.int64, "offs_b"),
                              n_pairs, ctypes.byref(sc), int(mode),
                              _dev_ptr(scores_out, torch.int32, "scores_out")
                              if n_pairs > 0 else ctypes.c_void_p(offs_a.data_ptr()),
                              ctypes.c_void_p(stream))
    del keep
    _check(rc)
    return scores_out


def set_i16_limit(limit: int) -> int:
    """Saturation threshold of the 16-bit local path (test hook; <= 0 resets)."""
    return int(lib().as_set_i16_limit(int(limit)))


def _seq_ptrs(seqs_a, offs_a, seqs_b, offs_b):
    import torch
    pa = _dev_ptr(seqs_a, torch.uint8, "seqs_a") if seqs_a.numel() else ctypes.c_void_p(offs_a.data_ptr())
    pb = _dev_ptr(seqs_b, torch.uint8, "seqs_b") if seqs_b.numel() else ctypes.c_void_p(offs_b.data_ptr())
    return (pa, _dev_ptr(offs_a, torch.int64, "offs_a"), pb, _dev_ptr(offs_b, torch.int64, "offs_b"))


def align_batch_band(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                     band_w0, max_rounds: int = 6, scores_out=None, stream=None):
    """Certified banded alignment (exact scores); returns (scores, stats dict)."""
    import torch
    n_pairs = offs_a.numel() - 1
    if scores_out is None:
        scores_out = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=offs_a.device)
    sc, keep = make_scoring(subst, alpha, beta)
    if stream is None:
        stream = torch.cuda.current_stream(offs_a.device).cuda_stream
    st = BandStats()
    rc = lib().as_align_batch_band(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                                   ctypes.byref(sc), int(mode),
                                   _dev_ptr(band_w0, torch.int32, "band_w0"), int(max_rounds),
                                   _dev_ptr(scores_out, torch.int32, "scores_out"),
                                   ctypes.byref(st), ctypes.c_void_p(stream))
    del keep
    _check(rc)
    return scores_out[:n_pairs], st.as_dict()


def band_scores(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int, band_w,
                stream=None):
    """Raw banded scores and the diagonal limits computed (lo, hi), device tensors."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    out = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    lo = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    hi = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    sc, keep = make_scoring(subst, alpha, beta)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib().as_band_scores(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                              ctypes.byref(sc), int(mode), _dev_ptr(band_w, torch.int32, "band_w"),
                              _dev_ptr(out, torch.int32, "scores_out"),
                              _dev_ptr(lo, torch.int32, "lo_out"), _dev_ptr(hi, torch.int32, "hi_out"),
                              ctypes.c_void_p(stream))
    del keep
    _check(rc)
    return out[:n_pairs], lo[:n_pairs], hi[:n_pairs]


def enable_timing(on: bool = True) -> bool:
    return bool(lib().as_enable_timing(1 if on else 0))


def last_timing() -> dict:
    t = Timing()
    _check(lib().as_last_timing(ctypes.byref(t)))
    return t.as_dict()


def to_device(batch, device="cuda"):
    """Copy a synth.Batch's arrays to device tensors (seqs_a, offs_a, seqs_b, offs_b)."""
    import torch
    return (torch.from_numpy(np.ascontiguousarray(batch.seqs_a)).to(device),
            torch.from_numpy(np.ascontiguousarray(batch.offs_a)).to(device),
            torch.from_numpy(np.ascontiguousarray(batch.seqs_b)).to(device),
            torch.from_numpy(np.ascontiguousarray(batch.offs_b)).to(device))


def align(batch, device="cuda"):
    """Convenience: align a synth.Batch, return numpy int32 scores."""
    sa, oa, sb, ob = to_device(batch, device)
    out = align_batch(sa, oa, sb, ob, batch.subst, batch.alpha, batch.beta, batch.mode)
    return out.cpu().numpy()
