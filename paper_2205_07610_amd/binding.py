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
N_FEATURES = 32
MLP_PARAMS = 6337
BAND_WIDE = 1024

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
                ("features_ms", ctypes.c_float), ("mlp_ms", ctypes.c_float),
                ("band16_ms", ctypes.c_float), ("long16_ms", ctypes.c_float),
                ("pairs_full32", ctypes.c_int64), ("pairs_full16", ctypes.c_int64),
                ("pairs_rerun32", ctypes.c_int64), ("pairs_long", ctypes.c_int64),
                ("pairs_fallback", ctypes.c_int64), ("cells", ctypes.c_int64),
                ("cells_full32", ctypes.c_int64), ("cells_full16", ctypes.c_int64),
                ("cells_long", ctypes.c_int64), ("pairs_long16", ctypes.c_int64),
                ("cells_long16", ctypes.c_int64), ("full16_cell_type", ctypes.c_int64),
                ("full32_variants", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BandStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("accepted", ctypes.c_int64 * 8), ("fallback", ctypes.c_int64),
                ("band_cells", ctypes.c_int64), ("cells", ctypes.c_int64),
                ("fallback_cells", ctypes.c_int64), ("band16_cells", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"rounds": self.rounds, "accepted": list(self.accepted)[:max(self.rounds, 1)],
                "fallback": self.fallback, "band_cells": self.band_cells, "cells": self.cells,
                "fallback_cells": self.fallback_cells, "band16_cells": self.band16_cells,
                "dp_cells": self.band_cells + self.fallback_cells}


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
    L.as_align_batch_noalloc.restype = ctypes.c_int
    L.as_align_batch_noalloc.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p]
    L.as_align_batch_traceback.restype = ctypes.c_int
    L.as_align_batch_traceback.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p, p, p]
    L.as_set_traceback_base.restype = ctypes.c_int
    L.as_set_traceback_base.argtypes = [i32]
    L.as_band_model_blob_size.restype = i64
    L.as_band_model_blob_size.argtypes = [i32]
    L.as_band_model_save.restype = ctypes.c_int
    L.as_band_model_save.argtypes = [p, p, p, i64, p, i64, ctypes.POINTER(ctypes.c_int64), p]
    L.as_band_model_load.restype = ctypes.c_int
    L.as_band_model_load.argtypes = [p, i64, p, p, p, ctypes.POINTER(ctypes.c_int64), p]
    L.as_align_all_vs_all.restype = ctypes.c_int
    L.as_align_all_vs_all.argtypes = [p, p, i64, p, p, i64, ctypes.POINTER(Scoring), i32, p, p]
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
    L.as_band_certify.restype = ctypes.c_int
    L.as_band_certify.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p, p, p]
    L.as_pair_features.restype = ctypes.c_int
    L.as_pair_features.argtypes = [p, p, p, p, i64, p, p]
    L.as_band_predict.restype = ctypes.c_int
    L.as_band_predict.argtypes = [p, p, i64, p, p, p]
    L.as_band_labels.restype = ctypes.c_int
    L.as_band_labels.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p]
    L.as_band_train.restype = ctypes.c_int
    L.as_band_train.argtypes = [p, p, p, p, p, i64, p, i32, i32, i32, ctypes.c_float,
                                ctypes.c_float, p, p]
    L.as_train_band_model.restype = ctypes.c_int
    L.as_train_band_model.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, p, i32,
                                      i32, ctypes.c_float, ctypes.c_float, p]
    L.as_align_batch_learned.restype = ctypes.c_int
    L.as_align_batch_learned.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p, i32, p,
                                         ctypes.POINTER(BandStats), p]
    L.as_plan_create.restype = ctypes.c_int
    L.as_plan_create.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, p,
                                 ctypes.POINTER(ctypes.c_void_p), p]
    L.as_plan_run.restype = ctypes.c_int
    L.as_plan_run.argtypes = [p, p]
    L.as_plan_destroy.restype = ctypes.c_int
    L.as_plan_destroy.argtypes = [p]
    L.as_set_band_packing.restype = ctypes.c_int
    L.as_set_band_packing.argtypes = [i32]
    L.as_set_variants.restype = ctypes.c_int
    L.as_set_variants.argtypes = [i32, p]
    L.as_get_variants.restype = ctypes.c_int
    L.as_get_variants.argtypes = [i32, p]
    L.as_autotune.restype = ctypes.c_int
    L.as_autotune.argtypes = [p, p, p, p, i64, ctypes.POINTER(Scoring), i32, i32, p, p, p]
    L.as_set_i16_limit.restype = ctypes.c_int
    L.as_set_i16_limit.argtypes = [ctypes.c_int32]
    L.as_set_half_cells.restype = ctypes.c_int
    L.as_set_half_cells.argtypes = [ctypes.c_int]
    L.as_half_cells_preference.restype = ctypes.c_int
    L.as_half_cells_preference.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.as_variant_tables_blob_size.restype = i64
    L.as_variant_tables_blob_size.argtypes = []
    L.as_variant_tables_save.restype = ctypes.c_int
    L.as_variant_tables_save.argtypes = [p, i64]
    L.as_variant_tables_load.restype = ctypes.c_int
    L.as_variant_tables_load.argtypes = [p, i64]
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
    return _align_full(lib().as_align_batch, seqs_a, offs_a, seqs_b, offs_b, subst, alpha, beta,
                       mode, scores_out, stream)


def align_batch_noalloc(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                        scores_out, stream=None):
    """align_batch through as_align_batch_noalloc (the library allocates
    nothing; scores_out must be given)."""
    return _align_full(lib().as_align_batch_noalloc, seqs_a, offs_a, seqs_b, offs_b, subst, alpha,
                       beta, mode, scores_out, stream)


def _align_full(fn, seqs_a, offs_a, seqs_b, offs_b, subst, alpha, beta, mode, scores_out, stream):
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
    rc = fn(pa, _dev_ptr(offs_a, torch.int64, "offs_a"),
            pb, _dev_ptr(offs_b, torch.int64, "offs_b"),
            n_pairs, ctypes.byref(sc), int(mode),
            _dev_ptr(scores_out, torch.int32, "scores_out")
            if n_pairs > 0 else ctypes.c_void_p(offs_a.data_ptr()),
            ctypes.c_void_p(stream))
    del keep
    _check(rc)
    return scores_out


def align_batch_traceback(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                          stream=None):
    """Scores and one optimal alignment per pair: (scores int32 [n], ops uint8
    [sum of m + n], span int32 [n, 5] = (n_ops, a0, a1, b0, b1)), device
    tensors; pair p's columns start at (offs_a[p] - offs_a[0]) + (offs_b[p] - offs_b[0])."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    total = int((offs_a[-1] - offs_a[0] + offs_b[-1] - offs_b[0]).item()) if n_pairs > 0 else 0
    scores = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    ops = torch.zeros(max(total, 1), dtype=torch.uint8, device=dev)
    span = torch.zeros((max(n_pairs, 1), 5), dtype=torch.int32, device=dev)
    sc, keep = make_scoring(subst, alpha, beta)
    rc = lib().as_align_batch_traceback(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                                        ctypes.byref(sc), int(mode),
                                        _dev_ptr(scores, torch.int32, "scores_out"),
                                        _dev_ptr(ops, torch.uint8, "ops_out"),
                                        _dev_ptr(span, torch.int32, "span_out"),
                                        ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return scores[:n_pairs], ops, span[:n_pairs]


def set_traceback_base(cells: int) -> int:
    """Explicit-predecessor limit of the traceback in cells (test hook; <= 0 resets)."""
    return int(lib().as_set_traceback_base(int(cells)))


def align_all_vs_all(seqs_q, offs_q, seqs_s, offs_s, subst, alpha: int, beta: int, mode: int,
                     scores_out=None, stream=None):
    """Scores of every query against every subject: int32 device tensor [n_q, n_s]."""
    import torch
    n_q, n_s = offs_q.numel() - 1, offs_s.numel() - 1
    dev = offs_q.device
    if scores_out is None:
        scores_out = torch.empty((max(n_q, 1), max(n_s, 1)), dtype=torch.int32, device=dev)
    sc, keep = make_scoring(subst, alpha, beta)
    pq = _dev_ptr(seqs_q, torch.uint8, "seqs_q") if seqs_q.numel() else ctypes.c_void_p(offs_q.data_ptr())
    ps = _dev_ptr(seqs_s, torch.uint8, "seqs_s") if seqs_s.numel() else ctypes.c_void_p(offs_s.data_ptr())
    rc = lib().as_align_all_vs_all(pq, _dev_ptr(offs_q, torch.int64, "offs_q"), n_q,
                                   ps, _dev_ptr(offs_s, torch.int64, "offs_s"), n_s,
                                   ctypes.byref(sc), int(mode), _dev_ptr(scores_out, torch.int32, "scores_out"),
                                   ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return scores_out[:n_q, :n_s]


def set_band_packing(on: bool) -> bool:
    """Packed 16-bit banded kernel for eligible global pairs (default on)."""
    return bool(lib().as_set_band_packing(1 if on else 0))


def set_i16_limit(limit: int) -> int:
    """Saturation threshold of the 16-bit local path (test hook; <= 0 resets)."""
    return int(lib().as_set_i16_limit(int(limit)))


def set_half_cells(mode: int) -> int:
    """Cell type of the packed full-DP kernel: 0 int16, 1 FP16 whenever the
    scoring admits it, 2 automatic (the default).  Returns the previous mode."""
    return int(lib().as_set_half_cells(int(mode)))


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


def _stream(dev, stream):
    import torch
    return torch.cuda.current_stream(dev).cuda_stream if stream is None else stream


def band_certify(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int, band_w,
                 stream=None):
    """Exact-band scores and certificate flags (device int32 tensors)."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    out = torch.zeros(max(n_pairs, 1), dtype=torch.int32, device=dev)
    acc = torch.zeros(max(n_pairs, 1), dtype=torch.int32, device=dev)
    sc, keep = make_scoring(subst, alpha, beta)
    rc = lib().as_band_certify(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                               ctypes.byref(sc), int(mode), _dev_ptr(band_w, torch.int32, "band_w"),
                               _dev_ptr(out, torch.int32, "scores_out"),
                               _dev_ptr(acc, torch.int32, "accept_out"),
                               ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return out[:n_pairs], acc[:n_pairs]


def pair_features(seqs_a, offs_a, seqs_b, offs_b, out=None, stream=None):
    """k-mer diagonal features, float32 device tensor [n_pairs, 32]."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    if out is None:
        out = torch.empty((max(n_pairs, 1), N_FEATURES), dtype=torch.float32, device=dev)
    _check(lib().as_pair_features(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                                  _dev_ptr(out, torch.float32, "features_out"),
                                  ctypes.c_void_p(_stream(dev, stream))))
    return out[:n_pairs]


def band_predict(params, features, with_y: bool = False, stream=None):
    """Predicted half-widths (int32) and optionally the network outputs y (float32)."""
    import torch
    n = features.shape[0]
    dev = features.device
    w = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    y = torch.empty(max(n, 1), dtype=torch.float32, device=dev) if with_y else None
    _check(lib().as_band_predict(_dev_ptr(params, torch.float32, "params"),
                                 _dev_ptr(features, torch.float32, "features"), n,
                                 _dev_ptr(w, torch.int32, "band_w_out"),
                                 _dev_ptr(y, torch.float32, "y_out") if with_y else None,
                                 ctypes.c_void_p(_stream(dev, stream))))
    return (w[:n], y[:n]) if with_y else w[:n]


def band_labels(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                stream=None):
    """Band labels from the full DP (int32 device tensor)."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    out = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    sc, keep = make_scoring(subst, alpha, beta)
    rc = lib().as_band_labels(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                              ctypes.byref(sc), int(mode), _dev_ptr(out, torch.int32, "labels_out"),
                              ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return out[:n_pairs]


def band_train(params, adam_m, adam_v, features, labels, order, n_steps: int, batch: int,
               t0: int = 1, lr: float = 1e-3, tau: float = 0.85, grads_out=None, stream=None):
    """Adam steps on the network (params, adam_m, adam_v updated in place)."""
    import torch
    dev = params.device
    _check(lib().as_band_train(_dev_ptr(params, torch.float32, "params"),
                               _dev_ptr(adam_m, torch.float32, "adam_m"),
                               _dev_ptr(adam_v, torch.float32, "adam_v"),
                               _dev_ptr(features, torch.float32, "features"),
                               _dev_ptr(labels, torch.int32, "labels"), labels.numel(),
                               _dev_ptr(order, torch.int32, "order"), int(n_steps), int(batch),
                               int(t0), float(lr), float(tau),
                               _dev_ptr(grads_out, torch.float32, "grads_out")
                               if grads_out is not None else None,
                               ctypes.c_void_p(_stream(dev, stream))))
    return params


def train_band_model(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                     params, order, n_steps: int, batch: int, lr: float = 1e-3, tau: float = 0.85,
                     stream=None):
    """Features, labels and training in one library call (params updated in place)."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    sc, keep = make_scoring(subst, alpha, beta)
    rc = lib().as_train_band_model(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                                   ctypes.byref(sc), int(mode),
                                   _dev_ptr(params, torch.float32, "params"),
                                   _dev_ptr(order, torch.int32, "order"), int(n_steps), int(batch),
                                   float(lr), float(tau), ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return params


def align_batch_learned(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                        params, max_rounds: int = 6, scores_out=None, stream=None):
    """Learned-band alignment (exact scores); returns (scores, stats dict)."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    if scores_out is None:
        scores_out = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    sc, keep = make_scoring(subst, alpha, beta)
    st = BandStats()
    rc = lib().as_align_batch_learned(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                                      ctypes.byref(sc), int(mode),
                                      _dev_ptr(params, torch.float32, "params"), int(max_rounds),
                                      _dev_ptr(scores_out, torch.int32, "scores_out"),
                                      ctypes.byref(st), ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return scores_out[:n_pairs], st.as_dict()


def band_model_save(params, adam_m=None, adam_v=None, adam_t: int = 0, stream=None) -> bytes:
    """Versioned blob of the band network (and its Adam state when given)."""
    import torch
    with_adam = adam_m is not None
    size = int(lib().as_band_model_blob_size(1 if with_adam else 0))
    buf = ctypes.create_string_buffer(size)
    got = ctypes.c_int64(0)
    _check(lib().as_band_model_save(_dev_ptr(params, torch.float32, "params"),
                                    _dev_ptr(adam_m, torch.float32, "adam_m") if with_adam else None,
                                    _dev_ptr(adam_v, torch.float32, "adam_v") if with_adam else None,
                                    int(adam_t), buf, size, ctypes.byref(got),
                                    ctypes.c_void_p(_stream(params.device, stream))))
    return buf.raw[:got.value]


def band_model_load(blob: bytes, params_out, adam_m_out=None, adam_v_out=None, stream=None) -> int:
    """Fill device tensors from a blob; returns the stored Adam step counter."""
    import torch
    with_adam = adam_m_out is not None
    t = ctypes.c_int64(0)
    raw = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib().as_band_model_load(raw, len(blob), _dev_ptr(params_out, torch.float32, "params_out"),
                                    _dev_ptr(adam_m_out, torch.float32, "adam_m_out") if with_adam else None,
                                    _dev_ptr(adam_v_out, torch.float32, "adam_v_out") if with_adam else None,
                                    ctypes.byref(t), ctypes.c_void_p(_stream(params_out.device, stream))))
    return int(t.value)


class Plan:
    """A batch captured as a replayable HIP graph (as_plan_*).  Keeps the
    device tensors it was made from alive; run() replays and raises on error."""

    def __init__(self, seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
                 scores_out=None, stream=None):
        import torch
        n_pairs = offs_a.numel() - 1
        dev = offs_a.device
        self.scores = scores_out if scores_out is not None else \
            torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
        self._keep = (seqs_a, offs_a, seqs_b, offs_b)
        self._dev = dev
        sc, keep = make_scoring(subst, alpha, beta)
        h = ctypes.c_void_p()
        rc = lib().as_plan_create(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs,
                                  ctypes.byref(sc), int(mode),
                                  _dev_ptr(self.scores, torch.int32, "scores_out"), ctypes.byref(h),
                                  ctypes.c_void_p(_stream(dev, stream)))
        del keep
        _check(rc)
        self._h = h
        self.n_pairs = n_pairs

    def run(self, stream=None):
        _check(lib().as_plan_run(self._h, ctypes.c_void_p(_stream(self._dev, stream))))
        return self.scores[:self.n_pairs]

    def close(self):
        if getattr(self, "_h", None):
            lib().as_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LEN_BINS = 12
VARIANTS = {"auto": -1, "packed16": 0, "k8": 1, "k16": 2, "k32": 3, "wavefront": 4, "packed_lds": 5}
N_VARIANTS = 6


def set_variants(mode: int, table=None):
    """Full-DP variant per length bin for a mode (None: all automatic)."""
    if table is None:
        _check(lib().as_set_variants(int(mode), None))
        return
    t = np.ascontiguousarray(np.asarray(table, dtype=np.int8))
    if t.shape != (LEN_BINS,):
        raise ValueError(f"table must have {LEN_BINS} entries")
    _check(lib().as_set_variants(int(mode), t.ctypes.data_as(ctypes.c_void_p)))


def get_variants(mode: int) -> np.ndarray:
    t = np.zeros(LEN_BINS, dtype=np.int8)
    _check(lib().as_get_variants(int(mode), t.ctypes.data_as(ctypes.c_void_p)))
    return t


def half_cells_preference(mode: int, pref=None) -> int:
    """The automatic setting's measured cell type for a mode (-1 none, 0
    int16, 1 FP16; as_autotune sets it).  With pref given, store it.
    Returns the previous value."""
    rc = int(lib().as_half_cells_preference(int(mode), 0 if pref is None else int(pref),
                                             0 if pref is None else 1))
    if rc < -1:
        _check(rc)
    return rc


def variant_tables_save() -> bytes:
    """The three modes' variant tables as a versioned blob (for a file)."""
    n = int(lib().as_variant_tables_blob_size())
    buf = ctypes.create_string_buffer(n)
    _check(lib().as_variant_tables_save(ctypes.cast(buf, ctypes.c_void_p), n))
    return buf.raw


def variant_tables_load(blob: bytes):
    """Replace the three modes' variant tables from a saved blob."""
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib().as_variant_tables_load(ctypes.cast(buf, ctypes.c_void_p), len(blob)))


def autotune(seqs_a, offs_a, seqs_b, offs_b, subst, alpha: int, beta: int, mode: int,
             sample_pairs: int = 8192, stream=None):
    """Run the autotuner; returns (table int8 [12], gcups float [12, N_VARIANTS])."""
    import torch
    n_pairs = offs_a.numel() - 1
    dev = offs_a.device
    sc, keep = make_scoring(subst, alpha, beta)
    g = np.zeros(LEN_BINS * N_VARIANTS, dtype=np.float32)
    t = np.zeros(LEN_BINS, dtype=np.int8)
    rc = lib().as_autotune(*_seq_ptrs(seqs_a, offs_a, seqs_b, offs_b), n_pairs, ctypes.byref(sc),
                           int(mode), int(sample_pairs), g.ctypes.data_as(ctypes.c_void_p),
                           t.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(_stream(dev, stream)))
    del keep
    _check(rc)
    return t, g.reshape(LEN_BINS, N_VARIANTS)


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
