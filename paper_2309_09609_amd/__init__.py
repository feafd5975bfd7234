"""MI355X Smith-Waterman protein database search: thin Python binding of libswsearch.

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  Device buffers are torch tensors on the GPU, streams are torch
streams.  The functions mirror the C ABI in include/swsearch.h
(``sw_db_pack``, ``sw_search``, ``sw_topk``, ``sw_search_batch``) and
``Database`` wraps a packed handle.

The library must have been built (``python -m paper_2309_09609_amd.build`` or
``__graft_entry__.build()``); loading raises if it is missing.  There is no
CPU fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswsearch.so")

SW_OK = 0
STATUS = {0: "SW_OK", -1: "SW_E_INVALID", -2: "SW_E_RESIDUE", -3: "SW_E_NOMEM", -4: "SW_E_HIP",
          -5: "SW_E_UNSUPPORTED", -6: "SW_E_SIZE"}

# Every entry point declared in include/swsearch.h.
EXPORTS = ("sw_db_pack", "sw_db_pack_bytes", "sw_db_pack_into", "sw_search_ws", "sw_batch_workspace_bytes",
           "sw_search_batch_ws", "sw_pair_workspace_bytes", "sw_pair", "sw_db_tune", "sw_db_free", "sw_db_info", "sw_search", "sw_topk", "sw_search_batch",
           "sw_search_multi", "sw_align", "sw_align_batch", "sw_search_mode", "sw_topk_ws_bytes", "sw_topk_ws", "sw_topk_noalloc",
           "sw_status_str", "sw_last_error", "sw_last_stats", "sw_profile_kernels", "sw_kernel_times")

_lib = None


class SwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libswsearch.so (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.sw_db_pack.restype = I32
    lib.sw_db_pack.argtypes = [P, P, I64, P, P, ctypes.POINTER(P)]
    lib.sw_db_pack_bytes.restype = I32
    lib.sw_db_pack_bytes.argtypes = [P, I64, P, P]
    lib.sw_db_pack_into.restype = I32
    lib.sw_db_pack_into.argtypes = [P, P, I64, P, P, I64, P, ctypes.POINTER(P)]
    lib.sw_search_ws.restype = I32
    lib.sw_search_ws.argtypes = [P, I32, P, P, I64, P, I32, I32, P, P, I64, P]
    lib.sw_batch_workspace_bytes.restype = I32
    lib.sw_batch_workspace_bytes.argtypes = [P, P, I32, I32, I32, P]
    lib.sw_search_batch_ws.restype = I32
    lib.sw_search_batch_ws.argtypes = [P, P, I32, P, P, I32, I32, I32, P, P, P, P, I64, P]
    lib.sw_pair_workspace_bytes.restype = I32
    lib.sw_pair_workspace_bytes.argtypes = [I64, I64, P]
    lib.sw_pair.restype = I32
    lib.sw_pair.argtypes = [P, I64, P, I64, I32, P, I32, I32, P, P, I64, P]
    lib.sw_db_tune.restype = I32
    lib.sw_db_tune.argtypes = [P, P]
    lib.sw_db_free.restype = None
    lib.sw_db_free.argtypes = [P]
    lib.sw_db_info.restype = I32
    lib.sw_db_info.argtypes = [P, P, P, P]
    lib.sw_search.restype = I32
    lib.sw_search.argtypes = [P, I32, P, P, I64, P, I32, I32, P, P]
    lib.sw_topk.restype = I32
    lib.sw_topk.argtypes = [P, I64, I32, P, P, P]
    lib.sw_search_batch.restype = I32
    lib.sw_search_batch.argtypes = [P, P, I32, P, P, I32, I32, I32, P, P, P, P]
    lib.sw_search_multi.restype = I32
    lib.sw_search_multi.argtypes = [P, P, I32, P, I32, P, P, I32, I32, P, P]
    lib.sw_topk_ws_bytes.restype = I32
    lib.sw_topk_ws_bytes.argtypes = [I64, I32, P]
    lib.sw_topk_ws.restype = I32
    lib.sw_topk_ws.argtypes = [P, I64, I32, P, P, P, I64, P]
    lib.sw_topk_noalloc.restype = I32
    lib.sw_topk_noalloc.argtypes = [P, I64, I32, P, P, P]
    lib.sw_search_mode.restype = I32
    lib.sw_search_mode.argtypes = [I32, P, I32, P, P, I64, P, I32, I32, P, P]
    lib.sw_align.restype = I32
    lib.sw_align.argtypes = [P, I32, P, P, I32, P, I32, I32, P, P, I64, P]
    lib.sw_align_batch.restype = I32
    lib.sw_align_batch.argtypes = [P, P, I32, P, P, P, P, I32, I32, P, P, I64, P]
    lib.sw_status_str.restype = ctypes.c_char_p
    lib.sw_status_str.argtypes = [I32]
    lib.sw_last_error.restype = ctypes.c_char_p
    lib.sw_last_error.argtypes = []
    lib.sw_last_stats.restype = I32
    lib.sw_last_stats.argtypes = [P, P]
    lib.sw_profile_kernels.restype = I32
    lib.sw_profile_kernels.argtypes = [P, I32]
    lib.sw_kernel_times.restype = I32
    lib.sw_kernel_times.argtypes = [P, P, I32, P]
    _lib = lib
    return lib


class Alignment(ctypes.Structure):
    """sw_alignment of include/swsearch.h."""
    _fields_ = [("score", ctypes.c_int32), ("q_begin", ctypes.c_int32), ("q_end", ctypes.c_int32),
                ("subject", ctypes.c_int64), ("s_begin", ctypes.c_int64), ("s_end", ctypes.c_int64),
                ("n_ops", ctypes.c_int64)]


def _check(status: int):
    if status != SW_OK:
        raise SwError(status, load().sw_last_error().decode())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host_i8(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int8))


def _host_i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _square(subst) -> np.ndarray:
    """Substitution matrix as flat int8, checked to be square (alphabet x alphabet, alphabet <= 24)."""
    sm = _host_i8(subst)
    a = int(round(np.sqrt(sm.size)))
    if sm.size == 0 or a * a != sm.size or a > 24 or (sm.ndim == 2 and sm.shape[0] != sm.shape[1]):
        raise ValueError("substitution matrix must be square, at most 24 x 24")
    return sm.reshape(-1)


def _ptr(a) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data if isinstance(a, np.ndarray) else a.data_ptr())


# --------------------------------------------------------------------------- C-ABI mirrors
class PackOpts(ctypes.Structure):
    _fields_ = [("max_qlen", ctypes.c_int32), ("force_lanes", ctypes.c_int32),
                ("rerun_threshold", ctypes.c_int32), ("rows_per_lane", ctypes.c_int32),
                ("unit_share", ctypes.c_int32), ("lane_pack", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("rerun_cap", ctypes.c_int32), ("poison", ctypes.c_int32), ("align_tiles", ctypes.c_int32)]


def sw_db_pack(d_residues, h_offsets, stream=None, force_lanes=0, rerun_threshold=0, rows_per_lane=0,
               unit_share=0, lane_pack=0, alphabet=0, rerun_cap=0, poison=0, align_tiles=0) -> ctypes.c_void_p:
    """Pack a database; ``d_residues`` is an int8 tensor on the GPU, ``h_offsets`` int64[n+1].
    ``alphabet`` is the residue alphabet size (0 = 20); ``force_lanes``, ``rerun_threshold``,
    ``rows_per_lane``, ``rerun_cap``, ``poison`` and ``align_tiles`` are tuning/test hooks (see sw_pack_opts)."""
    lib = load()
    offs = _host_i64(h_offsets)
    n = offs.size - 1
    h = ctypes.c_void_p()
    opts = PackOpts(0, int(force_lanes), int(rerun_threshold), int(rows_per_lane), int(unit_share), int(lane_pack),
                    int(alphabet), int(rerun_cap), int(poison), int(align_tiles))
    _check(lib.sw_db_pack(ctypes.c_void_p(d_residues.data_ptr()), _ptr(offs), n, ctypes.byref(opts),
                          _stream(stream), ctypes.byref(h)))
    return h


def sw_db_pack_bytes(h_offsets) -> int:
    """Device bytes of the packed image of a database with these offsets."""
    offs = _host_i64(h_offsets)
    out = ctypes.c_int64()
    _check(load().sw_db_pack_bytes(_ptr(offs), offs.size - 1, None, ctypes.byref(out)))
    return out.value


def sw_db_pack_into(d_residues, h_offsets, d_db, stream=None, force_lanes=0, rerun_threshold=0, rows_per_lane=0,
                    unit_share=0, lane_pack=0, alphabet=0, rerun_cap=0, poison=0, align_tiles=0) -> ctypes.c_void_p:
    """``sw_db_pack`` into ``d_db``, a caller-owned uint8 tensor of at least ``sw_db_pack_bytes`` bytes."""
    offs = _host_i64(h_offsets)
    h = ctypes.c_void_p()
    opts = PackOpts(0, int(force_lanes), int(rerun_threshold), int(rows_per_lane), int(unit_share), int(lane_pack),
                    int(alphabet), int(rerun_cap), int(poison), int(align_tiles))
    _check(load().sw_db_pack_into(ctypes.c_void_p(d_residues.data_ptr()), _ptr(offs), offs.size - 1,
                                  ctypes.byref(opts), _ptr(d_db), d_db.numel() * d_db.element_size(), _stream(stream),
                                  ctypes.byref(h)))
    return h


def sw_batch_workspace_bytes(handle, h_qoffsets, k=0, scores_in_ws=False) -> int:
    """Device bytes of the workspace of ``sw_search_ws`` (one query, k = 0) or ``sw_search_batch_ws``."""
    qo = _host_i64(h_qoffsets)
    out = ctypes.c_int64()
    _check(load().sw_batch_workspace_bytes(handle, _ptr(qo), qo.size - 1, int(k), 1 if scores_in_ws else 0,
                                           ctypes.byref(out)))
    return out.value


def sw_search_ws(query, handle, h_offsets, n, subst, gap_open, gap_extend, d_scores_out, d_ws, stream=None):
    lib = load()
    q = _host_i8(query)
    sm = _square(subst)
    offs = None if h_offsets is None else _host_i64(h_offsets)
    _check(lib.sw_search_ws(_ptr(q), q.size, handle, None if offs is None else _ptr(offs), int(n), _ptr(sm),
                            int(gap_open), int(gap_extend), ctypes.c_void_p(d_scores_out.data_ptr()), _ptr(d_ws),
                            d_ws.numel() * d_ws.element_size(), _stream(stream)))


def sw_search_batch_ws(h_queries, h_qoffsets, handle, subst, gap_open, gap_extend, k, d_scores, d_top_scores,
                       d_top_index, d_ws, stream=None):
    lib = load()
    q = _host_i8(h_queries)
    qo = _host_i64(h_qoffsets)
    sm = _square(subst)
    P = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
    _check(lib.sw_search_batch_ws(_ptr(q), _ptr(qo), qo.size - 1, handle, _ptr(sm), int(gap_open), int(gap_extend),
                                  int(k), P(d_scores), P(d_top_scores), P(d_top_index), _ptr(d_ws),
                                  d_ws.numel() * d_ws.element_size(), _stream(stream)))


def sw_pair_workspace_bytes(qlen, slen) -> int:
    out = ctypes.c_int64()
    _check(load().sw_pair_workspace_bytes(int(qlen), int(slen), ctypes.byref(out)))
    return out.value


def sw_pair(query, subject, subst, gap_open=10, gap_extend=2, alphabet=0, d_score=None, d_ws=None, stream=None):
    """Score of one (long) pair spread over the GPU; returns the device int32 score tensor [1].
    The workspace comes from torch unless ``d_ws`` is given."""
    import torch
    q, d = _host_i8(query), _host_i8(subject)
    sm = _square(subst)
    if d_score is None:
        d_score = torch.empty(1, dtype=torch.int32, device="cuda")
    if d_ws is None:
        need = sw_pair_workspace_bytes(q.size, d.size)
        d_ws = torch.empty(max(need, 1), dtype=torch.uint8, device=d_score.device)
    _check(load().sw_pair(_ptr(q), q.size, _ptr(d), d.size, int(alphabet), _ptr(sm), int(gap_open), int(gap_extend),
                          _ptr(d_score), _ptr(d_ws), d_ws.numel(), _stream(stream)))
    if stream is not None:
        d_ws.record_stream(stream)
    return d_score


def sw_search(query, handle, h_offsets, n, subst, gap_open, gap_extend, d_scores_out, stream=None):
    lib = load()
    q = _host_i8(query)
    sm = _square(subst)
    offs = None if h_offsets is None else _host_i64(h_offsets)
    _check(lib.sw_search(_ptr(q), q.size, handle, None if offs is None else _ptr(offs), int(n), _ptr(sm),
                         int(gap_open), int(gap_extend), ctypes.c_void_p(d_scores_out.data_ptr()), _stream(stream)))


def sw_topk(d_scores, n, k, d_top_scores, d_top_index, stream=None):
    _check(load().sw_topk(ctypes.c_void_p(d_scores.data_ptr()), int(n), int(k),
                          ctypes.c_void_p(d_top_scores.data_ptr()), ctypes.c_void_p(d_top_index.data_ptr()),
                          _stream(stream)))


def sw_topk_ws(d_scores, n, k, d_top_scores, d_top_index, d_workspace, ws_bytes, stream=None):
    _check(load().sw_topk_ws(_ptr(d_scores), int(n), int(k), _ptr(d_top_scores), _ptr(d_top_index),
                             None if d_workspace is None else _ptr(d_workspace), int(ws_bytes), _stream(stream)))


def sw_topk_ws_bytes(n, k) -> int:
    need = ctypes.c_int64()
    _check(load().sw_topk_ws_bytes(int(n), int(k), ctypes.byref(need)))
    return need.value


def sw_topk_noalloc(d_scores, n, k, d_top_scores, d_top_index, stream=None):
    """Top k of one score vector with no allocation (the library's fixed device array)."""
    _check(load().sw_topk_noalloc(_ptr(d_scores), int(n), int(k), _ptr(d_top_scores), _ptr(d_top_index),
                                  _stream(stream)))


def sw_search_batch(h_queries, h_qoffsets, handle, subst, gap_open, gap_extend, k, d_scores=None,
                    d_top_scores=None, d_top_index=None, stream=None):
    lib = load()
    q = _host_i8(h_queries)
    qo = _host_i64(h_qoffsets)
    sm = _square(subst)
    P = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
    _check(lib.sw_search_batch(_ptr(q), _ptr(qo), qo.size - 1, handle, _ptr(sm), int(gap_open), int(gap_extend),
                               int(k), P(d_scores), P(d_top_scores), P(d_top_index), _stream(stream)))


def sw_search_multi(h_queries, h_qoffsets, chunks, nchunks, handle, subst, gap_open, gap_extend, d_scores_list,
                    stream=None):
    """Each query scores one database chunk into its own score tensor (see the C header)."""
    lib = load()
    q = _host_i8(h_queries)
    qo = _host_i64(h_qoffsets)
    ch = np.ascontiguousarray(np.asarray(chunks, dtype=np.int32))
    sm = _square(subst)
    ptrs = (ctypes.c_void_p * max(len(d_scores_list), 1))(*[t.data_ptr() for t in d_scores_list])
    _check(lib.sw_search_multi(_ptr(q), _ptr(qo), qo.size - 1, _ptr(ch), int(nchunks), handle, _ptr(sm),
                               int(gap_open), int(gap_extend), ptrs, _stream(stream)))


# --------------------------------------------------------------------------- convenience layer
class Database:
    """A packed, device-resident protein database.

    ``memory="library"``: the handle allocates its image and search workspace.
    ``memory="torch"``: torch allocates both (the image through
    ``sw_db_pack_into``, workspaces for ``sw_search_ws`` / ``sw_search_batch_ws``);
    the handle then holds no device memory of its own (global and semi-global
    searches and alignments still use the handle's).  Searches through one
    Database share its workspace: queue them on one stream, or let one finish
    before starting the next on another stream."""

    def __init__(self, residues, offsets, device="cuda", stream=None, force_lanes=0, rerun_threshold=0,
                 rows_per_lane=0, unit_share=0, lane_pack=0, alphabet=0, rerun_cap=0, poison=0, memory="library",
                 align_tiles=0):
        import torch
        if memory not in ("library", "torch"):
            raise ValueError("memory must be 'library' or 'torch'")
        self.memory = memory
        self.image = None
        self.ws = None
        self.offsets = _host_i64(offsets)
        self.n = self.offsets.size - 1
        if isinstance(residues, torch.Tensor) and residues.is_cuda:
            d_res = residues.to(torch.int8).contiguous()
        else:
            d_res = torch.from_numpy(_host_i8(residues)).to(device)
        if self.n > 0 and (self.offsets[0] < 0 or self.offsets[-1] > d_res.numel()):
            raise ValueError("offsets reach outside the residue buffer")
        if d_res.numel() == 0:
            d_res = torch.zeros(1, dtype=torch.int8, device=device)
        self.device = d_res.device
        self.alphabet = int(alphabet) if alphabet else 20
        if memory == "torch":
            self.image = torch.empty(sw_db_pack_bytes(self.offsets), dtype=torch.uint8, device=d_res.device)
            self.handle = sw_db_pack_into(d_res, self.offsets, self.image, stream, force_lanes, rerun_threshold,
                                          rows_per_lane, unit_share, lane_pack, alphabet, rerun_cap, poison,
                                          align_tiles)
        else:
            self.handle = sw_db_pack(d_res, self.offsets, stream, force_lanes, rerun_threshold, rows_per_lane,
                                     unit_share, lane_pack, alphabet, rerun_cap, poison, align_tiles)
        del d_res

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().sw_db_free(self.handle)          # synchronises the device: the buffers below are idle
            self.handle = None
        self.image = None
        self.ws = None

    def workspace(self, qoffsets, k=0, scores_in_ws=False, stream=None):
        """A torch workspace of at least the size one search of these query lengths needs (grown, never
        shrunk; kept for the next call)."""
        import torch
        need = sw_batch_workspace_bytes(self.handle, qoffsets, k, scores_in_ws)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        if stream is not None:
            self.ws.record_stream(stream)
        return self.ws

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, r, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().sw_db_info(self.handle, ctypes.byref(n), ctypes.byref(r), ctypes.byref(b)))
        return {"n": n.value, "residues": r.value, "device_bytes": b.value}

    def stats(self):
        out = np.zeros(8, dtype=np.int64)
        _check(load().sw_last_stats(self.handle, _ptr(out)))
        return {"items": int(out[0]), "rerun_pairs": int(out[1]), "rows_per_lane": int(out[2]),
                "waves": int(out[3]), "side_items": int(out[4]), "side_rows_per_lane": int(out[5]),
                "recomputed": int(out[6]), "rerun_overflow": int(out[7])}

    def tune(self, force_lanes=0, rerun_threshold=0, rows_per_lane=0, unit_share=0, lane_pack=0, rerun_cap=0,
             poison=0, align_tiles=0):
        """Change the handle's tuning knobs (results are identical for every setting)."""
        opts = PackOpts(0, int(force_lanes), int(rerun_threshold), int(rows_per_lane), int(unit_share),
                        int(lane_pack), 0, int(rerun_cap), int(poison), int(align_tiles))
        _check(load().sw_db_tune(self.handle, ctypes.byref(opts)))

    def profile_kernels(self, enable=True):
        """Record HIP events around every 16-bit sweep launch of this handle."""
        _check(load().sw_profile_kernels(self.handle, 1 if enable else 0))

    def kernel_times(self):
        """Elapsed ms of the sweep launches recorded since the last call (synchronises)."""
        buf = np.zeros(4096, dtype=np.float32)        # the library remembers at most 4096 launches
        cnt = ctypes.c_int32()
        _check(load().sw_kernel_times(self.handle, _ptr(buf), buf.size, ctypes.byref(cnt)))
        return buf[: cnt.value].astype(np.float64)

    def matrix(self, subst) -> np.ndarray:
        """The substitution matrix as flat int8, checked against this database's alphabet."""
        sm = _square(subst)
        if sm.size != self.alphabet * self.alphabet:
            raise ValueError(f"substitution matrix must be {self.alphabet} x {self.alphabet} for this database")
        return sm

    def search(self, query, subst, gap_open=10, gap_extend=2, out=None, stream=None, mode="local"):
        """int32 tensor [n] of scores in database order; ``mode`` is "local"
        (Smith-Waterman), "global" or "semiglobal" (see sw_search_mode)."""
        import torch
        subst = self.matrix(subst)
        if out is None:
            with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
                out = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        # the handle was packed from self.offsets: no need for the library's O(n) offsets check per call
        if mode == "local" and self.memory == "torch":
            q = _host_i8(query)
            ws = self.workspace(np.array([0, q.size], np.int64), stream=stream)
            sw_search_ws(q, self.handle, None, self.n, subst, gap_open, gap_extend, out, ws, stream)
        elif mode == "local":
            sw_search(query, self.handle, None, self.n, subst, gap_open, gap_extend, out, stream)
        else:
            sw_search_mode(MODES[mode], query, self.handle, None, self.n, subst, gap_open, gap_extend, out, stream)
        return out[: self.n]

    def align(self, query, subjects, subst, gap_open=10, gap_extend=2, stream=None):
        """Optimal local alignments of ``query`` against the given subject indices
        (see ``sw_align``)."""
        subst = self.matrix(subst)
        subs = _host_i64(subjects)
        lens = np.diff(self.offsets)
        # out-of-range indices are left for the library to reject
        longest = int(lens[np.clip(subs, 0, self.n - 1)].max()) if subs.size and self.n > 0 else 0
        return sw_align(query, self.handle, subs, subst, gap_open, gap_extend, longest, stream)

    def align_batch(self, queries, subjects, subst, gap_open=10, gap_extend=2, stream=None):
        """Alignments of each query against its own list of subject indices, in
        one call (see ``sw_align_batch``): a list per query of ``align``'s dicts."""
        subst = self.matrix(subst)
        lens = np.diff(self.offsets)
        subs = [_host_i64(s) for s in subjects]
        if len(subs) != len(queries):
            raise ValueError("one subject list per query")
        # out-of-range indices are left for the library to reject
        longest = max([int(lens[np.clip(s, 0, self.n - 1)].max()) for s in subs if s.size and self.n > 0] or [0])
        return sw_align_batch(queries, self.handle, subs, subst, gap_open, gap_extend, longest, stream)

    def search_batch(self, queries, subst, gap_open=10, gap_extend=2, k=10, keep_scores=True, stream=None):
        """(scores [nq, n] or None, top scores [nq, k], top indices [nq, k])."""
        import torch
        subst = self.matrix(subst)
        qs = [_host_i8(q) for q in queries]
        qo = np.zeros(len(qs) + 1, dtype=np.int64)
        qo[1:] = np.cumsum([q.size for q in qs])
        cat = np.concatenate(qs) if qs else np.zeros(0, np.int8)
        nq = len(qs)
        # outputs come from the pool of the stream the search runs on
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            scores = torch.empty((nq, self.n), dtype=torch.int32, device=self.device) if keep_scores else None
            ts = ti = None
            if k > 0:
                ts = torch.empty((nq, k), dtype=torch.int32, device=self.device)
                ti = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        if self.memory == "torch":
            ws = self.workspace(qo, k, scores is None, stream)
            sw_search_batch_ws(cat, qo, self.handle, subst, gap_open, gap_extend, k, scores, ts, ti, ws, stream)
        else:
            sw_search_batch(cat, qo, self.handle, subst, gap_open, gap_extend, k, scores, ts, ti, stream)
        return scores, ts, ti


MODES = {"local": 0, "global": 1, "semiglobal": 2}


def sw_search_mode(mode, query, handle, h_offsets, n, subst, gap_open, gap_extend, d_scores_out, stream=None):
    lib = load()
    q = _host_i8(query)
    sm = _square(subst)
    offs = None if h_offsets is None else _host_i64(h_offsets)
    _check(lib.sw_search_mode(int(mode), _ptr(q), q.size, handle, None if offs is None else _ptr(offs), int(n),
                              _ptr(sm), int(gap_open), int(gap_extend), _ptr(d_scores_out), _stream(stream)))


def sw_align(query, handle, subjects, subst, gap_open, gap_extend, longest, stream=None):
    """List of dicts (score, q_begin, q_end, subject, s_begin, s_end, ops) for
    ``query`` against each subject index in ``subjects``; ``longest`` bounds
    the subject lengths (sizes the operation buffer)."""
    q = _host_i8(query)
    subs = _host_i64(subjects)
    sm = _square(subst)
    stride = int(q.size + longest + 1)
    out = (Alignment * max(subs.size, 1))()
    ops = np.empty(max(subs.size, 1) * stride, dtype=np.uint8)     # the library writes what is read back
    _check(load().sw_align(_ptr(q), int(q.size), handle, _ptr(subs), int(subs.size), _ptr(sm), int(gap_open),
                           int(gap_extend), ctypes.cast(out, ctypes.c_void_p), _ptr(ops), stride, _stream(stream)))
    res = []
    for k in range(subs.size):
        a = out[k]
        res.append({"score": a.score, "q_begin": a.q_begin, "q_end": a.q_end, "subject": a.subject,
                    "s_begin": a.s_begin, "s_end": a.s_end,
                    "ops": ops[k * stride: k * stride + a.n_ops].tobytes().decode()})
    return res


def sw_align_batch(queries, handle, subjects, subst, gap_open, gap_extend, longest, stream=None):
    """``sw_align`` for several queries: ``subjects[q]`` are the subject indices
    of query ``q``; returns one list of alignment dicts per query."""
    qs = [_host_i8(q) for q in queries]
    subs = [_host_i64(s) for s in subjects]
    qo = np.zeros(len(qs) + 1, dtype=np.int64)
    qo[1:] = np.cumsum([q.size for q in qs])
    so = np.zeros(len(subs) + 1, dtype=np.int64)
    so[1:] = np.cumsum([s.size for s in subs])
    cat_q = np.concatenate(qs) if qs else np.zeros(0, np.int8)
    cat_s = np.concatenate(subs) if subs else np.zeros(0, np.int64)
    sm = _square(subst)
    npairs = int(so[-1])
    stride = int(max([q.size for q in qs] or [0]) + longest + 1)
    out = (Alignment * max(npairs, 1))()
    ops = np.empty(max(npairs, 1) * stride, dtype=np.uint8)        # the library writes what is read back
    _check(load().sw_align_batch(_ptr(cat_q), _ptr(qo), len(qs), handle, _ptr(cat_s), _ptr(so), _ptr(sm),
                                 int(gap_open), int(gap_extend), ctypes.cast(out, ctypes.c_void_p), _ptr(ops), stride,
                                 _stream(stream)))
    res = []
    for q in range(len(qs)):
        row = []
        for k in range(int(so[q]), int(so[q + 1])):
            a = out[k]
            row.append({"score": a.score, "q_begin": a.q_begin, "q_end": a.q_end, "subject": a.subject,
                        "s_begin": a.s_begin, "s_end": a.s_end,
                        "ops": ops[k * stride: k * stride + a.n_ops].tobytes().decode()})
        res.append(row)
    return res


def topk(scores, k, stream=None):
    """(top scores int32[k], indices int64[k]) of a 1-D int32 score tensor; a long
    vector uses the two-launch form with a workspace from torch's allocator."""
    import torch
    lib = load()
    with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
        ts = torch.empty(k, dtype=torch.int32, device=scores.device)
        ti = torch.empty(k, dtype=torch.int64, device=scores.device)
    need = ctypes.c_int64()
    _check(lib.sw_topk_ws_bytes(scores.numel(), int(k), ctypes.byref(need)))
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=scores.device) if need.value > 0 else None
    if ws is not None and stream is not None:
        ws.record_stream(stream)
    _check(lib.sw_topk_ws(_ptr(scores), scores.numel(), int(k), _ptr(ts), _ptr(ti),
                          None if ws is None else _ptr(ws), need.value, _stream(stream)))
    return ts, ti
