"""Exact three-hop top-K path search over a typed knowledge graph on MI355X.

Thin Python binding of ``libmhr.so`` (the C ABI declared in
``include/mhr.h``).  It only marshals arguments: device memory comes from
torch tensors and the work is enqueued on torch's current HIP stream; every
step of the search runs in the library's kernels.  There is no fallback: if
the library is not built, importing this package raises ImportError.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import NamedTuple, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MHR_LIBRARY may name another build of the same library (the phase-clock
# profiling build, libmhr_phase.so); by default the regular build is loaded.
LIB_PATH = os.environ.get("MHR_LIBRARY") or os.path.join(_HERE, "libmhr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2406_07727_amd.build` "
                      "(or __graft_entry__.build()) first")

# torch first: its bundled HIP runtime (soname libamdhip64.so.7) is then the
# one libmhr.so's dependency resolves to, so device pointers and streams from
# torch are valid in the library.  Loading libmhr.so first would pull a
# second HIP runtime into the process.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

MHR_OK = 0
ERR_IO, ERR_CORRUPT, ERR_NOT_FOUND = 9, 10, 11
MHR_MAX_K = 224
NOALLOC_SCRATCH_BYTES = 64 << 20
Q_BAD_ID, Q_BAD_K, Q_EXACT_PASS = 1, 2, 4
PATH_RESCORED, PATH_PRECISION_TIE = 1, 2
DTYPE_F32, DTYPE_BF16 = 0, 1
SCORERS = {"distmult": 0, "transe_l1": 1}

PATH_DTYPE = np.dtype([("a", np.uint32), ("b", np.uint32), ("r1", np.uint16), ("r2", np.uint16),
                       ("r3", np.uint16), ("flags", np.uint16), ("score", np.float32),
                       ("err_bound", np.float32)])
assert PATH_DTYPE.itemsize == 24
BEAM_MAX_HOPS = 4
BEAM_DTYPE = np.dtype([("score", np.float64), ("len", np.uint32), ("v", np.uint32, (BEAM_MAX_HOPS,)),
                       ("r", np.uint16, (BEAM_MAX_HOPS,)), ("pad", np.uint32)])
assert BEAM_DTYPE.itemsize == 40


class _GraphDesc(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_uint32), ("num_relations", ctypes.c_uint32),
                ("num_edges", ctypes.c_uint64), ("head", ctypes.c_void_p),
                ("rel", ctypes.c_void_p), ("tail", ctypes.c_void_p)]


class _GraphStats(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_uint32), ("num_relations", ctypes.c_uint32),
                ("num_triples", ctypes.c_uint64), ("num_pairs", ctypes.c_uint64),
                ("max_out_degree", ctypes.c_uint32), ("max_in_degree", ctypes.c_uint32),
                ("dim", ctypes.c_uint32), ("dtype", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64),
                ("heavy_rows_out", ctypes.c_uint32), ("heavy_rows_in", ctypes.c_uint32)]


class PhaseEvents(ctypes.Structure):
    """hipEvent_t handles recorded around the phases of one query call."""
    _fields_ = [("begin", ctypes.c_void_p), ("gather_begin", ctypes.c_void_p),
                ("gather_end", ctypes.c_void_p), ("end", ctypes.c_void_p)]


class TrainOpts(ctypes.Structure):
    """mhr_train_opts (zero fields take the library's defaults)."""
    _fields_ = [("k", ctypes.c_uint32), ("batch_queries", ctypes.c_uint32), ("step_samples", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("neg_per_hop", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("pad", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("reserved", ctypes.c_uint32 * 8)]


class QueryOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("tile_edges", ctypes.c_uint32),
                ("grid_blocks", ctypes.c_uint32), ("hash_log2", ctypes.c_uint32),
                ("band_abs", ctypes.c_float), ("reserved", ctypes.c_uint32 * 7)]


_vp, _u32, _u64, _i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_lib.mhr_graph_create.restype = _i
_lib.mhr_graph_create.argtypes = [ctypes.POINTER(_GraphDesc), _vp, ctypes.POINTER(_vp)]
_lib.mhr_graph_buffer_sizes.restype = _i
_lib.mhr_graph_buffer_sizes.argtypes = [_u32, _u32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_size_t),
                                        ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_graph_create_in.restype = _i
_lib.mhr_graph_create_in.argtypes = [ctypes.POINTER(_GraphDesc), _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp,
                                     ctypes.POINTER(_vp)]
_lib.mhr_graph_set_embeddings.restype = _i
_lib.mhr_graph_set_embeddings.argtypes = [_vp, _i, _u32, _vp, _vp, _vp]
_lib.mhr_graph_set_scorer.restype = _i
_lib.mhr_graph_set_scorer.argtypes = [_vp, _i, ctypes.c_float]
_lib.mhr_graph_get_stats.restype = _i
_lib.mhr_graph_get_stats.argtypes = [_vp, ctypes.POINTER(_GraphStats)]
_lib.mhr_graph_export_csr.restype = _i
_lib.mhr_graph_export_csr.argtypes = [_vp, _i, _vp, _vp, _vp, _vp]
_lib.mhr_graph_destroy.restype = _i
_lib.mhr_graph_destroy.argtypes = [_vp]
_lib.mhr_workspace_size.restype = _i
_lib.mhr_workspace_size.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_topk_paths.restype = _i
_lib.mhr_topk_paths.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp,
                                _vp, _vp, ctypes.c_size_t, _vp]
_lib.mhr_topk_paths_profiled.restype = _i
_lib.mhr_topk_paths_profiled.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _vp, _vp, _vp, _u32, _vp, _vp,
                                         _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(PhaseEvents)]
_lib.mhr_topk_paths_noalloc.restype = _i
_lib.mhr_topk_paths_noalloc.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp,
                                        _vp, _vp]
_lib.mhr_edge_weights.restype = _i
_lib.mhr_edge_weights.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mhr_plan_create.restype = _i
_lib.mhr_plan_create.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp,
                                 _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
_lib.mhr_plan_launch.restype = _i
_lib.mhr_plan_launch.argtypes = [_vp, _vp]
_lib.mhr_plan_destroy.restype = _i
_lib.mhr_plan_destroy.argtypes = [_vp]
_lib.mhr_autotune.restype = _i
_lib.mhr_autotune.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp,
                              ctypes.c_size_t, _vp, _u32, ctypes.POINTER(QueryOpts), ctypes.POINTER(ctypes.c_float)]
_lib.mhr_topk_paths_pruned.restype = _i
_lib.mhr_topk_paths_pruned.argtypes = [_vp, ctypes.POINTER(QueryOpts), _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp,
                                       _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.mhr_pruner_param_count.restype = ctypes.c_size_t
_lib.mhr_pruner_param_count.argtypes = [_u32, _u32]
_lib.mhr_pruner_create.restype = _i
_lib.mhr_pruner_create.argtypes = [_u32, _u32, ctypes.POINTER(_vp)]
_lib.mhr_pruner_score_workspace_size.restype = _i
_lib.mhr_pruner_score_workspace_size.argtypes = [_vp, _vp, _u32, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_pruner_score.restype = _i
_lib.mhr_pruner_score.argtypes = [_vp, _vp, _u32, _vp, _vp, ctypes.c_uint64, _vp, _vp, _vp, _vp, _u32, _vp,
                                  ctypes.c_size_t, _vp]
_lib.mhr_pruner_buffer_bytes.restype = _i
_lib.mhr_pruner_buffer_bytes.argtypes = [_u32, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_pruner_create_in.restype = _i
_lib.mhr_pruner_create_in.argtypes = [_u32, _u32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
_lib.mhr_pruner_destroy.restype = _i
_lib.mhr_pruner_destroy.argtypes = [_vp]
_lib.mhr_pruner_set_params.restype = _i
_lib.mhr_pruner_set_params.argtypes = [_vp, _vp, _vp]
_lib.mhr_pruner_get_params.restype = _i
_lib.mhr_pruner_get_params.argtypes = [_vp, _vp, _vp, _vp]
_lib.mhr_pruner_workspace_size.restype = _i
_lib.mhr_pruner_workspace_size.argtypes = [_vp, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_pruner_forward.restype = _i
_lib.mhr_pruner_forward.argtypes = [_vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.mhr_pruner_train_step.restype = _i
_lib.mhr_pruner_train_step.argtypes = [_vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float, _i, _vp, _vp, ctypes.c_size_t,
                                       _vp]
_lib.mhr_pruner_train.restype = _i
_lib.mhr_pruner_train.argtypes = [_vp, _vp, ctypes.POINTER(TrainOpts), _u32, _vp, _vp, _vp, _u32,
                                  ctypes.POINTER(_u32), _vp]
_lib.mhr_pruner_candidate_weights.restype = _i
_lib.mhr_pruner_candidate_weights.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mhr_pruner_count.restype = _i
_lib.mhr_pruner_count.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp]
_lib.mhr_pruner_enumerate.restype = _i
_lib.mhr_pruner_enumerate.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mhr_pruner_select.restype = _i
_lib.mhr_pruner_select.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64, _u64, _u32, _vp, _vp, _vp,
                                   _vp]
_lib.mhr_pruner_label.restype = _i
_lib.mhr_pruner_label.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _u32, _vp, _vp]
_lib.mhr_pruner_sample_workspace.restype = ctypes.c_size_t
_lib.mhr_pruner_sample_workspace.argtypes = [_u32, _u64]
_lib.mhr_pruner_sample.restype = _i
_lib.mhr_pruner_sample.argtypes = [_u32, _vp, _vp, _u64, _vp, _vp, _vp, _vp, _vp, _u32, _u64, _vp, _vp, _vp, _vp, _vp,
                                   _vp, ctypes.c_size_t, _vp]
_lib.mhr_pruner_fallback.restype = _i
_lib.mhr_pruner_fallback.argtypes = [_u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp, ctypes.c_float, _vp, _vp, _vp, _vp,
                                     _vp, _vp]
_lib.mhr_scatter_results.restype = _i
_lib.mhr_scatter_results.argtypes = [_u32, _vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mhr_beam_workspace_size.restype = _i
_lib.mhr_beam_workspace_size.argtypes = [_vp, _u32, _u32, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_beam_search.restype = _i
_lib.mhr_beam_search.argtypes = [_vp, _u32, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.mhr_wide_graph_create.restype = _i
_lib.mhr_wide_graph_create.argtypes = [ctypes.POINTER(_GraphDesc), _vp, ctypes.POINTER(_vp)]
_lib.mhr_wide_graph_destroy.restype = _i
_lib.mhr_wide_graph_destroy.argtypes = [_vp]
_lib.mhr_wide_graph_set_embeddings.restype = _i
_lib.mhr_wide_graph_set_embeddings.argtypes = [_vp, _i, _u32, _vp, _vp, ctypes.c_double]
_lib.mhr_wide_graph_get_stats.restype = _i
_lib.mhr_wide_graph_get_stats.argtypes = [_vp, _vp]
_lib.mhr_wide_graph_export_csr.restype = _i
_lib.mhr_wide_graph_export_csr.argtypes = [_vp, _i, _vp, _vp, _vp, _vp]
_lib.mhr_wide_workspace_size.restype = _i
_lib.mhr_wide_workspace_size.argtypes = [_vp, _u32, _vp, _vp, _vp, _u32, ctypes.POINTER(ctypes.c_size_t), _vp]
_lib.mhr_wide_topk_paths.restype = _i
_lib.mhr_wide_topk_paths.argtypes = [_vp, _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp,
                                     _vp]
_lib.mhr_scan_workspace_size.restype = _i
_lib.mhr_scan_workspace_size.argtypes = [_u32, _u32, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_scan_topk.restype = _i
_lib.mhr_scan_topk.argtypes = [_i, _u32, _vp, _vp, _u32, _u32, _u32, _vp, _vp, _u32, _vp, _u32, _u32, _u32,
                               ctypes.c_float, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.mhr_scan_pipeline_workspace_size.restype = _i
_lib.mhr_scan_pipeline_workspace_size.argtypes = [_u32, _u32, _u32, _u32, ctypes.POINTER(ctypes.c_size_t)]
_lib.mhr_scan_pipeline.restype = _i
_lib.mhr_scan_pipeline.argtypes = [_i, _u32, _vp, _vp, _u32, _u32, _u32, _vp, _vp, _u32, _u32, _u32, _vp, _u32, _vp,
                                   _u32, _u32, ctypes.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                   _vp]
_cp = ctypes.c_char_p
_lib.mhr_crc32.restype = ctypes.c_uint32
_lib.mhr_crc32.argtypes = [ctypes.c_uint32, _vp, ctypes.c_size_t]
_lib.mhr_pruner_file_info.restype = _i
_lib.mhr_pruner_file_info.argtypes = [_cp, ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u32)]
_lib.mhr_pruner_save.restype = _i
_lib.mhr_pruner_save.argtypes = [_vp, _cp, _vp]
_lib.mhr_pruner_load.restype = _i
_lib.mhr_pruner_load.argtypes = [_vp, _cp, _vp]
_lib.mhr_tuning_file_records.restype = _i
_lib.mhr_tuning_file_records.argtypes = [_cp, ctypes.POINTER(_u32)]
_lib.mhr_tuning_save.restype = _i
_lib.mhr_tuning_save.argtypes = [_cp, _vp, _u32, _u32, ctypes.POINTER(QueryOpts), ctypes.c_float]
_lib.mhr_tuning_load.restype = _i
_lib.mhr_tuning_load.argtypes = [_cp, _vp, _u32, _u32, ctypes.POINTER(QueryOpts), ctypes.POINTER(ctypes.c_float)]
_lib.mhr_debug_phase_ticks.restype = _i
_lib.mhr_debug_phase_ticks.argtypes = [_vp, _u32, ctypes.POINTER(ctypes.c_double), _i]
_lib.mhr_status_string.restype = ctypes.c_char_p
_lib.mhr_status_string.argtypes = [_i]
_lib.mhr_last_error.restype = ctypes.c_char_p
_lib.mhr_last_error.argtypes = []


class MhrError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.mhr_last_error().decode(errors="replace")
        name = _lib.mhr_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != MHR_OK:
        raise MhrError(status, where)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_u32(t):
    """Contiguous 32-bit integer device tensor (int32 or uint32 storage)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t, dtype=np.int64).astype(np.uint32).view(np.int32))
    if t.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        t = t.to(torch.int64).to(torch.int32)
    if not t.is_cuda:
        t = t.cuda()
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class TopK:
    """Result tensors (on the device) of one batched query."""
    paths: "object"      # uint8 tensor [nq, k_max, 24] (mhr_path records)
    count: "object"      # int32 tensor [nq]
    total: "object"      # int64 tensor [nq]: |P(s,t)|
    status: "object"     # int32 tensor [nq]
    k_max: int

    def to_numpy(self):
        """(paths structured array [nq][k_max], count, total, status) on the host."""
        p = self.paths.cpu().numpy().view(PATH_DTYPE).reshape(self.paths.shape[0], self.k_max)
        return (p, self.count.cpu().numpy().view(np.uint32), self.total.cpu().numpy().view(np.uint64),
                self.status.cpu().numpy().view(np.uint32))


def graph_buffer_sizes(num_vertices: int, num_relations: int, num_edges: int) -> tuple:
    """(csr_bytes, tmp_bytes) that mhr_graph_create_in needs."""
    c, t = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.mhr_graph_buffer_sizes(int(num_vertices), int(num_relations), int(num_edges), ctypes.byref(c),
                                       ctypes.byref(t)), "mhr_graph_buffer_sizes")
    return int(c.value), int(t.value)


class Graph:
    """A typed directed graph resident on the current HIP device.

    head, rel, tail: integer device tensors (or host arrays) of one edge
    list (h, r, t).  Identical triples are merged.  caller_buffers: give the
    library torch-allocated buffers (mhr_graph_create_in) instead of letting
    it allocate its own.  The device memory of the handle is freed by
    ``close()`` or on garbage collection."""

    def __init__(self, head, rel, tail, num_vertices: int, num_relations: int, stream=None,
                 caller_buffers: bool = False):
        torch = _torch()
        h, r, t = _dev_u32(head), _dev_u32(rel), _dev_u32(tail)
        if not (h.numel() == r.numel() == t.numel()):
            raise ValueError("head, rel and tail must have the same length")
        desc = _GraphDesc(int(num_vertices), int(num_relations), int(h.numel()),
                          h.data_ptr(), r.data_ptr(), t.data_ptr())
        handle = ctypes.c_void_p()
        torch.cuda.synchronize()
        self._csr_buf = None
        if caller_buffers:
            cb, tb = graph_buffer_sizes(num_vertices, num_relations, h.numel())
            csr = torch.empty(cb + 256, dtype=torch.uint8, device="cuda")
            tmp = torch.empty(tb + 256, dtype=torch.uint8, device="cuda")
            co, to = (-csr.data_ptr()) % 256, (-tmp.data_ptr()) % 256   # 256-byte aligned views
            _check(_lib.mhr_graph_create_in(ctypes.byref(desc), csr.data_ptr() + co, cb, tmp.data_ptr() + to, tb,
                                            _stream_ptr(stream), ctypes.byref(handle)), "mhr_graph_create_in")
            self._csr_buf = csr   # borrowed by the handle until close()
            del tmp
        else:
            _check(_lib.mhr_graph_create(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(handle)),
                   "mhr_graph_create")
        self._h = handle
        self.n = int(num_vertices)
        self.R = int(num_relations)
        self._emb = None
        self._ws = {}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.mhr_graph_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._csr_buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_embeddings(self, entity, relation, dtype: Optional[str] = None, stream=None):
        """entity [n][d], relation [R][d] device tensors: float32, bfloat16, or
        int16/uint16 holding bfloat16 bit patterns.  The tensors are kept
        alive by this object (the library borrows them)."""
        torch = _torch()
        if dtype is None:
            dtype = "f32" if entity.dtype == torch.float32 else "bf16"
        code = DTYPE_F32 if dtype == "f32" else DTYPE_BF16
        X = entity.contiguous()
        Y = relation.contiguous()
        if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
            raise ValueError("embedding tables must be [n][d] and [R][d]")
        if X.shape[0] != self.n or Y.shape[0] != self.R:
            raise ValueError("embedding row counts must match the graph")
        _check(_lib.mhr_graph_set_embeddings(self._h, code, int(X.shape[1]), X.data_ptr(), Y.data_ptr(),
                                             _stream_ptr(stream)), "mhr_graph_set_embeddings")
        self._emb = (X, Y)
        self.dim = int(X.shape[1])

    def set_scorer(self, scorer: str = "distmult", gamma: float = 1.0):
        """Edge scorer for later queries: "distmult" (logsigmoid of the
        DistMult score, the default) or "transe_l1" (gamma minus the L1
        distance of head plus relation from tail)."""
        if scorer not in SCORERS:
            raise ValueError(f"unknown scorer {scorer!r}")
        _check(_lib.mhr_graph_set_scorer(self._h, SCORERS[scorer], float(gamma)), "mhr_graph_set_scorer")
        self.scorer, self.gamma = scorer, float(gamma)

    def stats(self) -> dict:
        s = _GraphStats()
        _check(_lib.mhr_graph_get_stats(self._h, ctypes.byref(s)), "mhr_graph_get_stats")
        return {f: getattr(s, f) for f, _ in _GraphStats._fields_}

    def export_csr(self, reverse: bool = False, stream=None):
        """(row_ptr, col, rmask) int32 device tensors of the forward (or
        reverse) CSR."""
        torch = _torch()
        st = self.stats()
        rp = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(1, st["num_pairs"]), dtype=torch.int32, device="cuda")
        rm = torch.empty(max(1, st["num_pairs"]), dtype=torch.int32, device="cuda")
        _check(_lib.mhr_graph_export_csr(self._h, int(reverse), rp.data_ptr(), col.data_ptr(), rm.data_ptr(),
                                         _stream_ptr(stream)), "mhr_graph_export_csr")
        return rp, col[:st["num_pairs"]], rm[:st["num_pairs"]]

    def workspace_bytes(self, nq: int, k_max: int, opts: Optional[QueryOpts] = None) -> int:
        n = ctypes.c_size_t()
        _check(_lib.mhr_workspace_size(self._h, ctypes.byref(opts) if opts else None, int(nq), int(k_max),
                                       ctypes.byref(n)), "mhr_workspace_size")
        return int(n.value)

    @staticmethod
    def _queries(src, dst, k, k_max, opts):
        s, d = _dev_u32(src), _dev_u32(dst)
        nq = s.numel()
        o = QueryOpts() if opts is None else opts
        kt = None
        if k is None or isinstance(k, (int, np.integer)):
            kk = int(k if k is not None else o.k)
            o = QueryOpts(kk, o.tile_edges, o.grid_blocks, o.hash_log2, o.band_abs)
            if k_max is None:
                k_max = kk
        else:
            kt = _dev_u32(k)
            if k_max is None:
                k_max = int(kt.max().item()) if nq else 1
        return s, d, kt, nq, o, int(k_max)

    @staticmethod
    def _new_out(nq, k_max):
        torch = _torch()
        return TopK(torch.empty((nq, k_max, 24), dtype=torch.uint8, device="cuda"),
                    torch.empty(nq, dtype=torch.int32, device="cuda"),
                    torch.empty(nq, dtype=torch.int64, device="cuda"),
                    torch.empty(nq, dtype=torch.int32, device="cuda"), k_max)

    def topk(self, src, dst, k=None, k_max: Optional[int] = None, opts: Optional[QueryOpts] = None,
             out: Optional[TopK] = None, stream=None, events: Optional[PhaseEvents] = None) -> TopK:
        """Exact top-K three-hop paths for each (src[q], dst[q]).  k: an int
        (same K for all) or a per-query integer tensor (then k_max bounds
        it).  Asynchronous on the current stream."""
        torch = _torch()
        s, d, kt, nq, o, k_max = self._queries(src, dst, k, k_max, opts)
        need = self.workspace_bytes(nq, k_max, o)
        ws = self._ws.get("buf")
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            self._ws["buf"] = ws
        if out is None:
            out = self._new_out(nq, k_max)
        if events is None:
            _check(_lib.mhr_topk_paths(self._h, ctypes.byref(o), nq, _ptr(s), _ptr(d), _ptr(kt), k_max,
                                       _ptr(out.paths), _ptr(out.count), _ptr(out.total), _ptr(out.status),
                                       _ptr(ws), ws.numel(), _stream_ptr(stream)), "mhr_topk_paths")
        else:
            _check(_lib.mhr_topk_paths_profiled(self._h, ctypes.byref(o), nq, _ptr(s), _ptr(d), _ptr(kt), k_max,
                                                _ptr(out.paths), _ptr(out.count), _ptr(out.total),
                                                _ptr(out.status), _ptr(ws), ws.numel(), _stream_ptr(stream),
                                                ctypes.byref(events)), "mhr_topk_paths_profiled")
        out._keep = (s, d, kt)
        return out

    def topk_noalloc(self, src, dst, k=None, k_max: Optional[int] = None, opts: Optional[QueryOpts] = None,
                     out: Optional[TopK] = None, stream=None) -> TopK:
        """topk through mhr_topk_paths_noalloc: the library's fixed scratch
        array serves as the workspace (nothing is allocated by the call; the
        batch's workspace must fit NOALLOC_SCRATCH_BYTES)."""
        s, d, kt, nq, o, k_max = self._queries(src, dst, k, k_max, opts)
        if out is None:
            out = self._new_out(nq, k_max)
        _check(_lib.mhr_topk_paths_noalloc(self._h, ctypes.byref(o), nq, _ptr(s), _ptr(d), _ptr(kt), k_max,
                                           _ptr(out.paths), _ptr(out.count), _ptr(out.total), _ptr(out.status),
                                           _stream_ptr(stream)), "mhr_topk_paths_noalloc")
        out._keep = (s, d, kt)
        return out

    def topk_pruned(self, src, dst, k, keep, keep_off, k_max: Optional[int] = None,
                    opts: Optional[QueryOpts] = None, out: Optional[TopK] = None, stream=None) -> TopK:
        """topk restricted by keep flags (uint8 device tensor) with per-query
        offsets keep_off (int64 device tensor [>= nq]); see
        mhr_topk_paths_pruned."""
        torch = _torch()
        s, d, kt, nq, o, k_max = self._queries(src, dst, k, k_max, opts)
        need = self.workspace_bytes(nq, k_max, o)
        ws = self._ws.get("buf")
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            self._ws["buf"] = ws
        if out is None:
            out = self._new_out(nq, k_max)
        _check(_lib.mhr_topk_paths_pruned(self._h, ctypes.byref(o), nq, _ptr(s), _ptr(d), _ptr(kt), k_max,
                                          _ptr(keep), _ptr(keep_off), _ptr(out.paths), _ptr(out.count),
                                          _ptr(out.total), _ptr(out.status), _ptr(ws), ws.numel(),
                                          _stream_ptr(stream)), "mhr_topk_paths_pruned")
        out._keep = (s, d, kt, keep, keep_off)
        return out

    def autotune(self, src, dst, k=None, k_max: Optional[int] = None, opts: Optional[QueryOpts] = None,
                 reps: int = 3, stream=None):
        """Fastest (tile_edges, hash_log2) for this batch, by timing each
        candidate; the library checks that every candidate gives identical
        results.  Returns (QueryOpts, ms per call).  Synchronises."""
        torch = _torch()
        s, d, kt, nq, o, k_max = self._queries(src, dst, k, k_max, opts)
        ws = torch.empty(self.workspace_bytes(nq, k_max, o), dtype=torch.uint8, device="cuda")
        out = self._new_out(nq, k_max)
        tuned = QueryOpts()
        ms = ctypes.c_float()
        _check(_lib.mhr_autotune(self._h, ctypes.byref(o), nq, _ptr(s), _ptr(d), _ptr(kt), k_max,
                                 _ptr(out.paths), _ptr(out.count), _ptr(out.total), _ptr(out.status),
                                 _ptr(ws), ws.numel(), _stream_ptr(stream), int(reps), ctypes.byref(tuned),
                                 ctypes.byref(ms)), "mhr_autotune")
        return tuned, float(ms.value)

    def save_tuning(self, path: str, nq: int, k_max: int, tuned: QueryOpts, ms: float):
        """Records tuned settings for this device, graph, nq and k_max in the
        tuning cache at path (mhr_tuning_save)."""
        _check(_lib.mhr_tuning_save(os.fsencode(path), self._h, int(nq), int(k_max), ctypes.byref(tuned),
                                    float(ms)), "mhr_tuning_save")

    def load_tuning(self, path: str, nq: int, k_max: int):
        """(QueryOpts, ms) from the tuning cache, or None when it holds no
        record for this device, graph, nq and k_max."""
        o = QueryOpts()
        ms = ctypes.c_float()
        st = _lib.mhr_tuning_load(os.fsencode(path), self._h, int(nq), int(k_max), ctypes.byref(o), ctypes.byref(ms))
        if st == ERR_NOT_FOUND:
            return None
        _check(st, "mhr_tuning_load")
        return o, float(ms.value)

    def plan(self, src, dst, k=None, k_max: Optional[int] = None, opts: Optional[QueryOpts] = None,
             stream=None) -> "Plan":
        """Captures one batched query call into a HIP graph (see Plan)."""
        return Plan(self, src, dst, k, k_max, opts, stream)

    def beam(self, src, dst, hops: int, k: int, stream=None):
        """The generic multi-hop search (mhr_beam_search): per query the best
        k recorded paths of at most `hops` edges.  Returns (paths [nq, k]
        uint8 records of BEAM_DTYPE, count [nq], recorded [nq]) device
        tensors; beam_to_numpy converts them."""
        torch = _torch()
        s, d = _dev_u32(src), _dev_u32(dst)
        nq = s.numel()
        need = ctypes.c_size_t()
        _check(_lib.mhr_beam_workspace_size(self._h, nq, int(hops), int(k), ctypes.byref(need)),
               "mhr_beam_workspace_size")
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device="cuda")
        out = torch.empty((nq, k, BEAM_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
        cnt = torch.empty(max(nq, 1), dtype=torch.int32, device="cuda")
        rec = torch.empty(max(nq, 1), dtype=torch.int64, device="cuda")
        _check(_lib.mhr_beam_search(self._h, nq, _ptr(s), _ptr(d), int(hops), int(k), _ptr(out), _ptr(cnt), _ptr(rec),
                                    _ptr(ws), ws.numel(), _stream_ptr(stream)), "mhr_beam_search")
        self._beam_keep = (s, d, ws)
        return out, cnt[:nq], rec[:nq]

    def edge_weights(self, u, r, v, stream=None):
        """FP32 log-sigmoid DistMult weights with their error bounds, and the
        compensated (hi, lo) values, for arbitrary (u, r, v) triples."""
        torch = _torch()
        U, Rr, V = _dev_u32(u), _dev_u32(r), _dev_u32(v)
        ne = U.numel()
        w = torch.empty(ne, dtype=torch.float32, device="cuda")
        e = torch.empty_like(w)
        hi = torch.empty_like(w)
        lo = torch.empty_like(w)
        _check(_lib.mhr_edge_weights(self._h, ne, _ptr(U), _ptr(Rr), _ptr(V), _ptr(w), _ptr(e), _ptr(hi),
                                     _ptr(lo), _stream_ptr(stream)), "mhr_edge_weights")
        return w, e, hi, lo


@dataclass
class Candidates:
    """Frontier candidates of a query batch (device tensors); see
    mhr_pruner_count / mhr_pruner_enumerate."""
    src: "object"
    dst: "object"
    entry_off: "object"   # int64 [nq + 1]: keep-flag offsets (entries of s's out-row, then t's in-row)
    cand_off: "object"    # int64 [nq + 1]
    cand_split: "object"  # int64 [nq]: first second-hop candidate of each query
    q: "object"           # int32 [n]
    v: "object"           # int32 [n]
    r: "object"           # int32 [n]
    e: "object"           # int64 [n]: keep-flag index
    n: int
    n_entries: int


def candidates(graph: Graph, src, dst, stream=None) -> Candidates:
    """Enumerates the first- and second-hop candidates of every query
    (synchronises once to size the outputs)."""
    torch = _torch()
    s, d = _dev_u32(src), _dev_u32(dst)
    nq = s.numel()
    eo = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    co = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    _check(_lib.mhr_pruner_count(graph._h, nq, _ptr(s), _ptr(d), _ptr(eo), _ptr(co), _stream_ptr(stream)),
           "mhr_pruner_count")
    n = int(co[nq].item())
    ne = int(eo[nq].item())
    cs = torch.empty(nq, dtype=torch.int64, device="cuda")
    cq = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    cv = torch.empty_like(cq)
    cr = torch.empty_like(cq)
    ce = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
    _check(_lib.mhr_pruner_enumerate(graph._h, nq, _ptr(s), _ptr(d), _ptr(eo), _ptr(co), _ptr(cs), _ptr(cq),
                                     _ptr(cv), _ptr(cr), _ptr(ce), _stream_ptr(stream)), "mhr_pruner_enumerate")
    return Candidates(s, d, eo, co, cs, cq[:n], cv[:n], cr[:n], ce[:n], n, ne)


def select(graph: Graph, c: Candidates, scores, keep_permille: int = 100, stream=None):
    """Keep flags (uint8 [n_entries]) of the top keep_permille / 1000 of each
    query's entries per hop, ranked by their best candidate score, and the
    kept sigmoid mass (float32 [nq, 2])."""
    torch = _torch()
    nq = c.src.numel()
    keep = torch.empty(max(c.n_entries, 1), dtype=torch.uint8, device="cuda")
    mass = torch.empty((nq, 2), dtype=torch.float32, device="cuda")
    key = torch.empty(max(c.n_entries, 1), dtype=torch.int32, device="cuda")
    sc = scores.contiguous() if c.n else None
    _check(_lib.mhr_pruner_select(graph._h, nq, _ptr(c.src), _ptr(c.dst), _ptr(c.entry_off), _ptr(c.cand_off),
                                  _ptr(c.cand_split), _ptr(sc), _ptr(c.e) if c.n else None, c.n, c.n_entries,
                                  int(keep_permille), _ptr(keep), _ptr(mass), _ptr(key), _stream_ptr(stream)),
           "mhr_pruner_select")
    return keep, mass


class Pruner:
    """The learned frontier pruner's network on the device (see
    include/mhr.h): FP32 master parameters, bfloat16 MFMA products."""

    def __init__(self, dim: int, hidden: int, caller_buffer: bool = False):
        """caller_buffer: keep the state in a torch-allocated buffer
        (mhr_pruner_create_in) instead of library allocations."""
        h = ctypes.c_void_p()
        self._buf = None
        if caller_buffer:
            torch = _torch()
            nb = ctypes.c_size_t()
            _check(_lib.mhr_pruner_buffer_bytes(int(dim), int(hidden), ctypes.byref(nb)), "mhr_pruner_buffer_bytes")
            buf = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
            off = (-buf.data_ptr()) % 256
            torch.cuda.synchronize()
            _check(_lib.mhr_pruner_create_in(int(dim), int(hidden), buf.data_ptr() + off, nb.value, None,
                                             ctypes.byref(h)), "mhr_pruner_create_in")
            self._buf = buf   # borrowed by the handle until close()
        else:
            _check(_lib.mhr_pruner_create(int(dim), int(hidden), ctypes.byref(h)), "mhr_pruner_create")
        self._h = h
        self.dim, self.hidden = int(dim), int(hidden)
        self.n_params = int(_lib.mhr_pruner_param_count(self.dim, self.hidden))
        self._ws = None

    @staticmethod
    def param_count(dim: int, hidden: int) -> int:
        return int(_lib.mhr_pruner_param_count(int(dim), int(hidden)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.mhr_pruner_destroy(self._h)
            self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta, stream=None):
        torch = _torch()
        t = torch.as_tensor(theta, dtype=torch.float32).cuda().contiguous()
        assert t.numel() == self.n_params
        _check(_lib.mhr_pruner_set_params(self._h, _ptr(t), _stream_ptr(stream)), "mhr_pruner_set_params")
        torch.cuda.synchronize()

    def params(self, stream=None):
        torch = _torch()
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_lib.mhr_pruner_get_params(self._h, _ptr(t), None, _stream_ptr(stream)), "mhr_pruner_get_params")
        return t

    def grad(self, stream=None):
        torch = _torch()
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_lib.mhr_pruner_get_params(self._h, None, _ptr(t), _stream_ptr(stream)), "mhr_pruner_get_params")
        return t

    def train(self, graph: "Graph", src, dst, opts: TrainOpts, max_steps: int = 1 << 20, stream=None):
        """A whole training run (mhr_pruner_train); returns the loss per step."""
        s, d = _dev_u32(src), _dev_u32(dst)
        losses = (ctypes.c_float * max(1, max_steps))()
        n = _u32()
        _check(_lib.mhr_pruner_train(self._h, graph._h, ctypes.byref(opts), s.numel(), _ptr(s), _ptr(d), losses,
                                     int(max_steps), ctypes.byref(n), _stream_ptr(stream)), "mhr_pruner_train")
        return [float(losses[i]) for i in range(min(int(n.value), max_steps))]

    def save(self, path: str, stream=None):
        """Checkpoint: parameters, Adam moments and step (mhr_pruner_save)."""
        _check(_lib.mhr_pruner_save(self._h, os.fsencode(path), _stream_ptr(stream)), "mhr_pruner_save")

    def load(self, path: str, stream=None):
        """Restores a checkpoint written by save (mhr_pruner_load)."""
        _check(_lib.mhr_pruner_load(self._h, os.fsencode(path), _stream_ptr(stream)), "mhr_pruner_load")

    def _workspace(self, n):
        torch = _torch()
        need = ctypes.c_size_t()
        _check(_lib.mhr_pruner_workspace_size(self._h, int(n), ctypes.byref(need)), "mhr_pruner_workspace_size")
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device="cuda")
        return self._ws

    def forward(self, graph: Graph, q, src, dst, v, r, stream=None):
        """Logits (float32 [n]) of samples (q[i], v[i], r[i])."""
        torch = _torch()
        q, s, d, v, r = (_dev_u32(x) for x in (q, src, dst, v, r))
        n = q.numel()
        out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        ws = self._workspace(n)
        _check(_lib.mhr_pruner_forward(self._h, graph._h, n, _ptr(q), _ptr(s), _ptr(d), _ptr(v), _ptr(r), _ptr(out),
                                       _ptr(ws), ws.numel(), _stream_ptr(stream)), "mhr_pruner_forward")
        return out[:n]

    def score(self, graph: Graph, src, dst, q, v, r, chunk: int = 1 << 18, stream=None):
        """Logits (float32 [n]) of frontier candidates (q[i], v[i], r[i]) of
        the queries (src, dst), through mhr_pruner_score (first layer split
        by input block, output fused)."""
        torch = _torch()
        s, d, q, v, r = (_dev_u32(x) for x in (src, dst, q, v, r))
        nq, n = s.numel(), q.numel()
        out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        if n == 0:
            return out[:0]
        chunk = int(max(1, min(chunk, n)))
        nb = ctypes.c_size_t()
        _check(_lib.mhr_pruner_score_workspace_size(self._h, graph._h, nq, chunk, ctypes.byref(nb)),
               "mhr_pruner_score_workspace_size")
        if getattr(self, "_sws", None) is None or self._sws.numel() < nb.value:
            self._sws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
        _check(_lib.mhr_pruner_score(self._h, graph._h, nq, _ptr(s), _ptr(d), n, _ptr(q), _ptr(v), _ptr(r),
                                     _ptr(out), chunk, _ptr(self._sws), self._sws.numel(), _stream_ptr(stream)),
               "mhr_pruner_score")
        return out[:n]

    def train_step(self, graph: Graph, q, src, dst, v, r, label, pos_weight=1.0, lr=1e-3, beta1=0.9,
                   beta2=0.999, eps=1e-8, update=True, stream=None):
        """One step (forward, loss, gradient, Adam if update); returns the
        loss as a device scalar tensor."""
        torch = _torch()
        q, s, d, v, r = (_dev_u32(x) for x in (q, src, dst, v, r))
        y = torch.as_tensor(label, dtype=torch.float32).cuda().contiguous()
        n = q.numel()
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        ws = self._workspace(n)
        _check(_lib.mhr_pruner_train_step(self._h, graph._h, n, _ptr(q), _ptr(s), _ptr(d), _ptr(v), _ptr(r), _ptr(y),
                                          float(pos_weight), float(lr), float(beta1), float(beta2), float(eps),
                                          1 if update else 0, _ptr(loss), _ptr(ws), ws.numel(), _stream_ptr(stream)),
               "mhr_pruner_train_step")
        return loss


WIDE_MAX_K = 256
WIDE_PATH_DTYPE = np.dtype([("score", np.float64), ("a", np.uint32), ("b", np.uint32), ("r1", np.uint16),
                            ("r2", np.uint16), ("r3", np.uint16), ("reserved", np.uint16)])
assert WIDE_PATH_DTYPE.itemsize == 24


class _WideStats(ctypes.Structure):
    _fields_ = [("num_vertices", _u32), ("num_relations", _u32), ("num_triples", ctypes.c_uint64),
                ("max_out_degree", _u32), ("max_in_degree", _u32), ("dim", _u32), ("dtype", _u32),
                ("device_bytes", ctypes.c_uint64)]


WIDE_WORK_FIELDS = ("scanned", "matches", "paths", "frontier", "distinct", "probe_len", "tiles", "forward")


class WideResult(NamedTuple):
    paths: object    # device uint8 [nq][k_max * 24] (mhr_wide_path records)
    count: object
    total: object
    status: object
    work: object     # device int64 [nq][8] (mhr_wide_work records)

    def work_numpy(self) -> dict:
        w = self.work.cpu().numpy().view(np.uint64)
        return {f: w[:, i] for i, f in enumerate(WIDE_WORK_FIELDS)}

    def to_numpy(self):
        """(paths [nq][k_max] of WIDE_PATH_DTYPE, count, total, status)."""
        nq = self.count.numel()
        p = self.paths.cpu().numpy().view(WIDE_PATH_DTYPE).reshape(nq, -1)
        return (p, self.count.cpu().numpy().view(np.uint32), self.total.cpu().numpy().view(np.uint64),
                self.status.cpu().numpy().view(np.uint32))


class WideGraph:
    """A knowledge graph with up to 65,535 relations (one CSR entry per
    distinct triple), searched with TransE-L1 scores in FP64
    (include/mhr.h, wide-relation graphs)."""

    def __init__(self, head, rel, tail, num_vertices: int, num_relations: int, stream=None):
        torch = _torch()
        h, r, t = _dev_u32(head), _dev_u32(rel), _dev_u32(tail)
        if not (h.numel() == r.numel() == t.numel()):
            raise ValueError("head, rel and tail must have the same length")
        desc = _GraphDesc(int(num_vertices), int(num_relations), int(h.numel()),
                          h.data_ptr(), r.data_ptr(), t.data_ptr())
        handle = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(_lib.mhr_wide_graph_create(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(handle)),
               "mhr_wide_graph_create")
        self._h = handle
        self.n = int(num_vertices)
        self.R = int(num_relations)
        self._emb = None

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.mhr_wide_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_embeddings(self, entity, relation, gamma: float = 1.0, dtype: Optional[str] = None):
        torch = _torch()
        if dtype is None:
            dtype = "f32" if entity.dtype == torch.float32 else "bf16"
        X, Y = entity.contiguous(), relation.contiguous()
        if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1] or X.shape[0] != self.n or Y.shape[0] != self.R:
            raise ValueError("embedding tables must be [n][d] and [R][d] matching the graph")
        _check(_lib.mhr_wide_graph_set_embeddings(self._h, DTYPE_F32 if dtype == "f32" else DTYPE_BF16,
                                                  int(X.shape[1]), X.data_ptr(), Y.data_ptr(), float(gamma)),
               "mhr_wide_graph_set_embeddings")
        self._emb = (X, Y)
        self.dim = int(X.shape[1])

    def stats(self) -> dict:
        st = _WideStats()
        _check(_lib.mhr_wide_graph_get_stats(self._h, ctypes.byref(st)), "mhr_wide_graph_get_stats")
        return {f: getattr(st, f) for f, _ in _WideStats._fields_}

    def export_csr(self, reverse: bool = False, stream=None):
        torch = _torch()
        st = self.stats()
        rp = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(st["num_triples"], 1), dtype=torch.int32, device="cuda")
        rel = torch.empty(max(st["num_triples"], 1), dtype=torch.int16, device="cuda")
        _check(_lib.mhr_wide_graph_export_csr(self._h, 1 if reverse else 0, rp.data_ptr(), col.data_ptr(),
                                              rel.data_ptr(), _stream_ptr(stream)), "mhr_wide_graph_export_csr")
        return rp, col[:st["num_triples"]], rel[:st["num_triples"]]

    def workspace_size(self, src, dst, k_max: int, k=None, stream=None) -> int:
        s, d = _dev_u32(src), _dev_u32(dst)
        kk = _dev_u32(k) if k is not None else None
        b = ctypes.c_size_t()
        _check(_lib.mhr_wide_workspace_size(self._h, s.numel(), _ptr(s), _ptr(d), _ptr(kk), int(k_max),
                                            ctypes.byref(b), _stream_ptr(stream)), "mhr_wide_workspace_size")
        return int(b.value)

    def topk(self, src, dst, k_max: int, k=None, workspace=None, stream=None, events=None) -> WideResult:
        """Exact top-K paths of each query (src[q], dst[q]); k: per-query K
        (None: k_max for all).  workspace: a device uint8 tensor of at least
        workspace_size() bytes, or None to allocate one."""
        torch = _torch()
        s, d = _dev_u32(src), _dev_u32(dst)
        kk = _dev_u32(k) if k is not None else None
        nq = s.numel()
        if workspace is None:
            workspace = torch.empty(max(self.workspace_size(s, d, k_max, kk, stream), 1), dtype=torch.uint8,
                                    device="cuda")
        paths = torch.empty((nq, int(k_max) * 24), dtype=torch.uint8, device="cuda")
        count = torch.empty(nq, dtype=torch.int32, device="cuda")
        total = torch.empty(nq, dtype=torch.int64, device="cuda")
        status = torch.empty(nq, dtype=torch.int32, device="cuda")
        work = torch.empty((nq, len(WIDE_WORK_FIELDS)), dtype=torch.int64, device="cuda")
        ev = ctypes.byref(events) if events is not None else None
        _check(_lib.mhr_wide_topk_paths(self._h, nq, _ptr(s), _ptr(d), _ptr(kk), int(k_max), _ptr(paths),
                                        _ptr(count), _ptr(total), _ptr(status), _ptr(work), _ptr(workspace),
                                        workspace.numel(), _stream_ptr(stream), ev), "mhr_wide_topk_paths")
        return WideResult(paths, count, total, status, work)


def beam_to_numpy(out, cnt, rec):
    """Host copies of mhr_beam_search's results: (paths [nq][k] of
    BEAM_DTYPE, count, recorded)."""
    nq, k = out.shape[0], out.shape[1]
    p = out.cpu().numpy().view(BEAM_DTYPE).reshape(nq, k)
    return p, cnt.cpu().numpy().view(np.uint32), rec.cpu().numpy().view(np.uint64)


def crc32(data: bytes, crc: int = 0) -> int:
    """The library's CRC-32 (the checksum its files carry)."""
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    return int(_lib.mhr_crc32(int(crc), buf, len(data)))


def pruner_file_info(path: str):
    """(dim, hidden, step) of a pruner checkpoint, checked on the host
    (raises MhrError for a damaged or foreign file)."""
    d, h, s = _u32(), _u32(), _u32()
    _check(_lib.mhr_pruner_file_info(os.fsencode(path), ctypes.byref(d), ctypes.byref(h), ctypes.byref(s)),
           "mhr_pruner_file_info")
    return int(d.value), int(h.value), int(s.value)


def tuning_file_records(path: str) -> int:
    """Number of records of a tuning cache, checked on the host."""
    n = _u32()
    _check(_lib.mhr_tuning_file_records(os.fsencode(path), ctypes.byref(n)), "mhr_tuning_file_records")
    return int(n.value)


GATHER_PHASES = ("fetch", "setup", "rows", "probe", "form", "score", "logsig", "bounds", "enum", "merge", "end")


GATHER_COUNTS = ("tiles", "row_batches", "chunks", "scanned", "sub_batches", "matches", "values", "items", "staged",
                 "merges")


def phase_ticks(reset: bool = False, by_kind: bool = False):
    """The gather kernel's per-phase wall-clock ticks summed over workgroups
    (phase-clock build only; see mhr_debug_phase_ticks) as {phase: ticks},
    and the clock rate in Hz.  by_kind: instead a pair of dicts (tiles with
    the probe side in the LDS table, tiles probing through the row
    directory), each holding the phase ticks and the work counts."""
    npz, nct = len(GATHER_PHASES), len(GATHER_COUNTS)
    slots = npz + nct
    buf = (ctypes.c_uint64 * (2 * slots))()
    rate = ctypes.c_double()
    _check(_lib.mhr_debug_phase_ticks(buf, 2 * slots, ctypes.byref(rate), 1 if reset else 0),
           "mhr_debug_phase_ticks")
    kinds = []
    for k in range(2):
        b = k * slots
        d = {p: int(buf[b + i]) for i, p in enumerate(GATHER_PHASES)}
        d.update({c: int(buf[b + npz + i]) for i, c in enumerate(GATHER_COUNTS)})
        kinds.append(d)
    if by_kind:
        return tuple(kinds), float(rate.value)
    return {p: kinds[0][p] + kinds[1][p] for p in GATHER_PHASES}, float(rate.value)


def _table(t, dtype):
    torch = _torch()
    if dtype is None:
        dtype = "f32" if t.dtype == torch.float32 else "bf16"
    return t.contiguous(), (DTYPE_F32 if dtype == "f32" else DTYPE_BF16)


def scan_topk(entity, relation, head, cand, k: int, rel=None, rel_default: int = 0, gamma: float = 1.0,
              cand_stride: int = 0, ncand: Optional[int] = None, dtype: Optional[str] = None, stream=None):
    """TransE-L1 candidate scan (mhr_scan_topk): for each query q the best k
    candidates of its list under gamma - |X[head[q]] + Y[rel[q]] - X[c]|_1
    (FP64).  entity / relation: device tables (float32, or int16/bfloat16
    bit patterns with dtype="bf16").  Returns (ids [nq, k] int32, scores
    [nq, k] float64, status [nq] int32) device tensors."""
    torch = _torch()
    X, code = _table(entity, dtype)
    Y, _ = _table(relation, dtype)
    h = _dev_u32(head)
    c = _dev_u32(cand)
    r = _dev_u32(rel) if rel is not None else None
    nq = h.numel()
    nc = int(c.numel() if ncand is None else ncand)
    need = ctypes.c_size_t()
    _check(_lib.mhr_scan_workspace_size(nq, nc, int(k), ctypes.byref(need)), "mhr_scan_workspace_size")
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device="cuda")
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    sc = torch.empty((nq, k), dtype=torch.float64, device="cuda")
    st = torch.empty(max(nq, 1), dtype=torch.int32, device="cuda")
    _check(_lib.mhr_scan_topk(code, int(X.shape[1]), _ptr(X), _ptr(Y), int(X.shape[0]), int(Y.shape[0]), nq, _ptr(h),
                              _ptr(r), int(rel_default), _ptr(c), nc, int(cand_stride), int(k), float(gamma),
                              _ptr(ids), _ptr(sc), _ptr(st), _ptr(ws), ws.numel(), _stream_ptr(stream)),
           "mhr_scan_topk")
    return ids, sc, st[:nq]


class ScanPipeline:
    """The three-hop award pipeline (mhr_scan_pipeline) with its buffers
    allocated once for npipe runs over fixed person and university lists;
    run() enqueues all three hops on the stream."""

    def __init__(self, entity, relation, persons, universities, k: int, npipe: int = 1, gamma: float = 1.0,
                 dtype: Optional[str] = None):
        torch = _torch()
        self.X, self.code = _table(entity, dtype)
        self.Y, _ = _table(relation, dtype)
        self.persons, self.univ = _dev_u32(persons), _dev_u32(universities)
        self.k, self.npipe, self.gamma = int(k), int(npipe), float(gamma)
        need = ctypes.c_size_t()
        _check(_lib.mhr_scan_pipeline_workspace_size(self.npipe, self.persons.numel(), self.univ.numel(), self.k,
                                                     ctypes.byref(need)), "mhr_scan_pipeline_workspace_size")
        self.ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device="cuda")
        P, K = self.npipe, self.k
        self.hop1_id = torch.empty((P, K), dtype=torch.int32, device="cuda")
        self.hop1_score = torch.empty((P, K), dtype=torch.float64, device="cuda")
        self.hop2_id = torch.empty((P, K), dtype=torch.int32, device="cuda")
        self.hop2_score = torch.empty((P, K), dtype=torch.float64, device="cuda")
        self.hop3_id = torch.empty((P, K, K), dtype=torch.int32, device="cuda")
        self.hop3_score = torch.empty((P, K, K), dtype=torch.float64, device="cuda")

    def run(self, award, field, r_award: int, r_works: int, r_affil: int, stream=None):
        a, f = _dev_u32(award), _dev_u32(field)
        if a.numel() != self.npipe or f.numel() != self.npipe:
            raise ValueError("award and field must hold npipe entities")
        self._keep = (a, f)
        _check(_lib.mhr_scan_pipeline(self.code, int(self.X.shape[1]), _ptr(self.X), _ptr(self.Y),
                                      int(self.X.shape[0]), int(self.Y.shape[0]), self.npipe, _ptr(a), _ptr(f),
                                      int(r_award), int(r_works), int(r_affil), _ptr(self.persons),
                                      self.persons.numel(), _ptr(self.univ), self.univ.numel(), self.k, self.gamma,
                                      _ptr(self.hop1_id), _ptr(self.hop1_score), _ptr(self.hop2_id),
                                      _ptr(self.hop2_score), _ptr(self.hop3_id), _ptr(self.hop3_score),
                                      _ptr(self.ws), self.ws.numel(), _stream_ptr(stream)), "mhr_scan_pipeline")
        return self


class Plan:
    """A batched query call captured once into a HIP graph and replayed with
    one launch.  The plan owns fixed device buffers for the queries
    (``src``, ``dst``, ``k``), the workspace and the results (``out``);
    ``set_queries`` copies a new batch of the same size into them."""

    def __init__(self, graph: Graph, src, dst, k, k_max, opts, stream):
        torch = _torch()
        s, d, kt, nq, o, k_max = Graph._queries(src, dst, k, k_max, opts)
        self.graph = graph
        self.nq, self.k_max, self.opts = nq, k_max, o
        self.src, self.dst = s.clone(), d.clone()
        self.k = kt.clone() if kt is not None else None
        self.ws = torch.empty(graph.workspace_bytes(nq, k_max, o), dtype=torch.uint8, device="cuda")
        self.out = Graph._new_out(nq, k_max)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(_lib.mhr_plan_create(graph._h, ctypes.byref(o), nq, _ptr(self.src), _ptr(self.dst), _ptr(self.k),
                                    k_max, _ptr(self.out.paths), _ptr(self.out.count), _ptr(self.out.total),
                                    _ptr(self.out.status), _ptr(self.ws), self.ws.numel(),
                                    _stream_ptr(stream), ctypes.byref(h)), "mhr_plan_create")
        self._h = h

    def set_queries(self, src, dst, k=None):
        """Writes a new batch (same size) into the plan's query buffers."""
        s, d = _dev_u32(src), _dev_u32(dst)
        if s.numel() != self.nq or d.numel() != self.nq:
            raise ValueError("a plan's batch size is fixed")
        self.src.copy_(s)
        self.dst.copy_(d)
        if k is not None:
            if self.k is None:
                raise ValueError("this plan was captured with one K for all queries")
            self.k.copy_(_dev_u32(k))

    def launch(self, stream=None) -> TopK:
        _check(_lib.mhr_plan_launch(self._h, _stream_ptr(stream)), "mhr_plan_launch")
        return self.out

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.mhr_plan_destroy(self._h), "mhr_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["WideGraph", "WideResult", "WIDE_PATH_DTYPE", "WIDE_MAX_K", "BEAM_DTYPE", "beam_to_numpy", "TrainOpts", "Graph", "Plan", "Pruner", "scan_topk", "ScanPipeline", "crc32", "pruner_file_info", "tuning_file_records", "Candidates", "candidates", "select", "TopK", "QueryOpts", "PhaseEvents", "MhrError", "PATH_DTYPE", "LIB_PATH", "MHR_MAX_K",
           "Q_BAD_ID", "Q_BAD_K", "Q_EXACT_PASS", "PATH_RESCORED", "PATH_PRECISION_TIE"]
