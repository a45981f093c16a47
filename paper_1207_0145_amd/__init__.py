"""P-MPSM equi-join on one AMD Instinct MI355X (gfx950).

Thin ctypes binding of ``libmpsm.so`` (declared in ``include/mpsm.h``).  The
functions here only marshal arguments; every step of the join runs in the
library's HIP kernels.  Torch supplies device memory and the stream.

Tensors: ``[n, 2]`` int64 or uint64 on the GPU, column 0 the key, column 1
the payload (bit patterns are taken as uint64).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpsm.so")

ROLE_AUTO, ROLE_AS_GIVEN, ROLE_SWAP = 0, 1, 2
SPLIT_SAMPLED, SPLIT_LEARNED, SPLIT_COST, SPLIT_NONE = 0, 1, 2, 3
SEARCH_BINARY, SEARCH_INTERP, SEARCH_LEARNED, SEARCH_INDEX = 0, 1, 2, 3
STATUS = {0: "MPSM_OK", 1: "MPSM_EINVAL", 2: "MPSM_ECAPACITY", 3: "MPSM_ENOMEM", 4: "MPSM_EHIP",
          5: "MPSM_EUNSUPPORTED"}

EXPORTS = ("mpsm_config_default", "mpsm_workspace_bytes", "mpsm_join", "mpsm_status_string",
           "mpsm_workspace_layout", "mpsm_join_events", "mpsm_marker_count", "mpsm_marker_name",
           "mpsm_events_create", "mpsm_events_destroy", "mpsm_events_elapsed", "mpsm_batch_create",
           "mpsm_batch_destroy", "mpsm_batch_workspace_bytes", "mpsm_batch_run", "mpsm_batch_autotune",
           "mpsm_batch_get_tuning", "mpsm_batch_set_tuning", "mpsm_clock_hz", "mpsm_join_slices_host",
           "mpsm_join_noalloc", "mpsm_join_batch", "mpsm_join_batch_workspace_bytes",
           "mpsm_lower_bound_window_host", "mpsm_join_host_runs", "mpsm_join_host_runs_workspace_bytes",
           "mpsm_join_spilled_runs", "mpsm_join_spilled_runs_workspace_bytes")


class MpsmConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("role", ctypes.c_int32), ("splitter", ctypes.c_int32),
                ("search", ctypes.c_int32), ("log2_run_len", ctypes.c_uint32), ("bucket_target", ctypes.c_uint32),
                ("join_chunk", ctypes.c_uint32), ("want_max", ctypes.c_uint32), ("oversample", ctypes.c_uint32),
                ("waves", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class MpsmStats(ctypes.Structure):
    _fields_ = [("max_payload_sum", ctypes.c_uint64), ("nonempty", ctypes.c_uint64),
                ("partitions", ctypes.c_uint64), ("runs", ctypes.c_uint64), ("oversize_buckets", ctypes.c_uint64),
                ("search_probes", ctypes.c_uint64), ("swapped", ctypes.c_uint64), ("ms_total", ctypes.c_double),
                ("search_fallbacks", ctypes.c_uint64), ("max_partition", ctypes.c_uint64),
                ("cdf_eps_r", ctypes.c_double), ("cdf_eps_s", ctypes.c_double),
                ("resorted_buckets", ctypes.c_uint64), ("retried_buckets", ctypes.c_uint64),
                ("pairs_truncated", ctypes.c_uint64), ("redone_runs", ctypes.c_uint64),
                ("redone_r_segments", ctypes.c_uint64)]


class MpsmLayout(ctypes.Structure):
    _fields_ = [("swapped", ctypes.c_uint32), ("levels", ctypes.c_uint32), ("run_len", ctypes.c_uint64),
                ("runs", ctypes.c_uint32), ("s_buckets", ctypes.c_uint32), ("r_buckets1", ctypes.c_uint32),
                ("r_buckets2", ctypes.c_uint32), ("s_oversample", ctypes.c_uint32),
                ("r_oversample1", ctypes.c_uint32), ("r_oversample2", ctypes.c_uint32),
                ("s_level_seed", ctypes.c_uint64), ("r_level_seed1", ctypes.c_uint64),
                ("r_level_seed2", ctypes.c_uint64), ("off_s_sorted", ctypes.c_uint64),
                ("off_r_sorted", ctypes.c_uint64), ("off_s_splitters", ctypes.c_uint64),
                ("off_r_splitters1", ctypes.c_uint64), ("off_r_splitters2", ctypes.c_uint64),
                ("off_s_bucket_start", ctypes.c_uint64), ("off_r_bucket_start1", ctypes.c_uint64),
                ("off_r_bucket_start", ctypes.c_uint64), ("off_partitions", ctypes.c_uint64),
                ("off_part_start", ctypes.c_uint64), ("off_part_len", ctypes.c_uint64),
                ("off_part_key", ctypes.c_uint64), ("off_offsets", ctypes.c_uint64), ("p_max", ctypes.c_uint32),
                ("idx_stride", ctypes.c_uint32), ("off_run_index", ctypes.c_uint64),
                ("idx_per_run", ctypes.c_uint32), ("padded_passes", ctypes.c_uint32),
                ("off_join_span", ctypes.c_uint64), ("off_cost_sample", ctypes.c_uint64),
                ("off_cost_s_below", ctypes.c_uint64), ("off_cost_best", ctypes.c_uint64),
                ("cost_cells", ctypes.c_uint32), ("reserved2", ctypes.c_uint32),
                ("off_cdf_model_r", ctypes.c_uint64), ("off_cdf_model_s", ctypes.c_uint64),
                ("cdf_seed_r", ctypes.c_uint64), ("cdf_seed_s", ctypes.c_uint64),
                ("cdf_sample", ctypes.c_uint32), ("cdf_knots", ctypes.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class MpsmJoinDesc(ctypes.Structure):
    _fields_ = [("d_R", ctypes.c_void_p), ("nR", ctypes.c_uint64), ("d_S", ctypes.c_void_p), ("nS", ctypes.c_uint64),
                ("d_out_count", ctypes.c_void_p), ("d_out_checksum", ctypes.c_void_p),
                ("d_out_times", ctypes.c_void_p)]


class MpsmBatchShape(ctypes.Structure):
    _fields_ = [("max_sum_nR", ctypes.c_uint64), ("max_sum_nS", ctypes.c_uint64), ("max_nS", ctypes.c_uint64)]


class MpsmBatchTuning(ctypes.Structure):
    _fields_ = [("log2_run_len", ctypes.c_uint32), ("bucket_target", ctypes.c_uint32),
                ("join_chunk", ctypes.c_uint32), ("from_cache", ctypes.c_uint32), ("ms", ctypes.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1207_0145_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        p, u64 = ctypes.c_void_p, ctypes.c_uint64
        L.mpsm_config_default.argtypes = [ctypes.POINTER(MpsmConfig)]
        L.mpsm_config_default.restype = None
        L.mpsm_workspace_bytes.argtypes = [u64, u64, ctypes.POINTER(MpsmConfig)]
        L.mpsm_workspace_bytes.restype = u64
        L.mpsm_join.argtypes = [p, u64, p, u64, p, p, p, u64, ctypes.POINTER(MpsmConfig), p, u64, p,
                                ctypes.POINTER(MpsmStats)]
        L.mpsm_join.restype = ctypes.c_int
        L.mpsm_status_string.argtypes = [ctypes.c_int]
        L.mpsm_status_string.restype = ctypes.c_char_p
        L.mpsm_workspace_layout.argtypes = [u64, u64, ctypes.POINTER(MpsmConfig), ctypes.POINTER(MpsmLayout)]
        L.mpsm_workspace_layout.restype = ctypes.c_int
        L.mpsm_join_events.argtypes = [p, u64, p, u64, p, p, p, u64, ctypes.POINTER(MpsmConfig), p, u64, p,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32]
        L.mpsm_join_events.restype = ctypes.c_int
        L.mpsm_marker_count.argtypes = []
        L.mpsm_marker_count.restype = ctypes.c_uint32
        L.mpsm_marker_name.argtypes = [ctypes.c_uint32]
        L.mpsm_marker_name.restype = ctypes.c_char_p
        L.mpsm_events_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32]
        L.mpsm_events_create.restype = ctypes.c_int
        L.mpsm_events_destroy.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32]
        L.mpsm_events_destroy.restype = None
        L.mpsm_events_elapsed.argtypes = [p, p, ctypes.POINTER(ctypes.c_float)]
        L.mpsm_events_elapsed.restype = ctypes.c_int
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.mpsm_batch_create.argtypes = [ctypes.POINTER(MpsmJoinDesc), ctypes.c_uint32, ctypes.POINTER(MpsmConfig), pp]
        L.mpsm_batch_create.restype = ctypes.c_int
        L.mpsm_batch_destroy.argtypes = [p]
        L.mpsm_batch_destroy.restype = None
        L.mpsm_batch_workspace_bytes.argtypes = [p]
        L.mpsm_batch_workspace_bytes.restype = u64
        L.mpsm_batch_run.argtypes = [p, p, u64, p, ctypes.c_int]
        L.mpsm_batch_run.restype = ctypes.c_int
        L.mpsm_batch_autotune.argtypes = [p, p, u64, p, ctypes.c_char_p, ctypes.POINTER(MpsmBatchTuning)]
        L.mpsm_batch_autotune.restype = ctypes.c_int
        L.mpsm_batch_get_tuning.argtypes = [p, ctypes.POINTER(MpsmBatchTuning)]
        L.mpsm_batch_get_tuning.restype = ctypes.c_int
        L.mpsm_batch_set_tuning.argtypes = [p, ctypes.POINTER(MpsmBatchTuning)]
        L.mpsm_batch_set_tuning.restype = ctypes.c_int
        L.mpsm_clock_hz.argtypes = []
        L.mpsm_clock_hz.restype = u64
        L.mpsm_join_slices_host.argtypes = [p, p, p, p, ctypes.c_uint32, p, p]
        L.mpsm_join_slices_host.restype = ctypes.c_int
        L.mpsm_lower_bound_window_host.argtypes = [p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                                   ctypes.c_uint64, ctypes.c_uint64, p, p]
        L.mpsm_lower_bound_window_host.restype = ctypes.c_int
        L.mpsm_join_noalloc.argtypes = [p, u64, p, u64, p, p, p, u64, ctypes.POINTER(MpsmConfig), p]
        L.mpsm_join_noalloc.restype = ctypes.c_int
        L.mpsm_join_host_runs_workspace_bytes.argtypes = [u64, u64, ctypes.POINTER(MpsmConfig), u64]
        L.mpsm_join_host_runs_workspace_bytes.restype = u64
        L.mpsm_join_host_runs.argtypes = [p, u64, p, u64, p, p, p, ctypes.POINTER(MpsmConfig), u64, p, u64, p]
        L.mpsm_join_host_runs.restype = ctypes.c_int
        L.mpsm_join_spilled_runs_workspace_bytes.argtypes = [u64, u64, ctypes.POINTER(MpsmConfig)]
        L.mpsm_join_spilled_runs_workspace_bytes.restype = u64
        L.mpsm_join_spilled_runs.argtypes = [p, u64, p, u64, p, p, ctypes.POINTER(MpsmConfig), p, u64, p]
        L.mpsm_join_spilled_runs.restype = ctypes.c_int
        L.mpsm_join_batch_workspace_bytes.argtypes = [ctypes.c_uint32, ctypes.POINTER(MpsmBatchShape),
                                                      ctypes.POINTER(MpsmConfig)]
        L.mpsm_join_batch_workspace_bytes.restype = u64
        L.mpsm_join_batch.argtypes = [p, ctypes.c_uint32, ctypes.POINTER(MpsmBatchShape), ctypes.POINTER(MpsmConfig),
                                      p, u64, p]
        L.mpsm_join_batch.restype = ctypes.c_int
        _lib = L
    return _lib


def config(**kw) -> MpsmConfig:
    """Default configuration with the given fields overridden."""
    c = MpsmConfig()
    lib().mpsm_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def _cfg_ptr(cfg):
    return None if cfg is None else ctypes.byref(cfg)


def workspace_bytes(nR: int, nS: int, cfg: MpsmConfig | None = None) -> int:
    return int(lib().mpsm_workspace_bytes(nR, nS, _cfg_ptr(cfg)))


def layout(nR: int, nS: int, cfg: MpsmConfig | None = None) -> dict:
    out = MpsmLayout()
    rc = lib().mpsm_workspace_layout(nR, nS, _cfg_ptr(cfg), ctypes.byref(out))
    if rc != 0:
        raise ValueError(f"mpsm_workspace_layout: {STATUS.get(rc, rc)}")
    return out.as_dict()


class MpsmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({lib().mpsm_status_string(code).decode()})")


def _check_tuples(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dim() != 2 or t.shape[1] != 2 or t.dtype not in (torch.int64, torch.uint64) or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous [n, 2] int64/uint64 tensor")


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def alloc_workspace(nR: int, nS: int, cfg: MpsmConfig | None = None, device="cuda"):
    import torch
    nbytes = workspace_bytes(nR, nS, cfg)
    if nbytes == 0:
        raise ValueError("unsupported sizes or configuration")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def join_into(R, S, out, workspace, cfg: MpsmConfig | None = None, stream=None, pairs=None,
              stats: MpsmStats | None = None) -> int:
    """Enqueue the join; out is a GPU int64 tensor of >= 2 elements that
    receives (count, checksum); pairs an optional GPU [cap, 3] tensor.
    Returns the status code (raises on errors other than ECAPACITY)."""
    _check_tuples(R, "R")
    _check_tuples(S, "S")
    pp = ctypes.c_void_p(pairs.data_ptr()) if pairs is not None and pairs.numel() else None
    cap = pairs.shape[0] if pp is not None else 0
    rc = lib().mpsm_join(ctypes.c_void_p(R.data_ptr()), R.shape[0], ctypes.c_void_p(S.data_ptr()), S.shape[0],
                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8), pp, cap,
                         _cfg_ptr(cfg), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                         _stream_handle(stream), None if stats is None else ctypes.byref(stats))
    if rc not in (0, 2):
        raise MpsmError(rc, "mpsm_join")
    return rc


# bytes of the library's own per-GPU workspace used by join_noalloc_into
NOALLOC_SCRATCH_BYTES = 64 << 20


def join_noalloc_into(R, S, out, cfg: MpsmConfig | None = None, stream=None, pairs=None) -> int:
    """mpsm_join_noalloc: the join with the library's own fixed workspace
    (no allocation anywhere in the call); out and pairs as in join_into.
    Raises MpsmError(MPSM_ENOMEM) for joins too large for that workspace."""
    _check_tuples(R, "R")
    _check_tuples(S, "S")
    pp = ctypes.c_void_p(pairs.data_ptr()) if pairs is not None and pairs.numel() else None
    cap = pairs.shape[0] if pp is not None else 0
    rc = lib().mpsm_join_noalloc(ctypes.c_void_p(R.data_ptr()), R.shape[0], ctypes.c_void_p(S.data_ptr()),
                                 S.shape[0], ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8),
                                 pp, cap, _cfg_ptr(cfg), _stream_handle(stream))
    if rc != 0:
        raise MpsmError(rc, "mpsm_join_noalloc")
    return rc


def join_host_runs_workspace_bytes(nR: int, nS: int, chunk_tuples: int, cfg: MpsmConfig | None = None) -> int:
    return int(lib().mpsm_join_host_runs_workspace_bytes(nR, nS, _cfg_ptr(cfg), chunk_tuples))


def _check_host_tuples(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.is_cuda or (t.numel() and not t.is_pinned()):
        raise TypeError(f"{name} must be a pinned host tensor")
    if t.dim() != 2 or t.shape[1] != 2 or t.dtype not in (torch.int64, torch.uint64) or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous [n, 2] int64/uint64 tensor")


def join_host_runs_into(R, S_host, runs_host, out, workspace, chunk_tuples: int, cfg: MpsmConfig | None = None,
                        stream=None) -> int:
    """mpsm_join_host_runs: the join with S (and its sorted runs, written to
    runs_host unless it is None) in pinned host memory; R, out and workspace
    on the GPU as in join_into.  Enqueues the work; runs_host is complete once
    the stream is."""
    _check_tuples(R, "R")
    _check_host_tuples(S_host, "S_host")
    if runs_host is not None:
        _check_host_tuples(runs_host, "runs_host")
        if runs_host.shape[0] != S_host.shape[0]:
            raise ValueError("runs_host must hold as many tuples as S_host")
    rc = lib().mpsm_join_host_runs(ctypes.c_void_p(R.data_ptr()), R.shape[0], ctypes.c_void_p(S_host.data_ptr()),
                                   S_host.shape[0], None if runs_host is None else ctypes.c_void_p(runs_host.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8),
                                   _cfg_ptr(cfg), chunk_tuples, ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel(), _stream_handle(stream))
    if rc != 0:
        raise MpsmError(rc, "mpsm_join_host_runs")
    return rc


def join_spilled_runs_workspace_bytes(nR: int, nS: int, cfg: MpsmConfig | None = None) -> int:
    return int(lib().mpsm_join_spilled_runs_workspace_bytes(nR, nS, _cfg_ptr(cfg)))


def join_spilled_runs_into(R, runs_host, out, workspace, cfg: MpsmConfig | None = None, stream=None) -> int:
    """mpsm_join_spilled_runs: R (on the GPU) joined with S's sorted runs
    already in pinned host memory (as join_host_runs_into leaves them);
    out and workspace as in join_into.  Enqueues the work."""
    _check_tuples(R, "R")
    _check_host_tuples(runs_host, "runs_host")
    rc = lib().mpsm_join_spilled_runs(ctypes.c_void_p(R.data_ptr()), R.shape[0],
                                      ctypes.c_void_p(runs_host.data_ptr()), runs_host.shape[0],
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8),
                                      _cfg_ptr(cfg), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                      _stream_handle(stream))
    if rc != 0:
        raise MpsmError(rc, "mpsm_join_spilled_runs")
    return rc


def marker_names() -> list[str]:
    L = lib()
    return [L.mpsm_marker_name(i).decode() for i in range(L.mpsm_marker_count())]


class EventSet:
    """n timing events owned by the library (for mpsm_join_events)."""

    def __init__(self, n: int):
        self.n = n
        self.arr = (ctypes.c_void_p * n)()
        rc = lib().mpsm_events_create(self.arr, n)
        if rc != 0:
            raise MpsmError(rc, "mpsm_events_create")

    def elapsed(self, i: int, j: int) -> float:
        ms = ctypes.c_float(0)
        rc = lib().mpsm_events_elapsed(self.arr[i], self.arr[j], ctypes.byref(ms))
        if rc != 0:
            raise MpsmError(rc, "mpsm_events_elapsed")
        return float(ms.value)

    def close(self):
        if self.arr is not None:
            lib().mpsm_events_destroy(self.arr, self.n)
            self.arr = None


def join_events_into(R, S, out, workspace, events: EventSet, cfg: MpsmConfig | None = None, stream=None) -> int:
    """mpsm_join that records the step markers into `events`."""
    _check_tuples(R, "R")
    _check_tuples(S, "S")
    rc = lib().mpsm_join_events(ctypes.c_void_p(R.data_ptr()), R.shape[0], ctypes.c_void_p(S.data_ptr()),
                                S.shape[0], ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8),
                                None, 0, _cfg_ptr(cfg), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                _stream_handle(stream), events.arr, events.n)
    if rc != 0:
        raise MpsmError(rc, "mpsm_join_events")
    return rc


def join(R, S, cfg: MpsmConfig | None = None, pairs: bool = False, pairs_capacity: int | None = None,
         workspace=None, with_stats: bool = False):
    """Synchronous convenience wrapper.  Returns a dict with count,
    checksum (Python ints, uint64), and optionally pairs (a CPU uint64
    [count, 3] tensor, sorted lexicographically) and stats."""
    import torch
    _check_tuples(R, "R")
    _check_tuples(S, "S")
    dev = R.device
    if workspace is None:
        workspace = alloc_workspace(R.shape[0], S.shape[0], cfg, dev)
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    res = {}
    pbuf = None
    if pairs:
        if pairs_capacity is None:
            first = join(R, S, cfg, workspace=workspace)
            pairs_capacity = first["count"]
        pbuf = torch.zeros((max(pairs_capacity, 1), 3), dtype=torch.int64, device=dev)
    st = MpsmStats() if (with_stats or pairs) else None
    rc = join_into(R, S, out, workspace, cfg, pairs=pbuf, stats=st)
    torch.cuda.synchronize(dev)
    o = out.cpu().tolist()
    res["count"] = o[0] & 0xFFFFFFFFFFFFFFFF
    res["checksum"] = o[1] & 0xFFFFFFFFFFFFFFFF
    res["status"] = STATUS[rc]
    if pairs:
        n = min(res["count"], pairs_capacity)
        import numpy as np
        p = pbuf[:n].cpu().numpy().view(np.uint64)
        order = np.lexsort((p[:, 2], p[:, 1], p[:, 0])) if n else np.zeros(0, np.int64)
        res["pairs"] = p[order]
    if st is not None:
        res["stats"] = {name: getattr(st, name) for name, _ in st._fields_}
    return res


def batch_shape(max_sum_nR: int, max_sum_nS: int, max_nS: int = 0) -> MpsmBatchShape:
    return MpsmBatchShape(max_sum_nR, max_sum_nS, max_nS)


def join_batch_workspace_bytes(n: int, shape: MpsmBatchShape, cfg: MpsmConfig | None = None) -> int:
    return int(lib().mpsm_join_batch_workspace_bytes(n, ctypes.byref(shape), _cfg_ptr(cfg)))


def write_descs(descs, joins, out, times=None):
    """Fill a GPU int64 [n, 7] tensor with the mpsm_join_desc records of
    joins (a list of (R, S) tensors): R, nR, S, nS, &out[i, 0], &out[i, 1],
    &times[i, 0] (or 0).  One host-to-device copy; no join arithmetic."""
    import torch
    rows = []
    for i, (R, S) in enumerate(joins):
        _check_tuples(R, "R")
        _check_tuples(S, "S")
        rows.append([R.data_ptr() if R.shape[0] else 0, R.shape[0], S.data_ptr() if S.shape[0] else 0, S.shape[0],
                     out.data_ptr() + 16 * i, out.data_ptr() + 16 * i + 8,
                     times.data_ptr() + 24 * i if times is not None else 0])
    descs.copy_(torch.tensor(rows, dtype=torch.int64).reshape(descs.shape))


def join_batch(descs, n: int, shape: MpsmBatchShape, workspace, cfg: MpsmConfig | None = None, stream=None) -> int:
    """mpsm_join_batch over the device descriptor array `descs` (a GPU
    int64 [n, 7] tensor, see write_descs); enqueues only."""
    rc = lib().mpsm_join_batch(ctypes.c_void_p(descs.data_ptr()), n, ctypes.byref(shape), _cfg_ptr(cfg),
                               ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_handle(stream))
    if rc != 0:
        raise MpsmError(rc, "mpsm_join_batch")
    return rc


class Batch:
    """A batch of independent joins run as one launch sequence
    (mpsm_batch_*).  joins: list of (R, S) tensors (``[n, 2]`` on the GPU,
    n may be 0).  Results land in ``self.out`` (int64 [n_joins, 2]: count,
    checksum) and ``self.times`` (int64 [n_joins, 3] GPU wall-clock ticks:
    batch start, first work item, last work item)."""

    def __init__(self, joins, cfg: MpsmConfig | None = None, device=None):
        import torch
        self.joins = list(joins)
        dev = device or (self.joins[0][0].device if self.joins else torch.device("cuda", 0))
        self.out = torch.zeros((len(self.joins), 2), dtype=torch.int64, device=dev)
        self.times = torch.zeros((len(self.joins), 3), dtype=torch.int64, device=dev)
        descs = (MpsmJoinDesc * len(self.joins))()
        for i, (R, S) in enumerate(self.joins):
            _check_tuples(R, "R")
            _check_tuples(S, "S")
            d = descs[i]
            d.d_R = R.data_ptr() if R.shape[0] else None
            d.nR = R.shape[0]
            d.d_S = S.data_ptr() if S.shape[0] else None
            d.nS = S.shape[0]
            d.d_out_count = self.out.data_ptr() + 16 * i
            d.d_out_checksum = self.out.data_ptr() + 16 * i + 8
            d.d_out_times = self.times.data_ptr() + 24 * i
        self.handle = ctypes.c_void_p()
        rc = lib().mpsm_batch_create(descs, len(self.joins), _cfg_ptr(cfg), ctypes.byref(self.handle))
        if rc != 0:
            raise MpsmError(rc, "mpsm_batch_create")
        nbytes = int(lib().mpsm_batch_workspace_bytes(self.handle))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    def run(self, use_graph: bool = False, stream=None):
        rc = lib().mpsm_batch_run(self.handle, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                  _stream_handle(stream), 1 if use_graph else 0)
        if rc != 0:
            raise MpsmError(rc, "mpsm_batch_run")

    def autotune(self, cache_path: str | None = None, stream=None) -> dict:
        t = MpsmBatchTuning()
        rc = lib().mpsm_batch_autotune(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), _stream_handle(stream),
                                       cache_path.encode() if cache_path else None, ctypes.byref(t))
        if rc != 0:
            raise MpsmError(rc, "mpsm_batch_autotune")
        return t.as_dict()

    def tuning(self) -> dict:
        t = MpsmBatchTuning()
        rc = lib().mpsm_batch_get_tuning(self.handle, ctypes.byref(t))
        if rc != 0:
            raise MpsmError(rc, "mpsm_batch_get_tuning")
        return t.as_dict()

    def set_tuning(self, log2_run_len: int, bucket_target: int, join_chunk: int):
        t = MpsmBatchTuning(log2_run_len, bucket_target, join_chunk, 0, 0.0)
        rc = lib().mpsm_batch_set_tuning(self.handle, ctypes.byref(t))
        if rc != 0:
            raise MpsmError(rc, "mpsm_batch_set_tuning")

    def results(self):
        """[(count, checksum)] as Python uint64 ints (synchronises)."""
        return [(c & 0xFFFFFFFFFFFFFFFF, s & 0xFFFFFFFFFFFFFFFF) for c, s in self.out.cpu().tolist()]

    def close(self):
        if self.handle:
            lib().mpsm_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def clock_hz() -> int:
    return int(lib().mpsm_clock_hz())


def join_slices_host(oa, ob, run_start, run_len):
    """The join kernel's slice plan, run on the host (no GPU): returns
    (cum[Q + 1], sbase[Q]) as numpy uint32 arrays."""
    import numpy as np
    arrs = [np.ascontiguousarray(a, dtype=np.uint32) for a in (oa, ob, run_start, run_len)]
    Q = len(arrs[0])
    cum = np.zeros(Q + 1, np.uint32)
    sbase = np.zeros(max(Q, 1), np.uint32)
    rc = lib().mpsm_join_slices_host(*[ctypes.c_void_p(a.ctypes.data) for a in arrs], Q,
                                     ctypes.c_void_p(cum.ctypes.data), ctypes.c_void_p(sbase.ctypes.data))
    if rc != 0:
        raise MpsmError(rc, "mpsm_join_slices_host")
    return cum, sbase[:Q]


def lower_bound_window_host(keys, a, b, klo, khi, key):
    """The start search's last step, run on the host (no GPU): (lower bound
    of key in keys[a, b), lines probed)."""
    import numpy as np
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    out, pr = ctypes.c_uint32(0), ctypes.c_uint32(0)
    rc = lib().mpsm_lower_bound_window_host(ctypes.c_void_p(k.ctypes.data if len(k) else 0), a, b, klo, khi, key,
                                            ctypes.byref(out), ctypes.byref(pr))
    if rc != 0:
        raise MpsmError(rc, "mpsm_lower_bound_window_host")
    return out.value, pr.value
