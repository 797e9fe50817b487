"""Python binding of librpq (MI355X / gfx950 regular path queries).

A thin ctypes layer over the C ABI declared in ``include/rpq.h``: the
functions carry the same names and only marshal arguments.  Device buffers
are torch tensors on the current HIP device and every call runs on torch's
current stream; all work happens in the library's HIP kernels.

uint32 device data is held in ``torch.int32`` tensors and uint64 keys in
``torch.int64`` tensors (same bits).  Result keys are ``(src << 32) | dst``.

There is no fallback: if the library is not built, or no GPU is visible,
the functions raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

__all__ = [
    "RpqError", "library_path", "load_library", "rpq_abi_version", "rpq_last_error", "rpq_nfa_compile",
    "rpq_nfa_reverse", "rpq_graph_create", "rpq_graph_destroy", "rpq_graph_info_get",
    "rpq_graph_export_csr", "rpq_eval_workspace_size", "rpq_eval", "rpq_eval_noalloc", "rpq_eval_stream", "rpq_eval_split",
    "rpq_nfa_append_label", "SplitInfo",
    "EvalResult", "Graph",
    "Nfa", "EvalOpts", "RPQ_NOALLOC_SCRATCH_BYTES",
    "RPQ_OK", "RPQ_EINVAL", "RPQ_ENOMEM", "RPQ_EOVERFLOW", "RPQ_EDEVICE", "RPQ_EUNSUPPORTED", "RPQ_ECANCELED",
    "RPQ_BUILD_IN_CSR", "RPQ_PAIRS", "RPQ_PER_SOURCE", "RPQ_ALL_SOURCES", "RPQ_REVERSE", "RPQ_SPARSE",
    "RPQ_LENGTH_BOUND", "rpq_batch_bound_length", "RPQ_VISIT_TWO_READS", "RPQ_VISIT_SEEN_OR",
    "RPQ_MAX_STATES", "RPQ_MAX_LABELS", "EXPORTED_SYMBOLS", "rpq_profile_enable", "rpq_profile_read",
    "Batch", "rpq_batch_create", "rpq_batch_destroy", "rpq_batch_add", "rpq_batch_workspace_size",
    "rpq_batch_run", "rpq_batch_result", "rpq_batch_stats", "rpq_batch_autotune",
    "crpq_eval", "CrpqOutput", "CrpqAtom", "CrpqVars", "CrpqResult", "CRPQ_FORCE_DENSE", "CRPQ_FORCE_SPARSE",
    "CRPQ_NO_EDGE_SCAN", "CRPQ_NO_REVERSE", "CRPQ_BATCH_ATOMS", "CRPQ_STRATEGY_EDGE_SCAN", "CRPQ_STRATEGY_DENSE",
    "CRPQ_STRATEGY_BATCHED",
    "CRPQ_STRATEGY_SPARSE", "CRPQ_STRATEGY_REVERSED", "Server", "Request", "Ticket", "ServerOpts", "ServerStats",
    "RPQ_REQ_RPQ", "RPQ_REQ_CRPQ",
]

_HERE = os.path.dirname(os.path.abspath(__file__))

RPQ_ECANCELED = -6
RPQ_OK, RPQ_EINVAL, RPQ_ENOMEM, RPQ_EOVERFLOW, RPQ_EDEVICE, RPQ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RPQ_BUILD_IN_CSR = 1
RPQ_PAIRS, RPQ_PER_SOURCE, RPQ_ALL_SOURCES, RPQ_REVERSE, RPQ_SPARSE, RPQ_LENGTH_BOUND = 1, 2, 4, 8, 16, 32
RPQ_MAX_STATES, RPQ_MAX_LABELS = 32, 64
RPQ_NOALLOC_SCRATCH_BYTES = 256 << 20
RPQ_VISIT_TWO_READS, RPQ_VISIT_SEEN_OR = 1, 2

_STATUS = {0: "RPQ_OK", -1: "RPQ_EINVAL", -2: "RPQ_ENOMEM", -3: "RPQ_EOVERFLOW", -4: "RPQ_EDEVICE",
           -5: "RPQ_EUNSUPPORTED", -6: "RPQ_ECANCELED"}


class RpqError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(code, str(code)), message))
        self.code = code


class Nfa(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_uint32), ("n_labels", ctypes.c_uint32),
                ("initial_mask", ctypes.c_uint32), ("final_mask", ctypes.c_uint32),
                ("delta", ctypes.c_uint32 * (RPQ_MAX_STATES * RPQ_MAX_LABELS))]

    def successors(self, q: int, l: int) -> int:
        return int(self.delta[q * RPQ_MAX_LABELS + l])


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint32), ("n_labels", ctypes.c_uint32),
                ("n_edges_in", ctypes.c_uint64), ("n_edges", ctypes.c_uint64),
                ("edges_per_label", ctypes.c_uint64 * RPQ_MAX_LABELS), ("nonempty_rows", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("has_in_csr", ctypes.c_uint32),
                ("has_vertex_labels", ctypes.c_uint32)]


class EvalOpts(ctypes.Structure):
    _fields_ = [("batch_width", ctypes.c_uint32), ("concurrency", ctypes.c_uint32),
                ("sync_every", ctypes.c_uint32), ("chunk_edges", ctypes.c_uint32),
                ("max_length", ctypes.c_uint32), ("visit", ctypes.c_uint32)]


class Profile(ctypes.Structure):
    _fields_ = [("expand_launches", ctypes.c_uint64), ("expand_ms", ctypes.c_double),
                ("finalize_launches", ctypes.c_uint64), ("finalize_ms", ctypes.c_double),
                ("edge_items", ctypes.c_uint64), ("descriptors", ctypes.c_uint64), ("row_words", ctypes.c_uint64),
                ("word_reads", ctypes.c_uint64), ("word_updates", ctypes.c_uint64),
                ("finalize_rows", ctypes.c_uint64), ("finalize_row_words", ctypes.c_uint64),
                ("finalize_words", ctypes.c_uint64), ("finalize_vis_words", ctypes.c_uint64),
                ("finalize_ans_words", ctypes.c_uint64), ("extract_launches", ctypes.c_uint64),
                ("extract_ms", ctypes.c_double), ("extract_words", ctypes.c_uint64),
                ("expand_extra_words", ctypes.c_uint64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("batch_width", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("chunk_edges", ctypes.c_uint32),
                ("list_share", ctypes.c_uint32), ("visit", ctypes.c_uint32)]


class SplitInfo(ctypes.Structure):
    _fields_ = [("head_pairs", ctypes.c_uint64), ("middle_vertices", ctypes.c_uint64),
                ("tail_pairs", ctypes.c_uint64), ("derived_edges", ctypes.c_uint64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_uint32), ("n_units", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("batch_width", ctypes.c_uint32), ("blocks", ctypes.c_uint32), ("visit", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("edge_items", ctypes.c_uint64), ("descriptors", ctypes.c_uint64), ("word_reads", ctypes.c_uint64),
                ("word_updates", ctypes.c_uint64), ("finalized_rows", ctypes.c_uint64),
                ("finalized_words", ctypes.c_uint64), ("touch_words", ctypes.c_uint64), ("row_words", ctypes.c_uint64),
                ("last_run_ms", ctypes.c_double), ("last_kernel_ms", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 8)]


PairSink = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64, ctypes.c_void_p)


class _PairStream(ctypes.Structure):
    _fields_ = [("device_chunks", ctypes.c_void_p), ("host_chunks", ctypes.c_void_p), ("chunk_keys", ctypes.c_uint64),
                ("sink", PairSink), ("user", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("per_source", ctypes.c_void_p),
                ("pair_offset", ctypes.c_uint64), ("written", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("hash", ctypes.c_uint64), ("product_edges", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("max_depth", ctypes.c_uint64), ("workspace_needed", ctypes.c_uint64)]


CRPQ_MAX_VARS = 16
CRPQ_MAX_ATOMS = 16
CRPQ_FORCE_DENSE, CRPQ_FORCE_SPARSE, CRPQ_NO_EDGE_SCAN, CRPQ_NO_REVERSE, CRPQ_BATCH_ATOMS = 1, 2, 4, 8, 16
CRPQ_STRATEGY_EDGE_SCAN, CRPQ_STRATEGY_DENSE, CRPQ_STRATEGY_SPARSE, CRPQ_STRATEGY_REVERSED = 1, 2, 3, 0x100
CRPQ_STRATEGY_BATCHED = 0x200


class CrpqAtom(ctypes.Structure):
    _fields_ = [("src_var", ctypes.c_uint32), ("dst_var", ctypes.c_uint32), ("nfa", Nfa)]


class CrpqVars(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_uint32), ("binding", ctypes.POINTER(ctypes.c_int64)),
                ("vertex_label", ctypes.POINTER(ctypes.c_int32)), ("domain", ctypes.POINTER(ctypes.c_void_p)),
                ("domain_size", ctypes.POINTER(ctypes.c_uint64)), ("neq", ctypes.POINTER(ctypes.c_uint32)),
                ("n_neq", ctypes.c_uint32)]


class CrpqResult(ctypes.Structure):
    _fields_ = [("tuples", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("hash", ctypes.c_uint64), ("written", ctypes.c_uint64), ("n_free", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("workspace_needed", ctypes.c_uint64),
                ("atom_pairs", ctypes.c_uint64 * CRPQ_MAX_ATOMS), ("atom_strategy", ctypes.c_uint32 * CRPQ_MAX_ATOMS),
                ("join_rows", ctypes.c_uint64)]


RPQ_REQ_RPQ, RPQ_REQ_CRPQ = 1, 2


class ServerOpts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("resident_slots", ctypes.c_uint32),
                ("resident_width", ctypes.c_uint32), ("resident_states", ctypes.c_uint32),
                ("resident_succ", ctypes.c_uint32), ("resident_iters", ctypes.c_uint32),
                ("resident_max_units", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("arrival_ms", ctypes.c_double),
                ("nfa", Nfa), ("sources", ctypes.c_void_p), ("n_sources", ctypes.c_uint64),
                ("pairs", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("per_source", ctypes.c_void_p),
                ("atoms", ctypes.POINTER(CrpqAtom)), ("n_atoms", ctypes.c_uint32), ("vars", CrpqVars),
                ("tuples", ctypes.c_void_p), ("tuple_capacity", ctypes.c_uint64)]


class Ticket(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("done", ctypes.c_uint32), ("count", ctypes.c_uint64),
                ("hash", ctypes.c_uint64), ("product_edges", ctypes.c_uint64), ("written", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64), ("arrival_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("end_ms", ctypes.c_double), ("resident", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "failed", "queued", "running",
                                                "pool_bytes", "pool_in_use", "pool_peak", "product_edges",
                                                "resident_completed", "resident_launches", "resident_bytes")]


# Every symbol include/rpq.h declares (checked by the CPU test suite).
EXPORTED_SYMBOLS = [
    "rpq_last_error", "rpq_abi_version", "rpq_graph_create", "rpq_graph_destroy", "rpq_graph_info_get",
    "rpq_graph_export_csr", "rpq_nfa_compile", "rpq_nfa_reverse", "rpq_eval_workspace_size", "rpq_eval",
    "rpq_eval_noalloc", "rpq_eval_stream", "rpq_eval_split", "rpq_nfa_append_label", "rpq_profile_enable",
    "rpq_profile_read",
    "rpq_batch_create", "rpq_batch_destroy", "rpq_batch_add", "rpq_batch_workspace_size", "rpq_batch_run",
    "rpq_batch_result", "rpq_batch_stats", "rpq_batch_autotune", "rpq_batch_bound_length",
    "crpq_eval", "rpq_serve_start", "rpq_serve_submit", "rpq_serve_poll", "rpq_serve_wait", "rpq_serve_clock_ms",
    "rpq_serve_stats", "rpq_serve_stop",
]

_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "_build", "librpq.so")


def load_library():
    """Load librpq.so (built by ``python -m paper_2602_20748_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError("librpq.so is not built (%s); run: python -m paper_2602_20748_amd.build" % path)
    lib = ctypes.CDLL(path)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    sig = {
        "rpq_last_error": (ctypes.c_char_p, []),
        "rpq_abi_version": (ctypes.c_int, []),
        "rpq_graph_create": (ctypes.c_int, [vp, vp, vp, u64, u32, u32, vp, u32, vp, ctypes.POINTER(vp)]),
        "rpq_graph_destroy": (ctypes.c_int, [vp]),
        "rpq_graph_info_get": (ctypes.c_int, [vp, ctypes.POINTER(GraphInfo)]),
        "rpq_graph_export_csr": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
        "rpq_nfa_compile": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p), u32,
                                           ctypes.POINTER(Nfa)]),
        "rpq_nfa_reverse": (ctypes.c_int, [ctypes.POINTER(Nfa), ctypes.POINTER(Nfa)]),
        "rpq_eval_workspace_size": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), u64, u32, ctypes.POINTER(EvalOpts),
                                                   ctypes.POINTER(u64)]),
        "rpq_eval": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), vp, u64, u32, ctypes.POINTER(EvalOpts), vp, u64,
                                    ctypes.POINTER(_Result), vp]),
        "rpq_eval_noalloc": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), vp, u64, u32, ctypes.POINTER(EvalOpts),
                                             ctypes.POINTER(_Result), vp]),
        "rpq_eval_stream": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), vp, u64, u32, ctypes.POINTER(EvalOpts), vp, u64,
                                            ctypes.POINTER(_PairStream), ctypes.POINTER(_Result), vp]),
        "rpq_eval_split": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), ctypes.POINTER(Nfa), vp, u64, u32,
                                          ctypes.POINTER(EvalOpts), vp, ctypes.POINTER(SplitInfo), vp]),
        "rpq_nfa_append_label": (ctypes.c_int, [ctypes.POINTER(Nfa), u32, ctypes.POINTER(Nfa)]),
        "rpq_profile_enable": (ctypes.c_int, [ctypes.c_int]),
        "rpq_batch_create": (ctypes.c_int, [vp, ctypes.POINTER(BatchOpts), ctypes.POINTER(vp)]),
        "rpq_batch_destroy": (ctypes.c_int, [vp]),
        "rpq_batch_add": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), vp, u64, u32, vp, u64, vp,
                                         ctypes.POINTER(u32)]),
        "rpq_batch_workspace_size": (ctypes.c_int, [vp, ctypes.POINTER(u64)]),
        "rpq_batch_bound_length": (ctypes.c_int, [vp, u32, u32]),
        "rpq_batch_run": (ctypes.c_int, [vp, vp, u64, vp]),
        "rpq_batch_result": (ctypes.c_int, [vp, u32, ctypes.POINTER(_Result)]),
        "rpq_batch_stats": (ctypes.c_int, [vp, ctypes.POINTER(BatchInfo)]),
        "rpq_batch_autotune": (ctypes.c_int, [vp, ctypes.POINTER(BatchOpts), u32, vp, u64, vp,
                                              ctypes.POINTER(BatchOpts)]),
        "rpq_profile_read": (ctypes.c_int, [ctypes.POINTER(Profile), ctypes.c_int]),
        "crpq_eval": (ctypes.c_int, [vp, ctypes.POINTER(CrpqAtom), u32, ctypes.POINTER(CrpqVars), u32, vp, u64,
                                     ctypes.POINTER(CrpqResult), vp]),
        "rpq_serve_start": (ctypes.c_int, [vp, ctypes.POINTER(ServerOpts), vp, u64, ctypes.POINTER(vp)]),
        "rpq_serve_submit": (ctypes.c_int, [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]),
        "rpq_serve_poll": (ctypes.c_int, [vp, u64, ctypes.POINTER(Ticket)]),
        "rpq_serve_wait": (ctypes.c_int, [vp, u64, ctypes.POINTER(Ticket)]),
        "rpq_serve_clock_ms": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double)]),
        "rpq_serve_stats": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
        "rpq_serve_stop": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def rpq_last_error() -> str:
    return load_library().rpq_last_error().decode("utf-8", "replace")


def _check(rc: int, allow=()):
    if rc != RPQ_OK and rc not in allow:
        raise RpqError(rc, rpq_last_error())
    return rc


def rpq_abi_version() -> int:
    return int(load_library().rpq_abi_version())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible; librpq needs an MI355X (gfx950)")
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_u32(x, torch):
    """uint32 data as a contiguous int32 CUDA tensor (same bits)."""
    import numpy as np
    if isinstance(x, torch.Tensor):
        t = x if x.dtype == torch.int32 else x.to(torch.int64).to(torch.int32)
        return t.contiguous().cuda()
    a = np.ascontiguousarray(np.asarray(x).astype(np.uint32)).view(np.int32)
    return torch.from_numpy(a.copy()).cuda()


def _dev_u8(x, torch):
    import numpy as np
    if isinstance(x, torch.Tensor):
        return x.to(torch.uint8).contiguous().cuda()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x).astype(np.uint8)).copy()).cuda()


# ------------------------------------------------------------------------------------------------
# automata
# ------------------------------------------------------------------------------------------------

def rpq_nfa_compile(regex: str, label_names: Sequence[str]) -> Nfa:
    lib = load_library()
    names = (ctypes.c_char_p * len(label_names))(*[n.encode("utf-8") for n in label_names])
    out = Nfa()
    _check(lib.rpq_nfa_compile(regex.encode("utf-8"), names, len(label_names), ctypes.byref(out)))
    return out


def rpq_nfa_reverse(nfa: Nfa) -> Nfa:
    out = Nfa()
    _check(load_library().rpq_nfa_reverse(ctypes.byref(nfa), ctypes.byref(out)))
    return out


# ------------------------------------------------------------------------------------------------
# graph
# ------------------------------------------------------------------------------------------------

class Graph:
    """Owner of an rpq_graph_t handle."""

    def __init__(self, handle: int, names: Optional[List[str]]):
        self.handle = ctypes.c_void_p(handle)
        self.names = names
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle is not None and self.handle.value:
            self._ws.clear()
            load_library().rpq_graph_destroy(self.handle)
        self.handle = None

    def info(self) -> dict:
        return rpq_graph_info_get(self)

    def release_workspace(self) -> None:
        """Drop the cached workspace (the memory returns to torch's allocator)."""
        self._ws.clear()

    def workspace(self, nbytes: int):
        """A cached device workspace of at least nbytes (grown on demand)."""
        torch = _torch()
        cur = self._ws.get("ws")
        if cur is None or cur.numel() < nbytes:
            self._ws["ws"] = None
            cur = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
            self._ws["ws"] = cur
        return cur


def rpq_graph_create(src, label, dst, n_vertices: int, n_labels: int, vertex_label=None, flags: int = 0,
                     names: Optional[Sequence[str]] = None, stream=None) -> Graph:
    """Build the device CSR from an edge list (numpy arrays or torch tensors)."""
    torch = _torch()
    s = _dev_u32(src, torch)
    d = _dev_u32(dst, torch)
    l = _dev_u8(label, torch)
    if not (s.numel() == d.numel() == l.numel()):
        raise ValueError("src, label and dst must have the same length")
    vl = _dev_u8(vertex_label, torch) if vertex_label is not None else None
    h = ctypes.c_void_p()
    _check(load_library().rpq_graph_create(
        s.data_ptr() if s.numel() else None, l.data_ptr() if l.numel() else None,
        d.data_ptr() if d.numel() else None, s.numel(), n_vertices, n_labels,
        vl.data_ptr() if vl is not None else None, flags, _stream(stream), ctypes.byref(h)))
    return Graph(h.value, list(names) if names is not None else None)


def rpq_graph_destroy(g: Graph) -> None:
    g.close()


def rpq_graph_info_get(g: Graph) -> dict:
    info = GraphInfo()
    _check(load_library().rpq_graph_info_get(g.handle, ctypes.byref(info)))
    L = info.n_labels
    return dict(n_vertices=info.n_vertices, n_labels=L, n_edges_in=info.n_edges_in, n_edges=info.n_edges,
                edges_per_label=[int(info.edges_per_label[i]) for i in range(L)],
                nonempty_rows=info.nonempty_rows, device_bytes=info.device_bytes,
                has_in_csr=bool(info.has_in_csr), has_vertex_labels=bool(info.has_vertex_labels))


def rpq_graph_export_csr(g: Graph, reverse: bool = False, stream=None):
    """(row_ptr, dst) as int32 CUDA tensors (uint32 bits)."""
    torch = _torch()
    info = rpq_graph_info_get(g)
    rp = torch.empty(info["n_vertices"] * info["n_labels"] + 1, dtype=torch.int32, device="cuda")
    ds = torch.empty(max(info["n_edges"], 1), dtype=torch.int32, device="cuda")
    _check(load_library().rpq_graph_export_csr(g.handle, 1 if reverse else 0, rp.data_ptr(), ds.data_ptr(),
                                               _stream(stream)))
    return rp, ds[: info["n_edges"]]


# ------------------------------------------------------------------------------------------------
# evaluation
# ------------------------------------------------------------------------------------------------

@dataclasses.dataclass
class EvalResult:
    count: int
    hash: int
    product_edges: int
    levels: int
    max_depth: int
    written: int
    pairs: object = None        # torch.int64 CUDA tensor [written] or None
    per_source: object = None   # torch.int64 CUDA tensor [n_sources, 2] or None
    status: int = RPQ_OK


def _fill(st, fields) -> None:
    """Set the named integer fields of a ctypes struct; an unknown name is an error."""
    names = {f[0] for f in type(st)._fields_}
    for k, v in dict(fields).items():
        if k not in names:
            raise ValueError("unknown %s field %r" % (type(st).__name__, k))
        setattr(st, k, int(v))


def _opts(opts) -> Optional[EvalOpts]:
    if opts is None:
        return None
    if isinstance(opts, EvalOpts):
        return opts
    o = EvalOpts()
    _fill(o, opts)
    return o


def rpq_eval_workspace_size(g: Graph, nfa: Nfa, n_sources: int, flags: int, opts=None) -> int:
    n = ctypes.c_uint64()
    o = _opts(opts)
    _check(load_library().rpq_eval_workspace_size(g.handle, ctypes.byref(nfa), n_sources, flags,
                                                  ctypes.byref(o) if o is not None else None, ctypes.byref(n)))
    return int(n.value)


def rpq_eval(g: Graph, nfa: Nfa, sources=None, flags: int = 0, opts=None, pairs=None, capacity: Optional[int] = None,
             pair_offset: int = 0, per_source=None, workspace=None, stream=None,
             allow_overflow: bool = False, max_length: Optional[int] = None) -> EvalResult:
    """Evaluate one RPQ.

    sources: CUDA/numpy uint32 ids (strictly ascending) or None with RPQ_ALL_SOURCES.
    pairs: a CUDA int64 tensor to receive keys (capacity = its length), or
      True to allocate one of exactly the needed size (two passes), or None.
    per_source: a CUDA int64 tensor [n, 2], or True to allocate one.
    max_length: only walks of at most this many edges count (RPQ_LENGTH_BOUND).
    """
    torch = _torch()
    lib = load_library()
    if max_length is not None:
        opts = dict(opts or {}) if not isinstance(opts, EvalOpts) else {k: getattr(opts, k) for k, _ in
                                                                          EvalOpts._fields_}
        opts["max_length"] = int(max_length)
        flags |= RPQ_LENGTH_BOUND
    if sources is None:
        flags |= RPQ_ALL_SOURCES
        src_t = None
        n = rpq_graph_info_get(g)["n_vertices"]
    else:
        src_t = _dev_u32(sources, torch)
        n = src_t.numel()
    o = _opts(opts)
    if per_source is True:
        per_source = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    if per_source is not None:
        flags |= RPQ_PER_SOURCE
    if pairs is True:
        first = rpq_eval(g, nfa, src_t, flags & ~RPQ_PAIRS, o, None, None, 0, per_source, workspace, stream)
        pairs = torch.empty(max(first.count - pair_offset, 1), dtype=torch.int64, device="cuda")
        capacity = max(first.count - pair_offset, 0)
    if pairs is not None:
        flags |= RPQ_PAIRS
        if capacity is None:
            capacity = pairs.numel()
    need = ctypes.c_uint64()
    _check(lib.rpq_eval_workspace_size(g.handle, ctypes.byref(nfa), n, flags,
                                       ctypes.byref(o) if o is not None else None, ctypes.byref(need)))
    ws_bytes = int(need.value)
    for _ in range(16):
        ws = workspace if workspace is not None else g.workspace(ws_bytes)
        res = _Result()
        res.pairs = pairs.data_ptr() if pairs is not None else None
        res.capacity = int(capacity or 0)
        res.per_source = per_source.data_ptr() if per_source is not None else None
        res.pair_offset = int(pair_offset)
        rc = lib.rpq_eval(g.handle, ctypes.byref(nfa), src_t.data_ptr() if (src_t is not None and n) else None, n,
                          flags, ctypes.byref(o) if o is not None else None, ws.data_ptr(), ws.numel(),
                          ctypes.byref(res), _stream(stream))
        # the sparse search asks for more room when the sources reach more than it planned for
        if rc == RPQ_ENOMEM and workspace is None and res.workspace_needed > ws.numel():
            ws_bytes = int(res.workspace_needed)
            continue
        break
    _check(rc, allow=(RPQ_EOVERFLOW,) if allow_overflow else ())
    out_pairs = pairs[: res.written] if pairs is not None else None
    return EvalResult(int(res.count), int(res.hash), int(res.product_edges), int(res.levels), int(res.max_depth),
                      int(res.written), out_pairs, per_source, rc)


def rpq_eval_stream(g: Graph, nfa: Nfa, sink, sources=None, flags: int = 0, opts=None, chunk_keys: int = 1 << 20,
                    per_source=None, workspace=None, stream=None, max_length: Optional[int] = None) -> EvalResult:
    """Evaluate one RPQ and stream its sorted keys to `sink(keys)`, a numpy uint64 view of one chunk
    (valid only during the call; copy what you keep).  sink returns None/False to go on, True to stop
    (RPQ_ECANCELED).  Chunk buffers: two device chunks (torch) and two pinned host chunks of
    chunk_keys keys each, allocated here; the library allocates nothing for them.
    Returns the EvalResult with written = keys delivered."""
    import numpy as np
    torch = _torch()
    lib = load_library()
    if max_length is not None:
        opts = dict(opts or {}) if not isinstance(opts, EvalOpts) else {k: getattr(opts, k) for k, _ in
                                                                          EvalOpts._fields_}
        opts["max_length"] = int(max_length)
        flags |= RPQ_LENGTH_BOUND
    if sources is None:
        flags |= RPQ_ALL_SOURCES
        src_t = None
        n = rpq_graph_info_get(g)["n_vertices"]
    else:
        src_t = _dev_u32(sources, torch)
        n = src_t.numel()
    o = _opts(opts)
    if per_source is True:
        per_source = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    if per_source is not None:
        flags |= RPQ_PER_SOURCE
    need = ctypes.c_uint64()
    _check(lib.rpq_eval_workspace_size(g.handle, ctypes.byref(nfa), n, flags | RPQ_PAIRS,
                                       ctypes.byref(o) if o is not None else None, ctypes.byref(need)))
    ws = workspace if workspace is not None else g.workspace(int(need.value))
    dev_chunks = torch.empty(2 * int(chunk_keys), dtype=torch.int64, device="cuda")
    host_chunks = torch.empty(2 * int(chunk_keys), dtype=torch.int64, pin_memory=True)
    errors = []

    def _cb(ptr, n_keys, _user):
        try:
            keys = np.ctypeslib.as_array(ptr, shape=(int(n_keys),))
            return 1 if sink(keys) else 0
        except BaseException as e:   # an exception stops the evaluation and is raised afterwards
            errors.append(e)
            return 1

    cb = PairSink(_cb)
    out = _PairStream(dev_chunks.data_ptr(), host_chunks.data_ptr(), int(chunk_keys), cb, None)
    res = _Result()
    res.per_source = per_source.data_ptr() if per_source is not None else None
    rc = lib.rpq_eval_stream(g.handle, ctypes.byref(nfa), src_t.data_ptr() if (src_t is not None and n) else None, n,
                             flags, ctypes.byref(o) if o is not None else None, ws.data_ptr(), ws.numel(),
                             ctypes.byref(out), ctypes.byref(res), _stream(stream))
    if errors:
        raise errors[0]
    _check(rc)
    return EvalResult(int(res.count), int(res.hash), int(res.product_edges), int(res.levels), int(res.max_depth),
                      int(res.written), None, per_source, rc)


def rpq_nfa_append_label(nfa: Nfa, label: int) -> Nfa:
    out = Nfa()
    _check(load_library().rpq_nfa_append_label(ctypes.byref(nfa), int(label), ctypes.byref(out)))
    return out


def rpq_eval_split(g: Graph, head: Nfa, tail: Nfa, sources=None, opts=None, pairs=None, per_source=None,
                   stream=None, allow_overflow: bool = False):
    """R(head . tail) through the materialized R(tail) from the middle vertices (rpq_eval_split).

    pairs: a CUDA int64 tensor (capacity = its length), or True for one of exactly the needed
    size (the plan runs twice), or None.  per_source: a CUDA int64 tensor [n, 2], or True.
    Returns (EvalResult, info dict)."""
    torch = _torch()
    lib = load_library()
    flags = 0
    if sources is None:
        flags |= RPQ_ALL_SOURCES
        src_t = None
        n = rpq_graph_info_get(g)["n_vertices"]
    else:
        src_t = _dev_u32(sources, torch)
        n = src_t.numel()
    o = _opts(opts)
    if per_source is True:
        per_source = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    if per_source is not None:
        flags |= RPQ_PER_SOURCE
    if pairs is True:
        first, _ = rpq_eval_split(g, head, tail, src_t, opts, None, per_source, stream)
        pairs = torch.empty(max(first.count, 1), dtype=torch.int64, device="cuda")
    if pairs is not None:
        flags |= RPQ_PAIRS
    res = _Result()
    res.pairs = pairs.data_ptr() if pairs is not None else None
    res.capacity = int(pairs.numel()) if pairs is not None else 0
    res.per_source = per_source.data_ptr() if per_source is not None else None
    info = SplitInfo()
    rc = lib.rpq_eval_split(g.handle, ctypes.byref(head), ctypes.byref(tail),
                            src_t.data_ptr() if (src_t is not None and n) else None, n, flags,
                            ctypes.byref(o) if o is not None else None, ctypes.byref(res), ctypes.byref(info),
                            _stream(stream))
    _check(rc, allow=(RPQ_EOVERFLOW,) if allow_overflow else ())
    out_pairs = pairs[: res.written] if pairs is not None else None
    return (EvalResult(int(res.count), int(res.hash), int(res.product_edges), int(res.levels), int(res.max_depth),
                       int(res.written), out_pairs, per_source, rc),
            {name: int(getattr(info, name)) for name, _ in SplitInfo._fields_})


def rpq_eval_noalloc(g: Graph, nfa: Nfa, sources=None, flags: int = 0, opts=None, pairs=None,
                     capacity: Optional[int] = None, pair_offset: int = 0, per_source=None, stream=None,
                     allow_overflow: bool = False, max_length: Optional[int] = None) -> EvalResult:
    """rpq_eval in the library's static device scratch (no workspace, no allocation inside the
    call).  Arguments as rpq_eval; pairs and per_source must be caller tensors or None."""
    torch = _torch()
    lib = load_library()
    if max_length is not None:
        opts = dict(opts or {}) if not isinstance(opts, EvalOpts) else {k: getattr(opts, k) for k, _ in
                                                                          EvalOpts._fields_}
        opts["max_length"] = int(max_length)
        flags |= RPQ_LENGTH_BOUND
    if sources is None:
        flags |= RPQ_ALL_SOURCES
        src_t = None
        n = rpq_graph_info_get(g)["n_vertices"]
    else:
        src_t = _dev_u32(sources, torch)
        n = src_t.numel()
    o = _opts(opts)
    if per_source is not None:
        flags |= RPQ_PER_SOURCE
    if pairs is not None:
        flags |= RPQ_PAIRS
        if capacity is None:
            capacity = pairs.numel()
    res = _Result()
    res.pairs = pairs.data_ptr() if pairs is not None else None
    res.capacity = int(capacity or 0)
    res.per_source = per_source.data_ptr() if per_source is not None else None
    res.pair_offset = int(pair_offset)
    rc = lib.rpq_eval_noalloc(g.handle, ctypes.byref(nfa), src_t.data_ptr() if (src_t is not None and n) else None,
                              n, flags, ctypes.byref(o) if o is not None else None, ctypes.byref(res),
                              _stream(stream))
    _check(rc, allow=(RPQ_EOVERFLOW,) if allow_overflow else ())
    out_pairs = pairs[: res.written] if pairs is not None else None
    return EvalResult(int(res.count), int(res.hash), int(res.product_edges), int(res.levels), int(res.max_depth),
                      int(res.written), out_pairs, per_source, rc)


# ------------------------------------------------------------------------------------------------
# profiling
# ------------------------------------------------------------------------------------------------

def rpq_profile_enable(on: bool = True) -> None:
    _check(load_library().rpq_profile_enable(1 if on else 0))


def rpq_profile_read(reset: bool = False) -> dict:
    p = Profile()
    _check(load_library().rpq_profile_read(ctypes.byref(p), 1 if reset else 0))
    return {name: getattr(p, name) for name, _ in Profile._fields_}


# ------------------------------------------------------------------------------------------------
# batched evaluation
# ------------------------------------------------------------------------------------------------

class Batch:
    """Owner of an rpq_batch_t plus the device buffers its queries write into."""

    def __init__(self, handle: int, graph: Graph):
        self.handle = ctypes.c_void_p(handle)
        self.graph = graph           # keeps the graph alive
        self.keep = []               # device tensors the batch reads or writes
        self.outputs = []            # per query: (pairs tensor or None, per_source tensor or None)
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().rpq_batch_destroy(self.handle)
        self.handle = None

    def add(self, nfa: Nfa, sources=None, pairs_capacity: Optional[int] = None, per_source: bool = False,
            max_length: Optional[int] = None) -> int:
        qid = rpq_batch_add(self, nfa, sources, pairs_capacity, per_source)
        if max_length is not None:
            rpq_batch_bound_length(self, qid, max_length)
        return qid

    def run(self, stream=None) -> None:
        rpq_batch_run(self, stream=stream)

    def result(self, qid: int) -> EvalResult:
        return rpq_batch_result(self, qid)

    def stats(self) -> dict:
        return rpq_batch_stats(self)

    def autotune(self, candidates=None, workspace_bytes: int = 0, stream=None) -> dict:
        return rpq_batch_autotune(self, candidates, workspace_bytes, stream)


def rpq_batch_create(g: Graph, opts=None) -> Batch:
    o = None
    if opts:
        o = BatchOpts()
        _fill(o, opts)
    h = ctypes.c_void_p()
    _check(load_library().rpq_batch_create(g.handle, ctypes.byref(o) if o is not None else None, ctypes.byref(h)))
    return Batch(h.value, g)


def rpq_batch_destroy(b: Batch) -> None:
    b.close()


def rpq_batch_add(b: Batch, nfa: Nfa, sources=None, pairs_capacity: Optional[int] = None,
                  per_source: bool = False) -> int:
    """Add a query; sources=None means every vertex.  Result buffers are allocated here."""
    torch = _torch()
    flags = 0
    if sources is None:
        flags |= RPQ_ALL_SOURCES
        src_t = None
        n = b.graph.info()["n_vertices"]
    else:
        src_t = _dev_u32(sources, torch)
        n = src_t.numel()
        b.keep.append(src_t)
    pairs = ps = None
    if pairs_capacity is not None:
        flags |= RPQ_PAIRS
        pairs = torch.empty(max(int(pairs_capacity), 1), dtype=torch.int64, device="cuda")
        b.keep.append(pairs)
    if per_source:
        flags |= RPQ_PER_SOURCE
        ps = torch.zeros((max(n, 1), 2), dtype=torch.int64, device="cuda")
        b.keep.append(ps)
    qid = ctypes.c_uint32()
    _check(load_library().rpq_batch_add(b.handle, ctypes.byref(nfa),
                                        src_t.data_ptr() if (src_t is not None and n) else None, n, flags,
                                        pairs.data_ptr() if pairs is not None else None,
                                        int(pairs_capacity or 0), ps.data_ptr() if ps is not None else None,
                                        ctypes.byref(qid)))
    b.outputs.append((pairs, ps[:n] if ps is not None else None))
    return int(qid.value)


def rpq_batch_bound_length(b: Batch, qid: int, max_length: int) -> None:
    """Only walks of at most max_length edges count for query qid (before the first run)."""
    _check(load_library().rpq_batch_bound_length(b.handle, int(qid), int(max_length)))


def rpq_batch_workspace_size(b: Batch) -> int:
    n = ctypes.c_uint64()
    _check(load_library().rpq_batch_workspace_size(b.handle, ctypes.byref(n)))
    return int(n.value)


def rpq_batch_run(b: Batch, workspace=None, stream=None) -> None:
    torch = _torch()
    need = rpq_batch_workspace_size(b)
    if workspace is None:
        if b.ws is None or b.ws.numel() < need:
            b.ws = None
            b.ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        workspace = b.ws
    _check(load_library().rpq_batch_run(b.handle, workspace.data_ptr(), workspace.numel(), _stream(stream)))


def rpq_batch_result(b: Batch, qid: int) -> EvalResult:
    res = _Result()
    rc = load_library().rpq_batch_result(b.handle, qid, ctypes.byref(res))
    _check(rc, allow=(RPQ_EOVERFLOW,))
    pairs, ps = b.outputs[qid]
    return EvalResult(int(res.count), int(res.hash), int(res.product_edges), int(res.levels), int(res.max_depth),
                      int(res.written), pairs[: res.written] if pairs is not None else None, ps, rc)


def rpq_batch_stats(b: Batch) -> dict:
    info = BatchInfo()
    _check(load_library().rpq_batch_stats(b.handle, ctypes.byref(info)))
    out = {name: getattr(info, name) for name, _ in BatchInfo._fields_}
    out["phase_ms"] = dict(zip(["expand", "compact", "decide", "retire_extract", "retire_keys", "retire_clear",
                                "refill_seed", "finalize"], [round(x, 3) for x in info.phase_ms]))
    return out


def rpq_batch_autotune(b: Batch, candidates=None, workspace_bytes: int = 0, stream=None) -> dict:
    """Pick the batch's width/slots/chunk by timing candidates (native tuner).

    A workspace of workspace_bytes (default: 4x the current plan, at least 1 GiB, at most three
    quarters of the free device memory) is allocated for the timing runs and kept for the batch;
    candidates whose plan does not fit it are skipped."""
    torch = _torch()
    if not workspace_bytes:
        plan = rpq_batch_workspace_size(b)
        free, _ = torch.cuda.mem_get_info()
        held = b.ws.numel() if b.ws is not None else 0
        workspace_bytes = max(plan, min(max(4 * plan, 1 << 30), (free + held) * 3 // 4))
    if b.ws is None or b.ws.numel() < workspace_bytes:
        b.ws = None
        b.ws = torch.empty(workspace_bytes, dtype=torch.uint8, device="cuda")
    arr = None
    n = 0
    if candidates:
        n = len(candidates)
        arr = (BatchOpts * n)()
        for i, c in enumerate(candidates):
            _fill(arr[i], c)
    best = BatchOpts()
    _check(load_library().rpq_batch_autotune(b.handle, arr, n, b.ws.data_ptr(), b.ws.numel(), _stream(stream),
                                             ctypes.byref(best)))
    return {name: getattr(best, name) for name, _ in BatchOpts._fields_}


# ---------------------------------------------------------------------------------------------
# CRPQ
# ---------------------------------------------------------------------------------------------
class CrpqOutput:
    """Result of crpq_eval: distinct assignments of the free variables."""

    def __init__(self, r: CrpqResult, tuples, n_atoms: int, status: int):
        self.count = int(r.count)
        self.hash = int(r.hash)
        self.written = int(r.written)
        self.n_free = int(r.n_free)
        self.tuples = tuples      # int32 CUDA tensor [written, n_free] (uint32 bits) or None
        self.atom_pairs = [int(r.atom_pairs[i]) for i in range(n_atoms)]
        self.atom_strategy = [int(r.atom_strategy[i]) for i in range(n_atoms)]
        self.join_rows = int(r.join_rows)
        self.status = status


def _crpq_marshal(g: Graph, atoms, n_vars: int, binding, vertex_label, domain, neq, torch):
    """ctypes atoms and variables of a CRPQ, plus the objects that must outlive the call."""
    n_atoms = len(atoms)
    arr = (CrpqAtom * max(1, n_atoms))()
    for i, (x, rx, y) in enumerate(atoms):
        arr[i].src_var = int(x)
        arr[i].dst_var = int(y)
        arr[i].nfa = rx if isinstance(rx, Nfa) else rpq_nfa_compile(rx, g.names)
    v = CrpqVars()
    v.n_vars = int(n_vars)
    keep = [arr]
    if binding is not None:
        b = (ctypes.c_int64 * n_vars)(*[(-1 if x is None else int(x)) for x in binding])
        keep.append(b)
        v.binding = ctypes.cast(b, ctypes.POINTER(ctypes.c_int64))
    if vertex_label is not None:
        vl = (ctypes.c_int32 * n_vars)(*[(-1 if x is None else int(x)) for x in vertex_label])
        keep.append(vl)
        v.vertex_label = ctypes.cast(vl, ctypes.POINTER(ctypes.c_int32))
    if domain is not None:
        ptrs = (ctypes.c_void_p * n_vars)()
        sizes = (ctypes.c_uint64 * n_vars)()
        for i, d in enumerate(domain):
            if d is None:
                continue
            t = _dev_u32(d, torch)
            keep.append(t)
            ptrs[i] = t.data_ptr() if t.numel() else None
            sizes[i] = t.numel()
            if not t.numel():   # an empty domain: a pointer is still needed to mean "constrained"
                z = torch.zeros(1, dtype=torch.int32, device="cuda")
                keep.append(z)
                ptrs[i] = z.data_ptr()
        keep += [ptrs, sizes]
        v.domain = ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p))
        v.domain_size = ctypes.cast(sizes, ctypes.POINTER(ctypes.c_uint64))
    neq = list(neq)
    if neq:
        nq = (ctypes.c_uint32 * (2 * len(neq)))(*[int(x) for p in neq for x in p])
        keep.append(nq)
        v.neq = ctypes.cast(nq, ctypes.POINTER(ctypes.c_uint32))
        v.n_neq = len(neq)
    return arr, v, keep


def _n_free(n_vars, binding):
    return sum(1 for i in range(n_vars) if binding is None or binding[i] is None or binding[i] < 0)


def crpq_eval(g: Graph, atoms, n_vars: int, binding=None, vertex_label=None, domain=None, neq=(),
              tuples: bool = False, capacity: Optional[int] = None, flags: int = 0,
              workspace_bytes: Optional[int] = None, stream=None, allow_overflow: bool = False) -> CrpqOutput:
    """Evaluate a CRPQ (see crpq_eval in include/rpq.h).

    atoms: sequence of (src_var, regex string or Nfa, dst_var).  binding / vertex_label: per
    variable, None or -1 for no constraint.  domain: per variable, None or a vertex list (host
    array or CUDA tensor).  neq: pairs of variables that must differ.  tuples=True returns the
    sorted tuples (capacity rows, default: all of them).  The device workspace grows as the
    library asks for it.
    """
    torch = _torch()
    lib = load_library()
    n_atoms = len(atoms)
    arr, v, keep = _crpq_marshal(g, atoms, n_vars, binding, vertex_label, domain, neq, torch)
    if workspace_bytes:
        ws_bytes = int(workspace_bytes)
    else:   # a quarter of the free device memory, at most 32 GiB
        free, _ = torch.cuda.mem_get_info()
        ws_bytes = max(256 << 20, min(free // 4, 32 << 30))
    cap = capacity if capacity is not None else (1 << 20)
    for attempt in range(12):
        r = CrpqResult()
        out_t = None
        if tuples:
            out_t = torch.empty((max(1, cap), max(1, _n_free(n_vars, binding))), dtype=torch.int32, device="cuda")
            r.tuples = out_t.data_ptr()
            r.capacity = cap
        ws = g.workspace(ws_bytes)
        rc = lib.crpq_eval(g.handle, arr, n_atoms, ctypes.byref(v), int(flags), ws.data_ptr(), ws.numel(),
                           ctypes.byref(r), _stream(stream))
        if rc == RPQ_ENOMEM and r.workspace_needed > ws.numel():
            ws_bytes = int(r.workspace_needed)
            continue
        if rc == RPQ_EOVERFLOW and tuples and capacity is None and not allow_overflow:
            cap = int(r.count)
            continue
        _check(rc, allow=(RPQ_EOVERFLOW,) if allow_overflow else ())
        tt = None
        if tuples:
            tt = out_t[: int(r.written), : int(r.n_free)] if r.n_free else out_t[: int(r.written), :0]
        return CrpqOutput(r, tt, n_atoms, rc)
    raise RpqError(RPQ_ENOMEM, "crpq_eval: workspace kept growing (%d bytes last asked)" % ws_bytes)


# ---------------------------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------------------------
def _ticket_dict(t: Ticket) -> dict:
    return dict(status=int(t.status), done=bool(t.done), count=int(t.count), hash=int(t.hash),
                product_edges=int(t.product_edges), written=int(t.written), workspace_bytes=int(t.workspace_bytes),
                arrival_ms=float(t.arrival_ms), start_ms=float(t.start_ms), end_ms=float(t.end_ms),
                resident=bool(t.resident))


class Server:
    """A request loop over one resident graph (rpq_serve_* in include/rpq.h).

    The device pool is one torch allocation of pool_bytes held by the server; requests run on
    `workers` streams as the pool admits them, or on the resident engine (resident_slots > 0)
    for the dense RPQs it takes.  Tensors a request names (sources, outputs, domains) are kept
    alive until its ticket is collected with wait() or a done poll()."""

    def __init__(self, g: Graph, pool_bytes: int, workers: int = 4, resident_slots: int = 0,
                 resident_width: int = 0, resident_states: int = 0, resident_succ: int = 0,
                 resident_iters: int = 0, resident_max_units: int = 0):
        torch = _torch()
        self.g = g
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        o = ServerOpts()
        o.workers = int(workers)
        o.resident_slots = int(resident_slots)
        o.resident_width = int(resident_width)
        o.resident_states = int(resident_states)
        o.resident_succ = int(resident_succ)
        o.resident_iters = int(resident_iters)
        o.resident_max_units = int(resident_max_units)
        h = ctypes.c_void_p()
        _check(load_library().rpq_serve_start(g.handle, ctypes.byref(o), self.pool.data_ptr(), self.pool.numel(),
                                              ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def clock_ms(self) -> float:
        x = ctypes.c_double()
        _check(load_library().rpq_serve_clock_ms(self.handle, ctypes.byref(x)))
        return float(x.value)

    def _submit(self, req: Request, keep) -> int:
        t = ctypes.c_uint64()
        _check(load_library().rpq_serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._keep[int(t.value)] = keep
        return int(t.value)

    def submit_rpq(self, nfa: Nfa, sources=None, flags: int = 0, pairs=None, per_source=None,
                   arrival_ms: float = -1.0) -> int:
        """Queue an RPQ (as rpq_eval).  pairs: a CUDA int64 tensor for keys; per_source: [n, 2]."""
        torch = _torch()
        req = Request()
        req.kind = RPQ_REQ_RPQ
        req.arrival_ms = float(arrival_ms)
        req.nfa = nfa
        keep = []
        if sources is None:
            flags |= RPQ_ALL_SOURCES
            req.n_sources = rpq_graph_info_get(self.g)["n_vertices"]
        else:
            st = _dev_u32(sources, torch)
            keep.append(st)
            req.sources = st.data_ptr() if st.numel() else None
            req.n_sources = st.numel()
        if pairs is not None:
            flags |= RPQ_PAIRS
            req.pairs = pairs.data_ptr()
            req.capacity = pairs.numel()
            keep.append(pairs)
        if per_source is not None:
            flags |= RPQ_PER_SOURCE
            req.per_source = per_source.data_ptr()
            keep.append(per_source)
        req.flags = flags
        return self._submit(req, keep)

    def submit_crpq(self, atoms, n_vars: int, binding=None, vertex_label=None, domain=None, neq=(),
                    tuples=None, flags: int = 0, arrival_ms: float = -1.0) -> int:
        """Queue a CRPQ (as crpq_eval).  tuples: a CUDA int32 tensor [capacity, n_free] or None."""
        torch = _torch()
        arr, v, keep = _crpq_marshal(self.g, atoms, n_vars, binding, vertex_label, domain, neq, torch)
        req = Request()
        req.kind = RPQ_REQ_CRPQ
        req.flags = int(flags)
        req.arrival_ms = float(arrival_ms)
        req.atoms = arr
        req.n_atoms = len(atoms)
        req.vars = v
        if tuples is not None:
            req.tuples = tuples.data_ptr()
            req.tuple_capacity = tuples.shape[0]
            keep.append(tuples)
        return self._submit(req, keep)

    def poll(self, ticket: int) -> dict:
        t = Ticket()
        _check(load_library().rpq_serve_poll(self.handle, int(ticket), ctypes.byref(t)))
        if t.done:
            self._keep.pop(int(ticket), None)
        return _ticket_dict(t)

    def wait(self, ticket: int) -> dict:
        t = Ticket()
        _check(load_library().rpq_serve_wait(self.handle, int(ticket), ctypes.byref(t)))
        self._keep.pop(int(ticket), None)
        return _ticket_dict(t)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load_library().rpq_serve_stats(self.handle, ctypes.byref(st)))
        return {n: int(getattr(st, n)) for n, _ in ServerStats._fields_}

    def stop(self) -> None:
        """Finish every request, join the workers and release the device pool."""
        if self.handle is not None and self.handle.value:
            _check(load_library().rpq_serve_stop(self.handle))
        self.handle = None
        self._keep.clear()
        self.pool = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
