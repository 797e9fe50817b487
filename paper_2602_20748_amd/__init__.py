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
    "rpq_graph_export_csr", "rpq_eval_workspace_size", "rpq_eval", "EvalResult", "Graph", "Nfa", "EvalOpts",
    "RPQ_OK", "RPQ_EINVAL", "RPQ_ENOMEM", "RPQ_EOVERFLOW", "RPQ_EDEVICE", "RPQ_EUNSUPPORTED",
    "RPQ_BUILD_IN_CSR", "RPQ_PAIRS", "RPQ_PER_SOURCE", "RPQ_ALL_SOURCES", "RPQ_REVERSE",
    "RPQ_MAX_STATES", "RPQ_MAX_LABELS", "EXPORTED_SYMBOLS", "rpq_profile_enable", "rpq_profile_read",
    "Batch", "rpq_batch_create", "rpq_batch_destroy", "rpq_batch_add", "rpq_batch_workspace_size",
    "rpq_batch_run", "rpq_batch_result", "rpq_batch_stats", "rpq_batch_autotune",
]

_HERE = os.path.dirname(os.path.abspath(__file__))

RPQ_OK, RPQ_EINVAL, RPQ_ENOMEM, RPQ_EOVERFLOW, RPQ_EDEVICE, RPQ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RPQ_BUILD_IN_CSR = 1
RPQ_PAIRS, RPQ_PER_SOURCE, RPQ_ALL_SOURCES, RPQ_REVERSE = 1, 2, 4, 8
RPQ_MAX_STATES, RPQ_MAX_LABELS = 32, 64

_STATUS = {0: "RPQ_OK", -1: "RPQ_EINVAL", -2: "RPQ_ENOMEM", -3: "RPQ_EOVERFLOW", -4: "RPQ_EDEVICE",
           -5: "RPQ_EUNSUPPORTED"}


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
                ("sync_every", ctypes.c_uint32), ("chunk_edges", ctypes.c_uint32)]


class Profile(ctypes.Structure):
    _fields_ = [("expand_launches", ctypes.c_uint64), ("expand_ms", ctypes.c_double),
                ("finalize_launches", ctypes.c_uint64), ("finalize_ms", ctypes.c_double),
                ("edge_items", ctypes.c_uint64), ("descriptors", ctypes.c_uint64), ("row_words", ctypes.c_uint64),
                ("word_reads", ctypes.c_uint64), ("word_updates", ctypes.c_uint64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("batch_width", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("chunk_edges", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_uint32), ("n_units", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("batch_width", ctypes.c_uint32), ("blocks", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("edge_items", ctypes.c_uint64), ("descriptors", ctypes.c_uint64), ("word_reads", ctypes.c_uint64),
                ("word_updates", ctypes.c_uint64), ("finalized_rows", ctypes.c_uint64),
                ("finalized_words", ctypes.c_uint64), ("touch_words", ctypes.c_uint64), ("row_words", ctypes.c_uint64),
                ("last_run_ms", ctypes.c_double), ("last_kernel_ms", ctypes.c_double),
                ("phase_ms", ctypes.c_double * 8)]


class _Result(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_void_p), ("capacity", ctypes.c_uint64), ("per_source", ctypes.c_void_p),
                ("pair_offset", ctypes.c_uint64), ("written", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("hash", ctypes.c_uint64), ("product_edges", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("max_depth", ctypes.c_uint64)]


# Every symbol include/rpq.h declares (checked by the CPU test suite).
EXPORTED_SYMBOLS = [
    "rpq_last_error", "rpq_abi_version", "rpq_graph_create", "rpq_graph_destroy", "rpq_graph_info_get",
    "rpq_graph_export_csr", "rpq_nfa_compile", "rpq_nfa_reverse", "rpq_eval_workspace_size", "rpq_eval",
    "rpq_profile_enable", "rpq_profile_read",
    "rpq_batch_create", "rpq_batch_destroy", "rpq_batch_add", "rpq_batch_workspace_size", "rpq_batch_run",
    "rpq_batch_result", "rpq_batch_stats", "rpq_batch_autotune",
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
        "rpq_profile_enable": (ctypes.c_int, [ctypes.c_int]),
        "rpq_batch_create": (ctypes.c_int, [vp, ctypes.POINTER(BatchOpts), ctypes.POINTER(vp)]),
        "rpq_batch_destroy": (ctypes.c_int, [vp]),
        "rpq_batch_add": (ctypes.c_int, [vp, ctypes.POINTER(Nfa), vp, u64, u32, vp, u64, vp,
                                         ctypes.POINTER(u32)]),
        "rpq_batch_workspace_size": (ctypes.c_int, [vp, ctypes.POINTER(u64)]),
        "rpq_batch_run": (ctypes.c_int, [vp, vp, u64, vp]),
        "rpq_batch_result": (ctypes.c_int, [vp, u32, ctypes.POINTER(_Result)]),
        "rpq_batch_stats": (ctypes.c_int, [vp, ctypes.POINTER(BatchInfo)]),
        "rpq_batch_autotune": (ctypes.c_int, [vp, ctypes.POINTER(BatchOpts), u32, vp, u64, vp,
                                              ctypes.POINTER(BatchOpts)]),
        "rpq_profile_read": (ctypes.c_int, [ctypes.POINTER(Profile), ctypes.c_int]),
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


def _opts(opts) -> Optional[EvalOpts]:
    if opts is None:
        return None
    if isinstance(opts, EvalOpts):
        return opts
    o = EvalOpts()
    for k, v in dict(opts).items():
        setattr(o, k, int(v))
    return o


def rpq_eval_workspace_size(g: Graph, nfa: Nfa, n_sources: int, flags: int, opts=None) -> int:
    n = ctypes.c_uint64()
    o = _opts(opts)
    _check(load_library().rpq_eval_workspace_size(g.handle, ctypes.byref(nfa), n_sources, flags,
                                                  ctypes.byref(o) if o is not None else None, ctypes.byref(n)))
    return int(n.value)


def rpq_eval(g: Graph, nfa: Nfa, sources=None, flags: int = 0, opts=None, pairs=None, capacity: Optional[int] = None,
             pair_offset: int = 0, per_source=None, workspace=None, stream=None,
             allow_overflow: bool = False) -> EvalResult:
    """Evaluate one RPQ.

    sources: CUDA/numpy uint32 ids (strictly ascending) or None with RPQ_ALL_SOURCES.
    pairs: a CUDA int64 tensor to receive keys (capacity = its length), or
      True to allocate one of exactly the needed size (two passes), or None.
    per_source: a CUDA int64 tensor [n, 2], or True to allocate one.
    """
    torch = _torch()
    lib = load_library()
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
        first = rpq_eval(g, nfa, src_t, flags & ~RPQ_PAIRS, opts, None, None, 0, per_source, workspace, stream)
        pairs = torch.empty(max(first.count - pair_offset, 1), dtype=torch.int64, device="cuda")
        capacity = max(first.count - pair_offset, 0)
    if pairs is not None:
        flags |= RPQ_PAIRS
        if capacity is None:
            capacity = pairs.numel()
    need = ctypes.c_uint64()
    _check(lib.rpq_eval_workspace_size(g.handle, ctypes.byref(nfa), n, flags,
                                       ctypes.byref(o) if o is not None else None, ctypes.byref(need)))
    ws = workspace if workspace is not None else g.workspace(int(need.value))
    res = _Result()
    res.pairs = pairs.data_ptr() if pairs is not None else None
    res.capacity = int(capacity or 0)
    res.per_source = per_source.data_ptr() if per_source is not None else None
    res.pair_offset = int(pair_offset)
    rc = lib.rpq_eval(g.handle, ctypes.byref(nfa), src_t.data_ptr() if (src_t is not None and n) else None, n, flags,
                      ctypes.byref(o) if o is not None else None, ws.data_ptr(), ws.numel(), ctypes.byref(res),
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

    def add(self, nfa: Nfa, sources=None, pairs_capacity: Optional[int] = None, per_source: bool = False) -> int:
        return rpq_batch_add(self, nfa, sources, pairs_capacity, per_source)

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
        for k, v in dict(opts).items():
            setattr(o, k, int(v))
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

    A workspace of workspace_bytes (default: 4x the current plan, at least 1 GiB) is
    allocated for the timing runs and kept for the batch."""
    torch = _torch()
    if not workspace_bytes:
        workspace_bytes = max(4 * rpq_batch_workspace_size(b), 1 << 30)
    if b.ws is None or b.ws.numel() < workspace_bytes:
        b.ws = None
        b.ws = torch.empty(workspace_bytes, dtype=torch.uint8, device="cuda")
    arr = None
    n = 0
    if candidates:
        n = len(candidates)
        arr = (BatchOpts * n)()
        for i, c in enumerate(candidates):
            for k, v in dict(c).items():
                setattr(arr[i], k, int(v))
    best = BatchOpts()
    _check(load_library().rpq_batch_autotune(b.handle, arr, n, b.ws.data_ptr(), b.ws.numel(), _stream(stream),
                                             ctypes.byref(best)))
    return {name: getattr(best, name) for name, _ in BatchOpts._fields_}
