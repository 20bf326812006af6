"""Python binding of the MI355X buffer k-d tree library (``libbkd.so``).

Argument marshalling only: every step of a query runs in the library's HIP
kernels.  The names follow the C ABI in ``include/bkd.h`` (``bkd_build`` ->
``build``, ``bkd_query`` -> ``query`` ...).  Host arrays are numpy; device
arrays are torch tensors on a HIP device (torch provides memory and streams
only).  There is no CPU fallback: if the library has not been built, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbkd.so")

OK, EINVAL, ENOMEM, EBUDGET, EDEVICE, EBUSY, ETIMEOUT, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
CHUNK_LEAF, CHUNK_POSITION = 0, 1
FLAG_TRACE, FLAG_TIMING, FLAG_SQUARED, FLAG_NO_TAIL, FLAG_DEVICE_BUILD, FLAG_DEVICE_PTRS = 1, 2, 4, 8, 16, 32
MAX_DIM, MAX_K, MAX_HEIGHT = 32, 64, 24
SPLIT_CYCLIC, SPLIT_LONGEST = 0, 1
PRUNE_PLANE, PRUNE_BOX = 0, 1

_lib = None


class BkdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bkd error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("buffer_size", ctypes.c_int64), ("fetch_size", ctypes.c_int64),
                ("leaf_budget_bytes", ctypes.c_int64), ("chunk_mode", ctypes.c_int32),
                ("num_chunks", ctypes.c_int32), ("device", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tail_max", ctypes.c_int64), ("split_rule", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("leaf_path", ctypes.c_char_p)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("height", ctypes.c_int32),
                ("buffer_size", ctypes.c_int64), ("fetch_size", ctypes.c_int64), ("num_chunks", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("leaf_bytes", ctypes.c_int64),
                ("chunk_capacity_bytes", ctypes.c_int64), ("on_disk", ctypes.c_int32), ("direct_io", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_int64), ("fetches", ctypes.c_int64), ("calls", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("visits", ctypes.c_int64), ("dense_launches", ctypes.c_int64),
                ("dense_pairs", ctypes.c_int64), ("sparse_launches", ctypes.c_int64),
                ("sparse_pairs", ctypes.c_int64), ("chunk_copies", ctypes.c_int64), ("bytes_h2d", ctypes.c_int64),
                ("dense_ms", ctypes.c_double), ("sparse_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("dense_visits", ctypes.c_int64), ("leaf_points_dense", ctypes.c_int64),
                ("leaf_points_other", ctypes.c_int64), ("alg_bytes", ctypes.c_int64),
                ("alg_bytes_dense", ctypes.c_int64), ("find_ms", ctypes.c_double), ("group_ms", ctypes.c_double),
                ("copy_ms", ctypes.c_double), ("wait_ms", ctypes.c_double), ("bytes_disk", ctypes.c_int64),
                ("disk_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes)
_V, _I64, _I32, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_PROTOS = {
    "bkd_last_error": (ctypes.c_char_p, []),
    "bkd_version": (ctypes.c_char_p, []),
    "bkd_default_options": (ctypes.c_int, [_I32, _V]),
    "bkd_build": (ctypes.c_int, [_V, _I64, _I32, _I32, _V, _V]),
    "bkd_free": (ctypes.c_int, [_V]),
    "bkd_query": (ctypes.c_int, [_V, _V, _I64, _I32, _V, _V]),
    "bkd_query_async": (ctypes.c_int, [_V, _V, _I64, _I32, _V, _V, _V]),
    "bkd_query_async_noalloc": (ctypes.c_int, [_V, _V, _I64, _I32, _V, _V, _V]),
    "bkd_outlier_scores": (ctypes.c_int, [_V, _V, _I64, _I32, _V, _V]),
    "bkd_tree_info_get": (ctypes.c_int, [_V, _V]),
    "bkd_tree_export": (ctypes.c_int, [_V, _V, _V, _V]),
    "bkd_chunk_plan": (ctypes.c_int, [_V, _V, _V]),
    "bkd_tree_rules_export": (ctypes.c_int, [_V, _V, _V]),
    "bkd_last_stats": (ctypes.c_int, [_V, _V]),
    "bkd_trace_size": (ctypes.c_int, [_V, _V, _V]),
    "bkd_trace_get": (ctypes.c_int, [_V, _V, _V, _V]),
    "bkd_batch_create": (ctypes.c_int, [_V, _I32, _I32, _I32, _V]),
    "bkd_batch_run": (ctypes.c_int, [_V, _V, _V]),
    "bkd_batch_results": (ctypes.c_int, [_V]),
    "bkd_batch_autotune": (ctypes.c_int, [_V, _V, _V]),
    "bkd_batch_tuning_save": (ctypes.c_int, [_V, ctypes.c_char_p]),
    "bkd_batch_tuning_load": (ctypes.c_int, [_V, ctypes.c_char_p, _V]),
    "bkd_batch_stats_get": (ctypes.c_int, [_V, _V]),
    "bkd_batch_free": (ctypes.c_int, [_V]),
    "bkd_server_create": (ctypes.c_int, [_V, _V]),
    "bkd_server_add_tree": (ctypes.c_int, [_V, _V, _V]),
    "bkd_submit": (ctypes.c_int, [_V, _I32, _V, _I64, _I32, _V, _V, _V]),
    "bkd_poll": (ctypes.c_int, [_V, _I64, _V]),
    "bkd_wait": (ctypes.c_int, [_V, _I64, _I64]),
    "bkd_cancel": (ctypes.c_int, [_V, _I64]),
    "bkd_request_times": (ctypes.c_int, [_V, _I64, _V, _V, _V]),
    "bkd_server_stats_get": (ctypes.c_int, [_V, _V]),
    "bkd_release": (ctypes.c_int, [_V, _I64]),
    "bkd_server_destroy": (ctypes.c_int, [_V]),
}


def exported_names():
    return list(_PROTOS)


def lib():
    """Load ``libbkd.so``; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1512_02831_amd.compile (hipcc, gfx950)")
    try:  # share torch's HIP runtime when torch is present (one runtime per process)
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise BkdError(rc, lib().bkd_last_error().decode())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def version() -> str:
    return lib().bkd_version().decode()


def default_options(height: int) -> Options:
    o = Options()
    _check(lib().bkd_default_options(height, ctypes.byref(o)))
    return o


def make_options(height: int, buffer_size=None, fetch_size=None, leaf_budget_bytes=None, chunk_mode=None,
                 num_chunks=None, device=None, flags=None, tail_max=None, split_rule=None, prune=None,
                 leaf_path=None) -> Options:
    o = default_options(height)
    if leaf_path is not None:
        o.leaf_path = os.fsencode(leaf_path)
    for name, val in (("buffer_size", buffer_size), ("fetch_size", fetch_size),
                      ("leaf_budget_bytes", leaf_budget_bytes), ("chunk_mode", chunk_mode),
                      ("num_chunks", num_chunks), ("device", device), ("flags", flags), ("tail_max", tail_max),
                      ("split_rule", split_rule), ("prune", prune)):
        if val is not None:
            setattr(o, name, val)
    return o


class Tree:
    """A built buffer k-d tree (owns a ``bkd_tree*``)."""

    def __init__(self, handle, n, d, height):
        self._h, self.n, self.d, self.height = handle, n, d, height

    @property
    def handle(self):
        if not self._h:
            raise ValueError("tree has been freed")
        return self._h

    def free(self):
        if self._h:
            _check(lib().bkd_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def build(P, height: int, options: Options | None = None, **kw) -> Tree:
    """``bkd_build``: P host float32 [n, d]."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    if P.ndim != 2:
        raise ValueError("P must be 2-D [n, d]")
    n, d = P.shape
    if options is None and kw:
        options = make_options(height, **kw)
    h = ctypes.c_void_p()
    _check(lib().bkd_build(_p(P), n, d, height, ctypes.byref(options) if options is not None else None,
                           ctypes.byref(h)))
    return Tree(h.value, n, d, height)


def query(tree: Tree, Q, k: int):
    """``bkd_query``: host Q float32 [m, d] -> (idx int64 [m, k], dist float32 [m, k])."""
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    if Q.ndim != 2 or Q.shape[1] != tree.d:
        raise ValueError("Q must be [m, d] with the tree's d")
    m = Q.shape[0]
    idx = np.empty((m, k), dtype=np.int64)
    dist = np.empty((m, k), dtype=np.float32)
    _check(lib().bkd_query(tree.handle, _p(Q), m, k, _p(idx), _p(dist)))
    return idx, dist


def outlier_scores(tree: Tree, P, k: int):
    """``bkd_outlier_scores``: the tree's own reference set P float32 [n, d] ->
    (score float32 [n], order int64 [n], highest score first)."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    if P.ndim != 2 or P.shape[1] != tree.d:
        raise ValueError("P must be [n, d] with the tree's d")
    n = P.shape[0]
    score = np.empty(n, dtype=np.float32)
    order = np.empty(n, dtype=np.int64)
    _check(lib().bkd_outlier_scores(tree.handle, _p(P), n, k, _p(score), _p(order)))
    return score, order


def query_async(tree: Tree, dQ, k: int, d_idx, d_dist, stream=None):
    """``bkd_query_async`` on torch device tensors: dQ [m, d] float32, d_idx [m, k] int64, d_dist [m, k] float32."""
    import torch
    for t, dt in ((dQ, torch.float32), (d_idx, torch.int64), (d_dist, torch.float32)):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dt):
            raise ValueError("device tensors must be contiguous HIP tensors of the documented dtypes")
    m = dQ.shape[0]
    if dQ.shape != (m, tree.d) or d_idx.shape != (m, k) or d_dist.shape != (m, k):
        raise ValueError("shape mismatch")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().bkd_query_async(tree.handle, dQ.data_ptr(), m, k, d_idx.data_ptr(), d_dist.data_ptr(),
                                 ctypes.c_void_p(s.cuda_stream)))


def query_async_noalloc(tree: Tree, dQ, k: int, d_idx, d_dist, stream=None):
    """``bkd_query_async_noalloc``: as ``query_async``, with the library's fixed 64 MiB
    device workspace instead of buffers it allocates (resident trees; calls that overlap
    on one device race)."""
    import torch
    for t, dt in ((dQ, torch.float32), (d_idx, torch.int64), (d_dist, torch.float32)):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dt):
            raise ValueError("device tensors must be contiguous HIP tensors of the documented dtypes")
    m = dQ.shape[0]
    if dQ.shape != (m, tree.d) or d_idx.shape != (m, k) or d_dist.shape != (m, k):
        raise ValueError("shape mismatch")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().bkd_query_async_noalloc(tree.handle, dQ.data_ptr(), m, k, d_idx.data_ptr(), d_dist.data_ptr(),
                                         ctypes.c_void_p(s.cuda_stream)))


def tree_rules_export(tree: Tree, boxes: bool = False):
    """(dims [2^h-1] int32, boxes [2^(h+1)-1, 2, d] float32 or None) of a tree: every internal
    node's splitting dimension and, for a tree built with PRUNE_BOX, every node's box."""
    nleaf = 1 << tree.height
    dims = np.zeros(max(nleaf - 1, 1), dtype=np.int32)
    box = np.zeros((2 * nleaf - 1, 2, tree.d), dtype=np.float32) if boxes else None
    _check(lib().bkd_tree_rules_export(tree.handle, _p(dims), _p(box) if boxes else None))
    return dims[: nleaf - 1], box


def tree_info(tree: Tree) -> TreeInfo:
    info = TreeInfo()
    _check(lib().bkd_tree_info_get(tree.handle, ctypes.byref(info)))
    return info


def tree_export(tree: Tree):
    """(split [2^h-1] float32, leaf_off [2^h+1] int64, perm [n] int32)."""
    nleaf = 1 << tree.height
    split = np.zeros(max(nleaf - 1, 1), dtype=np.float32)
    leaf_off = np.zeros(nleaf + 1, dtype=np.int64)
    perm = np.zeros(tree.n, dtype=np.int32)
    _check(lib().bkd_tree_export(tree.handle, _p(split), _p(leaf_off), _p(perm)))
    return split[: nleaf - 1], leaf_off, perm


def chunk_plan(tree: Tree):
    N = tree_info(tree).num_chunks
    lo = np.zeros(N, dtype=np.int64)
    hi = np.zeros(N, dtype=np.int64)
    _check(lib().bkd_chunk_plan(tree.handle, _p(lo), _p(hi)))
    return lo, hi


def last_stats(tree: Tree) -> dict:
    s = Stats()
    _check(lib().bkd_last_stats(tree.handle, ctypes.byref(s)))
    return s.as_dict()


def trace(tree: Tree):
    """(call_off int64 [calls+1], query int32 [len], leaf int32 [len]) of the last traced query."""
    nc, ln = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().bkd_trace_size(tree.handle, ctypes.byref(nc), ctypes.byref(ln)))
    off = np.zeros(nc.value + 1, dtype=np.int64)
    q = np.zeros(max(ln.value, 1), dtype=np.int32)
    leaf = np.zeros(max(ln.value, 1), dtype=np.int32)
    _check(lib().bkd_trace_get(tree.handle, _p(off), _p(q), _p(leaf)))
    return off, q[: ln.value], leaf[: ln.value]


# ---------------------------------------------------------------------------
# Batched form

class Instance(ctypes.Structure):
    _fields_ = [("P", ctypes.c_void_p), ("n", ctypes.c_int64), ("Q", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("d", ctypes.c_int32), ("k", ctypes.c_int32), ("height", ctypes.c_int32),
                ("out_idx", ctypes.c_void_p), ("out_dist", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("leaves_per_task", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32), ("solo_max", ctypes.c_int32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_int64), ("queries", ctypes.c_int64), ("tasks", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("pairs", ctypes.c_int64), ("flops", ctypes.c_int64),
                ("run_ms", ctypes.c_double), ("error", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("claim_wait_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Batch:
    """Handle of ``bkd_batch_create``; keeps the host arrays it refers to alive."""

    def __init__(self, handle, arrays, outputs):
        self._h, self._arrays, self.outputs = handle, arrays, outputs

    @property
    def handle(self):
        if not self._h:
            raise ValueError("batch has been freed")
        return self._h

    def free(self):
        if self._h:
            _check(lib().bkd_batch_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def batch_create(instances, device: int = 0, flags: int = 0) -> Batch:
    """``bkd_batch_create``: instances = iterable of (P [n,d], Q [m,d], k, height); numpy
    arrays, or with FLAG_DEVICE_PTRS torch float32 tensors on the GPU (the outputs are then
    torch tensors on the GPU too)."""
    inst = (Instance * max(1, len(instances)))()
    arrays, outputs = [], []
    if flags & FLAG_DEVICE_PTRS:
        import torch
        for i, (P, Q, k, h) in enumerate(instances):
            P = P.contiguous()
            Q = Q.contiguous()
            m = Q.shape[0]
            oi = torch.zeros((m, k), dtype=torch.int64, device=P.device)
            od = torch.zeros((m, k), dtype=torch.float32, device=P.device)
            arrays += [P, Q]
            outputs.append((oi, od))
            inst[i] = Instance(P.data_ptr(), P.shape[0], Q.data_ptr() if m else None, m, P.shape[1], k, h,
                               oi.data_ptr() if m else None, od.data_ptr() if m else None)
        h = ctypes.c_void_p()
        _check(lib().bkd_batch_create(ctypes.cast(inst, ctypes.c_void_p), len(instances), device, flags,
                                      ctypes.byref(h)))
        return Batch(h.value, arrays, outputs)
    for i, (P, Q, k, h) in enumerate(instances):
        P = np.ascontiguousarray(P, dtype=np.float32)
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        m = Q.shape[0]
        oi = np.zeros((m, k), dtype=np.int64)
        od = np.zeros((m, k), dtype=np.float32)
        arrays += [P, Q]
        outputs.append((oi, od))
        inst[i] = Instance(P.ctypes.data, P.shape[0], Q.ctypes.data, m, P.shape[1], k, h, oi.ctypes.data,
                           od.ctypes.data)
    h = ctypes.c_void_p()
    _check(lib().bkd_batch_create(ctypes.cast(inst, ctypes.c_void_p), len(instances), device, flags,
                                  ctypes.byref(h)))
    return Batch(h.value, arrays, outputs)


def batch_run(batch: Batch, tuning: Tuning | None = None, stream=None):
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib().bkd_batch_run(batch.handle, ctypes.byref(tuning) if tuning is not None else None, s))


def batch_results(batch: Batch):
    """``bkd_batch_results``: list of (idx [m,k], dist [m,k]) per instance."""
    _check(lib().bkd_batch_results(batch.handle))
    return batch.outputs


def batch_autotune(batch: Batch):
    t = Tuning()
    ms = ctypes.c_double()
    _check(lib().bkd_batch_autotune(batch.handle, ctypes.byref(t), ctypes.byref(ms)))
    return t, ms.value


def batch_tuning_save(batch: Batch, path: str):
    """``bkd_batch_tuning_save``: the batch's tuning into the cache file."""
    _check(lib().bkd_batch_tuning_save(batch.handle, path.encode()))


def batch_tuning_load(batch: Batch, path: str):
    """``bkd_batch_tuning_load``: the cached tuning of this batch (raises ENOTFOUND if absent)."""
    t = Tuning()
    _check(lib().bkd_batch_tuning_load(batch.handle, path.encode(), ctypes.byref(t)))
    return t


def batch_stats(batch: Batch) -> dict:
    st = BatchStats()
    _check(lib().bkd_batch_stats_get(batch.handle, ctypes.byref(st)))
    return st.as_dict()


# ---------------------------------------------------------------------------
# Served form

REQ_WAITING, REQ_RUNNING, REQ_DONE, REQ_CANCELLED = 0, 1, 2, 3


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots_per_session", ctypes.c_int64), ("max_requests", ctypes.c_int32), ("device", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("age_max", ctypes.c_int32), ("tail_max", ctypes.c_int64),
                ("straggle_max", ctypes.c_int32)]


class Request:
    def __init__(self, rid, Q, idx, dist):
        self.id, self._Q, self.idx, self.dist = rid, Q, idx, dist


class Server:
    """Handle of ``bkd_server_create``.  It keeps the served trees alive, and every
    submitted request's arrays (queries, idx and dist outputs, which the library
    writes when the request completes) until ``release`` or ``destroy``: a caller may
    drop a request handle, or cancel a running request, without the library writing
    into freed memory."""

    def __init__(self, handle):
        self._h, self.trees, self.requests = handle, [], {}

    @property
    def handle(self):
        if not self._h:
            raise ValueError("server has been destroyed")
        return self._h

    def request(self, rid: int) -> Request:
        """The live request with id ``rid`` (submitted and not yet released)."""
        return self.requests[rid]

    def destroy(self):
        if self._h:
            _check(lib().bkd_server_destroy(self._h))
            self._h = None
        # the library no longer writes to any request's arrays
        self.requests.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def server_create(slots_per_session: int = 0, max_requests: int = 0, device: int = 0, flags: int = 0,
                  age_max: int = 0, tail_max: int = 0, straggle_max: int = 0) -> Server:
    o = ServerOpts(slots_per_session, max_requests, device, flags, age_max, tail_max, straggle_max)
    h = ctypes.c_void_p()
    _check(lib().bkd_server_create(ctypes.byref(o), ctypes.byref(h)))
    return Server(h.value)


def server_add_tree(srv: Server, tree: Tree) -> int:
    tid = ctypes.c_int32()
    _check(lib().bkd_server_add_tree(srv.handle, tree.handle, ctypes.byref(tid)))
    srv.trees.append(tree)
    return tid.value


def submit(srv: Server, tree_id: int, Q, k: int) -> Request:
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    m = Q.shape[0]
    idx = np.zeros((m, k), dtype=np.int64)
    dist = np.zeros((m, k), dtype=np.float32)
    rid = ctypes.c_int64()
    _check(lib().bkd_submit(srv.handle, tree_id, _p(Q), m, k, _p(idx), _p(dist), ctypes.byref(rid)))
    req = Request(rid.value, Q, idx, dist)
    srv.requests[req.id] = req
    return req


def _rid(req) -> int:
    return req.id if isinstance(req, Request) else int(req)


def wait(srv: Server, req, timeout_us: int = -1):
    """Block until the request (a Request or its id) is done; returns its (idx, dist)."""
    rid = _rid(req)
    _check(lib().bkd_wait(srv.handle, rid, timeout_us))
    r = srv.requests[rid]
    return r.idx, r.dist


def poll(srv: Server, req) -> int:
    st = ctypes.c_int32()
    _check(lib().bkd_poll(srv.handle, _rid(req), ctypes.byref(st)))
    return st.value


def cancel(srv: Server, req):
    _check(lib().bkd_cancel(srv.handle, _rid(req)))


class ServerStats(ctypes.Structure):
    _fields_ = [("sessions", ctypes.c_int32), ("rounds", ctypes.c_int64), ("scan_rounds", ctypes.c_int64),
                ("tail_rounds", ctypes.c_int64), ("queries", ctypes.c_int64), ("busy_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("complete_s", ctypes.c_double), ("direct_launches", ctypes.c_int64),
                ("aged_queries", ctypes.c_int64)]


def server_stats(srv: Server) -> dict:
    """``bkd_server_stats_get``."""
    st = ServerStats()
    _check(lib().bkd_server_stats_get(srv.handle, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in ServerStats._fields_}


def request_times(srv: Server, req):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().bkd_request_times(srv.handle, _rid(req), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def release(srv: Server, req):
    """Forget a finished request; its arrays are no longer kept by the server."""
    rid = _rid(req)
    _check(lib().bkd_release(srv.handle, rid))
    srv.requests.pop(rid, None)
