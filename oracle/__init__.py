"""Python access to the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline call this package; the product library never does.  The oracle is a
plain C program built with gcc (no GPU code); see ``oracle.c`` for which
passage of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EMPTY_KEY = np.uint64(0x7F800000FFFFFFFF)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE float32 semantics: no contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    lib.orc_build.argtypes = [P, i64, i32, i32, P, P, P]
    lib.orc_build.restype = ctypes.c_int
    lib.orc_build_rules.argtypes = [P, i64, i32, i32, i32, P, P, P, P]
    lib.orc_build_rules.restype = ctypes.c_int
    lib.orc_node_boxes.argtypes = [P, i32, i32, P, P, P]
    lib.orc_node_boxes.restype = ctypes.c_int
    lib.orc_traverse_f32_rules.argtypes = [P, i32, i32, P, P, P, P, P, P, i32, P, i64, P]
    lib.orc_traverse_f32_rules.restype = i64
    lib.orc_traverse_many_f32_rules.argtypes = [P, i32, i32, P, P, P, P, P, P, i64, i32, P, P, i32]
    lib.orc_traverse_many_f32_rules.restype = ctypes.c_int
    lib.orc_brute_f64.argtypes = [P, i64, P, i64, i32, i32, P, P, i32]
    lib.orc_brute_f64.restype = ctypes.c_int
    lib.orc_brute_f32c.argtypes = [P, i64, P, i64, i32, i32, P, i32]
    lib.orc_brute_f32c.restype = ctypes.c_int
    lib.orc_kdtree_f64.argtypes = [P, i64, P, i64, i32, i32, i32, P, P, i32]
    lib.orc_kdtree_f64.restype = ctypes.c_int
    lib.orc_kdtree_f64_build.argtypes = [P, i64, i32, i32, i32]
    lib.orc_kdtree_f64_build.restype = P
    lib.orc_kdtree_f64_query.argtypes = [P, P, i64, i32, P, P, i32]
    lib.orc_kdtree_f64_query.restype = ctypes.c_int
    lib.orc_kdtree_f64_free.argtypes = [P]
    lib.orc_kdtree_f64_free.restype = None
    lib.orc_leaf_chunks.argtypes = [P, i32, i32, i64, i64, P]
    lib.orc_leaf_chunks.restype = i64
    lib.orc_traverse_f32.argtypes = [P, i32, i32, P, P, P, P, i32, P, i64, P]
    lib.orc_traverse_f32.restype = i64
    lib.orc_traverse_many_f32.argtypes = [P, i32, i32, P, P, P, P, i64, i32, P, P, P, i32]
    lib.orc_traverse_many_f32.restype = ctypes.c_int
    lib.orc_replay_run.argtypes = [P, i64, i32, i32, P, P, P, P, i64, i32, i64, i64, i32, i32]
    lib.orc_replay_run.restype = P
    for name in ("orc_replay_ncalls", "orc_replay_nfetch", "orc_replay_pairs", "orc_replay_trace_len"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = i64
    lib.orc_replay_get.argtypes = [P, P, P, P, P]
    lib.orc_replay_get.restype = None
    lib.orc_replay_free.argtypes = [P]
    lib.orc_replay_free.restype = None
    lib.orc_chunk_bounds.argtypes = [i64, i64, P, P]
    lib.orc_chunk_bounds.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def max_threads() -> int:
    return int(_load().orc_max_threads())


class Tree:
    """Canonical tree arrays: split (heap order), leaf_off, perm."""

    def __init__(self, split, leaf_off, perm, height, d, dims=None):
        self.split, self.leaf_off, self.perm, self.height, self.d = split, leaf_off, perm, height, d
        # splitting dimension per internal node (None: level mod d, the original rule)
        self.dims = dims


def build_tree(P, height: int) -> Tree:
    P = _f32(P)
    n, d = P.shape
    nleaf = 1 << height
    split = np.zeros(max(nleaf - 1, 1), dtype=np.float32)
    leaf_off = np.zeros(nleaf + 1, dtype=np.int64)
    perm = np.zeros(n, dtype=np.int32)
    rc = _load().orc_build(_ptr(P), n, d, height, _ptr(split), _ptr(leaf_off), _ptr(perm))
    if rc != 0:
        raise ValueError("orc_build rejected its arguments")
    return Tree(split[: nleaf - 1], leaf_off, perm, height, d)


SPLIT_CYCLIC, SPLIT_LONGEST = 0, 1


def build_tree_rules(P, height: int, rule: int) -> Tree:
    """The canonical tree under a splitting rule: SPLIT_CYCLIC (level mod d) or SPLIT_LONGEST
    (longest side of the node's bounding box); dims holds each internal node's dimension."""
    P = _f32(P)
    n, d = P.shape
    nleaf = 1 << height
    split = np.zeros(max(nleaf - 1, 1), dtype=np.float32)
    dims = np.zeros(max(nleaf - 1, 1), dtype=np.int32)
    leaf_off = np.zeros(nleaf + 1, dtype=np.int64)
    perm = np.zeros(n, dtype=np.int32)
    rc = _load().orc_build_rules(_ptr(P), n, d, height, rule, _ptr(split), _ptr(dims), _ptr(leaf_off), _ptr(perm))
    if rc != 0:
        raise ValueError("orc_build_rules rejected its arguments")
    return Tree(split[: nleaf - 1], leaf_off, perm, height, d, dims[: nleaf - 1])


def node_boxes(P, tree: Tree) -> np.ndarray:
    """Bounding box of every node's points, heap order over all 2^(h+1)-1 nodes: [nodes, 2, d]
    (row 0 the minima, row 1 the maxima)."""
    P = _f32(P)
    nodes = (2 << tree.height) - 1
    box = np.zeros((nodes, 2, tree.d), dtype=np.float32)
    if _load().orc_node_boxes(_ptr(P), tree.d, tree.height, _ptr(tree.leaf_off), _ptr(tree.perm), _ptr(box)) != 0:
        raise ValueError("orc_node_boxes rejected its arguments")
    return box


def traverse_f32_rules(P, tree: Tree, q, k: int, boxes=None, max_leaves: int = 1 << 16):
    """Leaf sequence and final keys of one query, walking with the tree's per-node dimensions
    and, if boxes is given, the far child's box term instead of the plane term."""
    P = _f32(P)
    q = _f32(q).reshape(-1)
    leaves = np.zeros(max_leaves, dtype=np.int32)
    keys = np.zeros(k, dtype=np.uint64)
    dims = np.ascontiguousarray(tree.dims, dtype=np.int32) if tree.dims is not None else None
    bx = np.ascontiguousarray(boxes, dtype=np.float32) if boxes is not None else None
    cnt = _load().orc_traverse_f32_rules(_ptr(P), tree.d, tree.height, _ptr(tree.split),
                                         _ptr(dims) if dims is not None else None,
                                         _ptr(bx) if bx is not None else None, _ptr(tree.leaf_off),
                                         _ptr(tree.perm), _ptr(q), k, _ptr(leaves), max_leaves, _ptr(keys))
    return leaves[: min(cnt, max_leaves)].copy(), keys


def traverse_many_f32_rules(P, tree: Tree, Q, k: int, boxes=None, threads: int = 0):
    """Final keys and leaves visited per query under the tree's rules (see traverse_f32_rules)."""
    P, Q = _f32(P), _f32(Q)
    m = Q.shape[0]
    keys = np.zeros((m, k), dtype=np.uint64)
    visits = np.zeros(m, dtype=np.int64)
    dims = np.ascontiguousarray(tree.dims, dtype=np.int32) if tree.dims is not None else None
    bx = np.ascontiguousarray(boxes, dtype=np.float32) if boxes is not None else None
    _load().orc_traverse_many_f32_rules(_ptr(P), tree.d, tree.height, _ptr(tree.split),
                                        _ptr(dims) if dims is not None else None,
                                        _ptr(bx) if bx is not None else None, _ptr(tree.leaf_off),
                                        _ptr(tree.perm), _ptr(Q), m, k, _ptr(keys), _ptr(visits), threads)
    return keys, visits


def brute_f64(P, Q, k: int, threads: int = 0):
    """Exact kNN in float64: (idx int64 [m,k], d2 float64 [m,k]), ties by smaller index."""
    P, Q = _f32(P), _f32(Q)
    m = Q.shape[0]
    idx = np.zeros((m, k), dtype=np.int64)
    d2 = np.zeros((m, k), dtype=np.float64)
    rc = _load().orc_brute_f64(_ptr(P), P.shape[0], _ptr(Q), m, P.shape[1], k, _ptr(idx), _ptr(d2), threads)
    if rc != 0:
        raise ValueError("orc_brute_f64 rejected its arguments")
    return idx, d2


def brute_f32c(P, Q, k: int, threads: int = 0) -> np.ndarray:
    """Exhaustive kNN under the float32 distance reading: uint64 keys [m,k]."""
    P, Q = _f32(P), _f32(Q)
    m = Q.shape[0]
    keys = np.zeros((m, k), dtype=np.uint64)
    rc = _load().orc_brute_f32c(_ptr(P), P.shape[0], _ptr(Q), m, P.shape[1], k, _ptr(keys), threads)
    if rc != 0:
        raise ValueError("orc_brute_f32c rejected its arguments")
    return keys


def kdtree_f64(P, Q, k: int, leaf_size: int = 32, threads: int = 0):
    P, Q = _f32(P), _f32(Q)
    m = Q.shape[0]
    idx = np.zeros((m, k), dtype=np.int64)
    d2 = np.zeros((m, k), dtype=np.float64)
    rc = _load().orc_kdtree_f64(_ptr(P), P.shape[0], _ptr(Q), m, P.shape[1], k, leaf_size, _ptr(idx), _ptr(d2),
                                threads)
    if rc != 0:
        raise ValueError("orc_kdtree_f64 rejected its arguments")
    return idx, d2


class KdTree64:
    """Classical float64 k-d tree (leaves of about `leaf_size` points), built once."""

    def __init__(self, P, leaf_size: int = 32, threads: int = 0):
        self.P = _f32(P)  # the C tree refers to these points
        self.d = self.P.shape[1]
        self._h = _load().orc_kdtree_f64_build(_ptr(self.P), self.P.shape[0], self.d, leaf_size, threads)
        if not self._h:
            raise ValueError("orc_kdtree_f64_build failed")

    def query(self, Q, k: int, threads: int = 0):
        Q = _f32(Q)
        m = Q.shape[0]
        idx = np.zeros((m, k), dtype=np.int64)
        d2 = np.zeros((m, k), dtype=np.float64)
        if _load().orc_kdtree_f64_query(self._h, _ptr(Q), m, k, _ptr(idx), _ptr(d2), threads) != 0:
            raise ValueError("orc_kdtree_f64_query failed")
        return idx, d2

    def __del__(self):
        if getattr(self, "_h", None):
            _load().orc_kdtree_f64_free(self._h)
            self._h = None


def traverse_f32(P, tree: Tree, q, k: int, max_leaves: int = 1 << 16):
    """Leaf sequence and final keys of one query (stackless float32 traversal)."""
    P = _f32(P)
    q = _f32(q).reshape(-1)
    leaves = np.zeros(max_leaves, dtype=np.int32)
    keys = np.zeros(k, dtype=np.uint64)
    cnt = _load().orc_traverse_f32(_ptr(P), tree.d, tree.height, _ptr(tree.split), _ptr(tree.leaf_off),
                                   _ptr(tree.perm), _ptr(q), k, _ptr(leaves), max_leaves, _ptr(keys))
    return leaves[: min(cnt, max_leaves)].copy(), keys


def traverse_many_f32(P, tree: Tree, Q, k: int, threads: int = 0):
    """Final keys, leaves visited and pairs scanned per query, each traversed on its own."""
    P, Q = _f32(P), _f32(Q)
    m = Q.shape[0]
    keys = np.zeros((m, k), dtype=np.uint64)
    visits = np.zeros(m, dtype=np.int64)
    pairs = np.zeros(m, dtype=np.int64)
    _load().orc_traverse_many_f32(_ptr(P), tree.d, tree.height, _ptr(tree.split), _ptr(tree.leaf_off),
                                  _ptr(tree.perm), _ptr(Q), m, k, _ptr(keys), _ptr(visits), _ptr(pairs), threads)
    return keys, visits, pairs


class Replay:
    """Result of replaying Algorithm 1: final keys and the per-call trace."""

    def __init__(self, keys, call_off, trace_q, trace_r, nfetch, pairs):
        self.keys, self.call_off, self.trace_q, self.trace_r = keys, call_off, trace_q, trace_r
        self.nfetch, self.pairs = nfetch, pairs

    @property
    def ncalls(self) -> int:
        return len(self.call_off) - 1

    def call(self, c: int):
        """(query, leaf) pairs fetched before call c, in fetch order (leaf -1 = finished)."""
        a, b = self.call_off[c], self.call_off[c + 1]
        return self.trace_q[a:b], self.trace_r[a:b]

    def buffers(self, c: int):
        """Buffer contents processed by call c: (leaf, query) in ascending leaf, buffer order."""
        q, r = self.call(c)
        keep = r >= 0
        q, r = q[keep], r[keep]
        order = np.argsort(r, kind="stable")
        return r[order], q[order]


def replay(P, tree: Tree, Q, k: int, B: int, M: int, trace: bool = True, threads: int = 0) -> Replay:
    P, Q = _f32(P), _f32(Q)
    lib = _load()
    m = Q.shape[0]
    h = lib.orc_replay_run(_ptr(P), P.shape[0], tree.d, tree.height, _ptr(tree.split), _ptr(tree.leaf_off),
                           _ptr(tree.perm), _ptr(Q), m, k, B, M, 1 if trace else 0, threads)
    if not h:
        raise ValueError("orc_replay_run failed")
    try:
        nc = lib.orc_replay_ncalls(h)
        tl = lib.orc_replay_trace_len(h)
        keys = np.zeros((m, k), dtype=np.uint64)
        call_off = np.zeros(nc + 1, dtype=np.int64)
        tq = np.zeros(max(tl, 1), dtype=np.int64)
        tr = np.zeros(max(tl, 1), dtype=np.int32)
        lib.orc_replay_get(h, _ptr(keys), _ptr(call_off), _ptr(tq), _ptr(tr))
        return Replay(keys, call_off, tq[:tl], tr[:tl], lib.orc_replay_nfetch(h), lib.orc_replay_pairs(h))
    finally:
        lib.orc_replay_free(h)


def chunk_bounds(n: int, N: int):
    lo = np.zeros(N, dtype=np.int64)
    hi = np.zeros(N, dtype=np.int64)
    if _load().orc_chunk_bounds(n, N, _ptr(lo), _ptr(hi)) != 0:
        raise ValueError("bad chunk arguments")
    return lo, hi


def leaf_chunks(tree: Tree, N: int = 0, cap_bytes: int = 0):
    """Leaf-aligned chunk plan: array of first leaves, chunk j holds leaves [first[j], first[j+1])."""
    nleaf = 1 << tree.height
    first = np.zeros(nleaf + 1, dtype=np.int64)
    c = _load().orc_leaf_chunks(_ptr(np.ascontiguousarray(tree.leaf_off, dtype=np.int64)), tree.height, tree.d,
                                N, cap_bytes, _ptr(first))
    if c < 0:
        raise ValueError("bad leaf chunk arguments")
    return first[: c + 1].copy()


def keys_split(keys: np.ndarray):
    """(d2 float32, index int64) from uint64 keys."""
    keys = np.asarray(keys, dtype=np.uint64)
    d2 = (keys >> np.uint64(32)).astype(np.uint32).view(np.float32)
    idx = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    return d2, idx


def outlier_scores(P, k: int, threads: int = 0):
    """Proximity-based outlier scores (Section 4, large-scale outlier detection; the score of
    a point is its mean distance to its k nearest neighbours among the other reference points,
    and points are ranked by it).  Written from the definition: exhaustive float32-contract
    kNN of every reference point against the reference set with k + 1 neighbours, the point's
    own entry dropped once (the first k kept when it is absent), distances sqrt(d2) in
    float32, their float64 sum in ascending order divided by k, rounded to float32.
    Returns (score float32 [n], order int64 [n]): order lists indices by score, largest first,
    equal scores by smaller index."""
    P = _f32(P)
    n = P.shape[0]
    keys = brute_f32c(P, P, k + 1, threads)
    d2, idx = keys_split(keys)
    dist = np.sqrt(d2)  # float32, correctly rounded
    score = np.empty(n, dtype=np.float32)
    for i in range(n):
        row = [j for j in range(k + 1)]
        own = np.nonzero(idx[i] == i)[0]
        if len(own):
            row.remove(int(own[0]))
        s = 0.0
        for j in row[:k]:
            s += float(dist[i, j])
        score[i] = np.float32(s / k)
    order = np.lexsort((np.arange(n), -score.astype(np.float64)))
    return score, order.astype(np.int64)
