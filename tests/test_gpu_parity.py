"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars:
  * tree (split, leaf_off, perm): bit-exact with the oracle's canonical build;
  * per-call buffer contents and leaf assignments: bit-exact with the oracle's
    replay of Algorithm 1 under the same B and M;
  * (index, float32 squared distance) keys: bit-exact with the oracle's
    exhaustive float32 search;
  * Euclidean distances: |gpu - fp64| <= 1e-5 * fp64 per rank, index lists
    equal to the float64 ones except inside that tie band.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import datagen
import oracle
import paper_1512_02831_amd as bkd

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32_keys(idx, d2):
    return (d2.astype(np.float32).view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)


def gpu_keys(P, Q, k, height, **opts):
    flags = opts.pop("flags", 0) | bkd.FLAG_SQUARED
    with bkd.build(P, height, flags=flags, **opts) as t:
        idx, d2 = bkd.query(t, Q, k)
        tr = bkd.trace(t) if flags & bkd.FLAG_TRACE else None
        st = bkd.last_stats(t)
        info = bkd.tree_info(t)
    return f32_keys(idx, d2), tr, st, info


def check_fp64(P, Q, idx, dist, k, ref=None):
    """Distances within TOL of float64; index lists equal outside the tie band."""
    i64, d64sq = ref if ref is not None else oracle.brute_f64(P, Q, k)
    d64 = np.sqrt(d64sq)
    assert np.all(np.abs(dist.astype(np.float64) - d64) <= TOL * d64 + 1e-30)
    assert np.all(np.diff(dist, axis=1) >= 0)
    kth = d64[:, -1:]
    for qi in np.nonzero(np.any(idx != i64, axis=1))[0]:
        extra = set(idx[qi]) - set(i64[qi])
        for j in extra:
            dj = math.sqrt(float(np.sum((P[j].astype(np.float64) - Q[qi].astype(np.float64)) ** 2)))
            assert dj <= (1 + TOL) * kth[qi, 0], (qi, j)
        # ranks may only swap inside the tie band
        for r in range(k):
            if idx[qi, r] != i64[qi, r]:
                assert abs(dist[qi, r] - d64[qi, r]) <= TOL * d64[qi, r] + 1e-30


def check_trace(tr, rep):
    off, q, leaf = tr
    assert len(off) - 1 == rep.ncalls
    assert np.array_equal(off, rep.call_off)
    assert np.array_equal(q, rep.trace_q.astype(np.int32))
    assert np.array_equal(leaf, rep.trace_r)


# ---------------------------------------------------------------------------

def test_small_uniform_config_full_parity():
    # 2^15 points, 2^12 queries, d=10 uniform, k=10, height 6, paper B and M
    say("case: small uniform n=2^15 m=2^12 d=10 k=10 h=6")
    P, Q = datagen.small_uniform()
    k, h = 10, 6
    t_or = oracle.build_tree(P, h)
    with bkd.build(P, h, flags=bkd.FLAG_TRACE | bkd.FLAG_SQUARED) as t:
        split, leaf_off, perm = bkd.tree_export(t)
        assert np.array_equal(split.view(np.uint32), t_or.split.view(np.uint32))
        assert np.array_equal(leaf_off, t_or.leaf_off) and np.array_equal(perm, t_or.perm)
        info = bkd.tree_info(t)
        assert (info.buffer_size, info.fetch_size, info.resident) == (1 << 18, 10 << 18, 1)
        idx, d2 = bkd.query(t, Q, k)
        tr = bkd.trace(t)
        st = bkd.last_stats(t)
    keys = f32_keys(idx, d2)
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))
    rep = oracle.replay(P, t_or, Q, k, B=1 << 18, M=10 << 18)
    check_trace(tr, rep)
    assert st["pairs"] == rep.pairs and st["calls"] == rep.ncalls
    with bkd.build(P, h) as t:
        idx2, dist = bkd.query(t, Q, k)
    assert np.array_equal(idx2, idx)
    check_fp64(P, Q, idx2, dist, k)


@pytest.mark.parametrize("B,M", [(-1, -1), (64, 300), (8, 1000), (1, 37)])
def test_schedules_match_replay(B, M):
    say(f"case: schedule B={B} M={M}")
    P, Q = datagen.mixture_pq(seed=21, n=20_000, m=3000, d=6, comps=8)
    k, h = 7, 5
    keys, tr, st, _ = gpu_keys(P, Q, k, h, buffer_size=B, fetch_size=M, flags=bkd.FLAG_TRACE)
    t_or = oracle.build_tree(P, h)
    rep = oracle.replay(P, t_or, Q, k, B=max(B, 0), M=max(M, 0))
    check_trace(tr, rep)
    assert np.array_equal(keys, rep.keys)
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))


def visit_multiset(tr):
    _, q, leaf = tr
    keep = leaf >= 0
    return sorted(zip(q[keep].tolist(), leaf[keep].tolist()))


@pytest.mark.parametrize("mode,budget,N", [(bkd.CHUNK_LEAF, 0, 2), (bkd.CHUNK_LEAF, 0, 7), (bkd.CHUNK_POSITION, 0, 3),
                                           (bkd.CHUNK_POSITION, 0, 64), (bkd.CHUNK_LEAF, 200_000, 0),
                                           (bkd.CHUNK_POSITION, 150_000, 0), (bkd.CHUNK_LEAF, 0, 64)])
def test_streamed_lockstep_identical_to_resident(mode, budget, N):
    # Leaf-aligned chunks run the chunk sweep (drain one resident chunk at a time); position chunks
    # stream every chunk holding a buffered leaf in each round.  Results, pairs and the multiset of
    # (query, leaf) visits equal the resident run.
    say(f"case: lock-step chunks mode={mode} budget={budget} N={N}")
    P, Q = datagen.mixture_pq(seed=5, n=30_001, m=2500, d=5, comps=6)
    k, h = 10, 6
    ref, tr_ref, st_ref, _ = gpu_keys(P, Q, k, h, fetch_size=-1, buffer_size=-1, flags=bkd.FLAG_TRACE)
    keys, tr, st, info = gpu_keys(P, Q, k, h, fetch_size=-1, buffer_size=-1, flags=bkd.FLAG_TRACE,
                                  chunk_mode=mode, leaf_budget_bytes=budget, num_chunks=N)
    assert info.resident == 0 and info.num_chunks >= 2
    assert np.array_equal(keys, ref)
    assert visit_multiset(tr) == visit_multiset(tr_ref)
    if mode == bkd.CHUNK_POSITION:
        for a, b in zip(tr, tr_ref):
            assert np.array_equal(a, b)
    assert st["pairs"] == st_ref["pairs"] and st["chunk_copies"] >= 1
    with bkd.build(P, h, chunk_mode=mode, leaf_budget_bytes=budget, num_chunks=N) as t:
        lo, hi = bkd.chunk_plan(t)
        if mode == bkd.CHUNK_POSITION:
            olo, ohi = oracle.chunk_bounds(P.shape[0], len(lo))
            assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
        else:
            _, leaf_off, _ = bkd.tree_export(t)
            assert set(lo.tolist()) <= set(leaf_off.tolist()) and set(hi.tolist()) <= set(leaf_off.tolist())
        assert lo[0] == 0 and hi[-1] == P.shape[0] and np.all(lo[1:] == hi[:-1])
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))


@pytest.mark.parametrize("budget,N,tail_max", [(0, 5, 0), (0, 12, 300), (200_000, 0, 1), (0, 3, 2)])
def test_streamed_sweep_tail_matches_resident(budget, N, tail_max):
    # The chunk sweep hands a resident chunk's pending queries to the tail kernel once at most
    # tail_max are left there; each walks on while its next leaf is in that chunk.  Keys, visits and
    # pairs equal a resident run that keeps rounds to the end.
    say(f"case: sweep tail budget={budget} N={N} tail_max={tail_max}")
    P, Q = datagen.mixture_pq(seed=9, n=40_000, m=3000, d=6, comps=6)
    k, h = 10, 7
    ref, _, st_ref, _ = gpu_keys(P, Q, k, h, fetch_size=-1, buffer_size=-1, flags=bkd.FLAG_NO_TAIL)
    keys, _, st, info = gpu_keys(P, Q, k, h, fetch_size=-1, buffer_size=-1, chunk_mode=bkd.CHUNK_LEAF,
                                 leaf_budget_bytes=budget, num_chunks=N, tail_max=tail_max)
    assert info.resident == 0 and info.num_chunks >= 2
    assert np.array_equal(keys, ref)
    assert st["visits"] == st_ref["visits"] and st["pairs"] == st_ref["pairs"]
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))


def test_streamed_sweep_wide_tail_matches_oracle():
    # leaves of 4096 points: the chunk sweep's tail runs 512-lane workgroups
    say("case: sweep tail with 4096-point leaves, N=3")
    P, Q = datagen.mixture_pq(seed=21, n=1 << 16, m=4000, d=10, comps=6)
    k, h = 10, 4
    ref, _, st_ref, _ = gpu_keys(P, Q, k, h, fetch_size=-1, buffer_size=-1, flags=bkd.FLAG_NO_TAIL)
    keys, _, st, info = gpu_keys(P, Q, k, h, fetch_size=-1, buffer_size=-1, chunk_mode=bkd.CHUNK_LEAF,
                                 num_chunks=3, tail_max=0)
    assert info.resident == 0 and info.num_chunks >= 2
    assert np.array_equal(keys, ref)
    assert st["visits"] == st_ref["visits"] and st["pairs"] == st_ref["pairs"]
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))


@pytest.mark.parametrize("mode,N,B,M", [(bkd.CHUNK_LEAF, 5, 64, 500), (bkd.CHUNK_POSITION, 4, 0, 0),
                                        (bkd.CHUNK_POSITION, 9, 16, 100)])
def test_streamed_algorithm1_matches_replay(mode, N, B, M):
    # The paper's scheme: each ProcessAllBuffers call streams the chunks holding buffered leaves
    # through two device buffers; buffer contents per call equal the oracle's replay.
    say(f"case: Algorithm 1 streamed mode={mode} N={N} B={B} M={M}")
    P, Q = datagen.mixture_pq(seed=15, n=12_345, m=1500, d=7, comps=5)
    k, h = 6, 5
    keys, tr, st, info = gpu_keys(P, Q, k, h, chunk_mode=mode, num_chunks=N, buffer_size=B, fetch_size=M,
                                  flags=bkd.FLAG_TRACE)
    assert info.resident == 0
    o = bkd.default_options(h)
    t_or = oracle.build_tree(P, h)
    rep = oracle.replay(P, t_or, Q, k, B=B or o.buffer_size, M=M or o.fetch_size)
    check_trace(tr, rep)
    assert np.array_equal(keys, rep.keys)
    assert st["chunk_copies"] >= 1


@pytest.mark.parametrize("n,m,d,k,h", [
    (1000, 300, 3, 5, 0),      # one leaf: the loop reduces to one exhaustive scan
    (777, 500, 1, 4, 5),       # d = 1
    (5000, 400, 32, 8, 4),     # largest dimension
    (60, 20, 4, 60, 2),        # k = n
    (3000, 200, 7, 64, 3),     # largest k, ragged leaves
    (4097, 1, 9, 1, 7),        # one query, k = 1
    (999, 257, 15, 32, 6),     # d=15, k=32 (batched-form shapes)
    (2048, 300, 11, 3, 11),    # leaves of one point
])
def test_edge_shapes(n, m, d, k, h):
    say(f"case: edge n={n} m={m} d={d} k={k} h={h}")
    P, Q = datagen.mixture_pq(seed=n + d, n=n, m=m, d=d, comps=3)
    keys, tr, st, _ = gpu_keys(P, Q, k, h, flags=bkd.FLAG_TRACE)
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))
    t_or = oracle.build_tree(P, h)
    o = bkd.default_options(h)
    check_trace(tr, oracle.replay(P, t_or, Q, k, B=o.buffer_size, M=o.fetch_size))


@pytest.mark.parametrize("n,m,d,k,h,tail_max", [
    (1 << 16, 6000, 10, 10, 6, 2048),  # rounds first, then the tail below 2048 pending queries
    (20000, 700, 5, 32, 5, 0),         # default threshold: tail right after the first round's sort
    (5000, 300, 15, 64, 4, 0),         # largest k in the tail
    (3000, 2048, 3, 1, 8, 2048),       # exactly the hand-over size
    (40000, 3000, 10, 10, 7, 1),       # a single pending query left for the tail
    (1 << 16, 5000, 10, 10, 4, 0),     # leaves of 4096 points: 512-lane tail workgroups
    (1 << 15, 1000, 5, 64, 3, 0),      # the same with the largest k
])
def test_lockstep_tail_matches_rounds_and_oracle(n, m, d, k, h, tail_max):
    say(f"case: tail n={n} m={m} d={d} k={k} h={h} tail_max={tail_max}")
    P, Q = datagen.mixture_pq(seed=n + m, n=n, m=m, d=d, comps=5)
    tail, _, st_tail, _ = gpu_keys(P, Q, k, h, buffer_size=-1, fetch_size=-1, tail_max=tail_max)
    rounds, _, st_rounds, _ = gpu_keys(P, Q, k, h, buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_NO_TAIL)
    assert np.array_equal(tail, rounds)
    assert np.array_equal(tail, oracle.brute_f32c(P, Q, k))
    # the same visits and pairs, whichever schedule finished the traversals
    assert st_tail["visits"] == st_rounds["visits"] and st_tail["pairs"] == st_rounds["pairs"]


def test_wide_reference_coordinates_keep_results_exact():
    """Reference points in clusters around +-1e20 (beyond the dense filter's range): the dense scan
    takes its exact path, and keys stay bit-exact (finite distances inside a cluster, +inf across)."""
    say("case: wide reference coordinates")
    rng = np.random.default_rng(11)
    d, n, m, k = 5, 12000, 3000, 10
    centres = rng.choice([-1e20, 1e20], size=(4, d))
    P = (centres[rng.integers(0, 4, n)] + rng.normal(0, 1e17, (n, d))).astype(np.float32)
    Q = (centres[rng.integers(0, 4, m)] + rng.normal(0, 1e17, (m, d))).astype(np.float32)
    keys, _, st, _ = gpu_keys(P, Q, k, 5, buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_NO_TAIL)
    assert st["dense_pairs"] > 0
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))


def test_one_wide_query_keeps_results_exact():
    """A single query beyond the filter's range switches the whole call to exact dense scans."""
    say("case: one wide query")
    P, Q = datagen.mixture_pq(seed=77, n=30000, m=2000, d=10, comps=5)
    Q = Q.copy()
    Q[5] = np.float32(3e19)
    Q[6, 0] = np.float32(-7e18)
    k = 10
    keys, _, st, _ = gpu_keys(P, Q, k, 6, buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_NO_TAIL)
    assert st["dense_pairs"] > 0
    assert np.array_equal(keys, oracle.brute_f32c(P, Q, k))


def test_lattice_exact_including_ties():
    say("case: lattice ties")
    P = datagen.lattice(2, 1, 6000, 5, side=5)
    Q = datagen.lattice(2, 2, 800, 5, side=5)
    k = 12
    with bkd.build(P, 6, flags=bkd.FLAG_SQUARED) as t:
        idx, d2 = bkd.query(t, Q, k)
    Pi, Qi = P.astype(np.int64), Q.astype(np.int64)
    for qi in range(len(Q)):
        dd = ((Pi - Qi[qi]) ** 2).sum(axis=1)
        order = np.lexsort((np.arange(len(P)), dd))[:k]
        assert np.array_equal(idx[qi], order)
        assert np.array_equal(d2[qi], dd[order].astype(np.float32))


def test_duplicates_and_self_queries():
    say("case: duplicates / self")
    rng = np.random.default_rng(3)
    base = rng.random((500, 4)).astype(np.float32)
    P = np.concatenate([base, base, base[:100]])  # every point twice or three times
    with bkd.build(P, 5) as t:
        idx, dist = bkd.query(t, base, 3)
    assert np.all(dist[:, :2] == 0)
    assert np.all(idx[:, 0] == np.arange(500)) and np.all(idx[:, 1] == np.arange(500) + 500)
    first = np.arange(100)
    assert np.all(idx[first, 2] == first + 1000)


def test_async_device_path_matches_host_path():
    import torch
    say("case: async device tensors")
    P, Q = datagen.mixture_pq(seed=9, n=50_000, m=5000, d=10, comps=16)
    k = 10
    with bkd.build(P, 7, fetch_size=-1, buffer_size=-1) as t:
        idx, dist = bkd.query(t, Q, k)
        dQ = torch.from_numpy(Q).to("cuda")
        di = torch.empty((len(Q), k), dtype=torch.int64, device="cuda")
        dd = torch.empty((len(Q), k), dtype=torch.float32, device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            bkd.query_async(t, dQ, k, di, dd, stream=s)
        s.synchronize()
        assert np.array_equal(di.cpu().numpy(), idx) and np.array_equal(dd.cpu().numpy(), dist)


def test_error_paths_on_device():
    say("case: errors")
    P, Q = datagen.mixture_pq(seed=1, n=1000, m=10, d=3, comps=2)
    with bkd.build(P, 3) as t:
        bad = Q.copy()
        bad[4, 1] = np.inf
        with pytest.raises(bkd.BkdError) as e:
            bkd.query(t, bad, 3)
        assert e.value.code == bkd.EINVAL
        with pytest.raises(bkd.BkdError) as e:
            bkd.query(t, Q, 1001)
        assert e.value.code == bkd.EINVAL
        idx, _ = bkd.query(t, Q, 3)  # tree still valid
        assert idx.shape == (10, 3)
        idx0, _ = bkd.query(t, Q[:0], 3)
        assert idx0.shape == (0, 3)
    with pytest.raises(bkd.BkdError) as e:
        bkd.build(P, 3, leaf_budget_bytes=1000)
    assert e.value.code == bkd.EBUDGET


def test_on_device_config_sampled_parity():
    # 2^22 reference and query points, d=10 16-component mixture, k=10, height 10, in the
    # benchmark's launch configuration (lock-step rounds); outputs checked on a sample.
    say("case: on-device n=m=2^22 h=10 (sampled)")
    P, Q = datagen.mixture_pq()
    k, h = 10, 10
    with bkd.build(P, h, fetch_size=-1, buffer_size=-1, flags=bkd.FLAG_SQUARED) as t:
        split, leaf_off, perm = bkd.tree_export(t)
        idx, d2 = bkd.query(t, Q, k)
        st = bkd.last_stats(t)
    say("  gpu done", st)
    assert np.all(np.diff(d2, axis=1) >= 0) and idx.min() >= 0 and idx.max() < len(P)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(len(Q), 3000, replace=False))
    # the oracle traverses its own canonical tree, built from P alone
    t_or = oracle.build_tree(P, h)
    assert np.array_equal(split.view(np.uint32), t_or.split.view(np.uint32))
    assert np.array_equal(leaf_off, t_or.leaf_off)
    okeys, _, _ = oracle.traverse_many_f32(P, t_or, Q[sample], k)
    assert np.array_equal(f32_keys(idx[sample], d2[sample]), okeys)
    sub = sample[:200]
    check_fp64(P, Q[sub], idx[sub], np.sqrt(d2[sub]), k)


@pytest.mark.parametrize("n,d,h,kind", [
    (1000, 3, 0, "normal"),
    (5000, 4, 5, "normal"),
    (33_333, 10, 9, "normal"),
    (4096, 2, 12, "normal"),        # leaves of one point
    (20_000, 5, 7, "duplicates"),   # many equal coordinates: ties by index
    (6000, 3, 6, "signed_zeros"),   # -0 and +0 compare equal
    (1 << 20, 10, 13, "normal"),    # node keys of 13 bits: more radix passes
])
def test_device_build_matches_oracle(n, d, h, kind):
    say(f"case: device build n={n} d={d} h={h} {kind}")
    rng = np.random.default_rng(n + d + h)
    P = rng.standard_normal((n, d)).astype(np.float32)
    if kind == "duplicates":
        P = np.round(P * 2.0).astype(np.float32)
    if kind == "signed_zeros":
        P[rng.random((n, d)) < 0.3] = np.float32(0.0)
        P[rng.random((n, d)) < 0.3] = np.float32(-0.0)
    t_or = oracle.build_tree(P, h)
    with bkd.build(P, h, flags=bkd.FLAG_DEVICE_BUILD | bkd.FLAG_SQUARED) as t:
        split, leaf_off, perm = bkd.tree_export(t)
        Q = P[rng.choice(n, 200)] + np.float32(0.01)
        idx, d2 = bkd.query(t, Q, 5)
    assert np.array_equal(split.view(np.uint32), t_or.split.view(np.uint32))
    assert np.array_equal(leaf_off, t_or.leaf_off)
    assert np.array_equal(perm, t_or.perm)
    assert np.array_equal(f32_keys(idx, d2), oracle.brute_f32c(P, Q, 5))
