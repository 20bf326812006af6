"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers.  It holds none of the method's
arithmetic (no distances, no tree, no selection), so the CPU oracle and the
HIP path can both consume its arrays without sharing any computation.

Generation is block-parallel and bit-reproducible: rows are produced in blocks
of ``BLOCK`` rows and block ``b`` of stream ``s`` draws from
``numpy.random.SeedSequence([seed, s, b])``.  The same (seed, stream, n, d)
therefore always yields the same float32 array, independent of thread count.

Streams: 0 = mixture parameters, 1 = reference points P, 2 = query points Q,
3 = instance shapes of the batched workload, 4 = request trace of the served
workload.  Workload recipes (sizes, distributions) are the synthetic stand-ins
for the astronomy catalogues of the paper's experiments (Section 4.1); none of
those catalogues' records is reproduced here.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BLOCK = 1 << 20
DEFAULT_SEED = 1512

STREAM_PARAMS = 0
STREAM_P = 1
STREAM_Q = 2
STREAM_BATCH = 3
STREAM_TRACE = 4


def _rng(seed: int, stream: int, block: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, block])))


def _blocks(n: int):
    nb = (n + BLOCK - 1) // BLOCK
    for b in range(nb):
        lo = b * BLOCK
        yield b, lo, min(n, lo + BLOCK)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def uniform(seed: int, stream: int, n: int, d: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n x d float32 points, i.i.d. uniform on [lo, hi)^d."""
    out = np.empty((n, d), dtype=np.float32)

    def fill(args):
        b, a, e = args
        g = _rng(seed, stream, b)
        out[a:e] = (lo + (hi - lo) * g.random((e - a, d))).astype(np.float32)

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill, _blocks(n)))
    return out


def mixture_params(seed: int, d: int, comps: int, mean_range=(0.0, 20.0), std_range=(0.1, 2.0)):
    """Means ~ U[mean_range]^d and diagonal stds ~ U[std_range]^d per component (stream 0)."""
    g = _rng(seed, STREAM_PARAMS, 0)
    means = g.uniform(mean_range[0], mean_range[1], size=(comps, d))
    stds = g.uniform(std_range[0], std_range[1], size=(comps, d))
    return means, stds


def mixture(seed: int, stream: int, n: int, d: int, comps: int, params=None) -> np.ndarray:
    """n x d float32 points from an equal-weight anisotropic Gaussian mixture."""
    means, stds = params if params is not None else mixture_params(seed, d, comps)
    out = np.empty((n, d), dtype=np.float32)

    def fill(args):
        b, a, e = args
        g = _rng(seed, stream, b)
        c = g.integers(0, comps, size=e - a)
        z = g.standard_normal((e - a, d))
        out[a:e] = (means[c] + stds[c] * z).astype(np.float32)

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill, _blocks(n)))
    return out


def lattice(seed: int, stream: int, n: int, d: int, side: int = 8) -> np.ndarray:
    """n x d float32 points with integer coordinates in {0..side-1}.

    Every float32 and float64 operation on such inputs is exact, so exact ties
    between distances are frequent and every result is exactly defined.
    """
    g = _rng(seed, stream, 0)
    return g.integers(0, side, size=(n, d)).astype(np.float32)


# ---------------------------------------------------------------------------
# Workload recipes

def small_uniform(seed: int = DEFAULT_SEED, n: int = 1 << 15, m: int = 1 << 12, d: int = 10):
    """Small plain case: P and Q i.i.d. uniform on [0,1]^d."""
    return uniform(seed, STREAM_P, n, d), uniform(seed, STREAM_Q, m, d)


def mixture_pq(seed: int = DEFAULT_SEED, n: int = 1 << 22, m: int = 1 << 22, d: int = 10, comps: int = 16):
    """P and Q from the same seeded mixture, on independent streams."""
    params = mixture_params(seed, d, comps)
    return (mixture(seed, STREAM_P, n, d, comps, params),
            mixture(seed, STREAM_Q, m, d, comps, params))


def batch_shapes(seed: int = DEFAULT_SEED, count: int = 1024, logn=(10, 18), logm=(8, 16),
                 dims=(3, 5, 10, 15), ks=(1, 5, 10, 32)):
    """Per-instance (n, m, d, k, h) of the batched workload.

    n = floor(2^U(logn)), m = floor(2^U(logm)), d and k uniform over the given
    sets, height h = floor(log2(n / 64)).
    """
    g = _rng(seed, STREAM_BATCH, 0)
    n = np.floor(2.0 ** g.uniform(logn[0], logn[1], size=count)).astype(np.int64)
    m = np.floor(2.0 ** g.uniform(logm[0], logm[1], size=count)).astype(np.int64)
    d = g.choice(np.asarray(dims), size=count)
    k = g.choice(np.asarray(ks), size=count)
    h = np.array([max(0, int(math.floor(math.log2(x / 64.0)))) for x in n], dtype=np.int64)
    return [dict(n=int(n[i]), m=int(m[i]), d=int(d[i]), k=int(k[i]), h=int(h[i])) for i in range(count)]


def batch_instance(seed: int, index: int, n: int, m: int, d: int, comps: int = 4):
    """Points of batched instance ``index``: a 4-component mixture of its own."""
    s = seed * 1_000_003 + index
    params = mixture_params(s, d, comps)
    return (mixture(s, STREAM_P, n, d, comps, params), mixture(s, STREAM_Q, m, d, comps, params))


def request_trace(seed: int, count: int, rate: float, logm=(0, 16), ks=(1, 10, 32), trees: int = 2):
    """Poisson arrival trace: (arrival_s, tree, m, k) per request."""
    g = _rng(seed, STREAM_TRACE, 0)
    gaps = g.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    tree = g.integers(0, trees, size=count)
    m = np.maximum(1, np.floor(2.0 ** g.uniform(logm[0], logm[1], size=count))).astype(np.int64)
    k = g.choice(np.asarray(ks), size=count)
    return [dict(t=float(t[i]), tree=int(tree[i]), m=int(m[i]), k=int(k[i])) for i in range(count)]
