"""Pins of two readings against the sizes the paper states (tests/golden/paper_sizes.json).

* "Height": a tree of height h has h levels of splitting nodes, 2^h - 1 split
  values and 2^h leaves (h = 0 is one leaf, i.e. brute force).  The footnote
  on the top tree in Section 3.1 fixes this: at h = 20 the top tree needs less
  than ten megabytes and buffers of 128 indices per leaf less than a gigabyte.
  2^20 leaves fit both; one more level (2^21 leaves, the reading that counts
  the leaf level as a level of its own) breaks the buffer bound.
* Storage precision: one billion points in R^15 take about 60 gigabytes
  (Section 3.1), i.e. four bytes per coordinate.
* Schedule defaults: B = 2^(24 - h) and M = 10 B (Section 4.1, footnote on
  the parameters), as the library's bkd_default_options returns them.

The oracle's build supplies the node and leaf counts; nothing here runs on a GPU.
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle
import paper_1512_02831_amd as bkd

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_sizes.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def oracle_counts(h: int):
    """(split values, leaves) of the oracle's canonical tree of height h."""
    P = np.random.default_rng(h).random((max(1 << h, 4) * 3, 3), dtype=np.float32)
    t = oracle.build_tree(P, h)
    return len(t.split), len(t.leaf_off) - 1


def test_height_reading_counts_internal_levels():
    for h in range(0, 9):
        splits, leaves = oracle_counts(h)
        assert (splits, leaves) == ((1 << h) - 1, 1 << h)


def test_top_tree_and_buffer_sizes_of_the_footnote():
    g = golden()
    h = g["top_tree"]["height"]
    splits = (1 << h) - 1
    assert 4 * splits < g["top_tree"]["max_bytes"]                     # float32 split values
    b = g["buffers"]
    leaves = 1 << b["height"]
    assert leaves * b["buffer_size"] * 4 < b["max_bytes"]             # int32 query indices per leaf
    # the alternative reading (one more level: 2^(h+1) leaves) contradicts the buffer bound
    assert (2 * leaves) * b["buffer_size"] * 4 > b["max_bytes"]


def test_storage_precision_is_float32():
    g = golden()["leaf_structure"]
    n, d, approx = g["n"], g["d"], g["approx_bytes"]
    assert abs(n * d * 4 - approx) <= 0.05 * approx
    assert abs(n * d * 8 - approx) > 0.5 * approx                     # float64 would be twice as large


def test_library_defaults_follow_the_parameter_footnote():
    for case in golden()["parameters"]["cases"]:
        o = bkd.default_options(case["h"])
        assert (o.buffer_size, o.fetch_size) == (case["B"], case["M"])
        assert case["B"] == 1 << (24 - case["h"]) and case["M"] == 10 * case["B"]
