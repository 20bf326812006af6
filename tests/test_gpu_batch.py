"""Batched form: every instance's result equals the exhaustive float32 oracle and the
single-instance path, in any mix and under any tuning."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import datagen
import oracle
import paper_1512_02831_amd as bkd

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def keys_of(idx, d2):
    return (d2.astype(np.float32).view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)


def mixed_instances(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = int(rng.choice([1, 2, 3, 5, 10, 15, 16, 20, 32]))
        n = int(rng.integers(64, 6000))
        m = int(rng.choice([0, 1, int(rng.integers(2, 2000))]))
        k = int(min(n, rng.choice([1, 5, 10, 32, 64])))
        h = int(rng.integers(0, min(12, int(np.log2(n))) + 1))
        P, Q = datagen.batch_instance(seed, i, n, m, d)
        out.append((P, Q, k, h))
    return out


def test_batch_mixed_shapes_match_oracle_and_single_path():
    say("case: batch of 40 mixed instances")
    inst = mixed_instances(7, 40)
    with bkd.batch_create(inst, flags=bkd.FLAG_SQUARED) as b:
        bkd.batch_run(b)
        res = bkd.batch_results(b)
        st = bkd.batch_stats(b)
    assert st["error"] == 0 and st["queries"] == sum(len(x[1]) for x in inst)
    for i, ((P, Q, k, h), (idx, d2)) in enumerate(zip(inst, res)):
        if len(Q) == 0:
            continue
        assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q, k)), i
        with bkd.build(P, h, flags=bkd.FLAG_SQUARED) as t:
            i2, e2 = bkd.query(t, Q, k)
        assert np.array_equal(i2, idx) and np.array_equal(e2, d2), i


def test_batch_device_pointers_match_host_pointers():
    """BKD_FLAG_DEVICE_PTRS: P, Q and the outputs on the GPU (torch tensors) give the host
    form's results, and the oracle's; a host pointer under the flag is refused."""
    import torch
    say("case: batch of 16 mixed instances from device pointers")
    inst = mixed_instances(23, 16)
    dev = [(torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda(), k, h) for P, Q, k, h in inst]
    with bkd.batch_create(dev, flags=bkd.FLAG_SQUARED | bkd.FLAG_DEVICE_PTRS) as b:
        bkd.batch_run(b)
        res = [(i.cpu().numpy(), d.cpu().numpy()) for i, d in bkd.batch_results(b)]
    with bkd.batch_create(inst, flags=bkd.FLAG_SQUARED) as b:
        bkd.batch_run(b)
        ref = bkd.batch_results(b)
    for i, ((P, Q, k, h), (idx, d2), (ri, rd)) in enumerate(zip(inst, res, ref)):
        assert np.array_equal(idx, ri) and np.array_equal(d2, rd), i
        if len(Q):
            assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q, k)), i
    # a host array where the flag promises device memory
    P, Q, k, h = inst[0]
    bad = [(dev[0][0], dev[0][1], k, h)]
    host_p = np.ascontiguousarray(P)
    inst_t = (bkd.Instance * 1)()
    oi = torch.zeros((len(Q), k), dtype=torch.int64, device="cuda")
    od = torch.zeros((len(Q), k), dtype=torch.float32, device="cuda")
    inst_t[0] = bkd.Instance(host_p.ctypes.data, len(P), bad[0][1].data_ptr(), len(Q), P.shape[1], k, h,
                             oi.data_ptr(), od.data_ptr())
    import ctypes
    hnd = ctypes.c_void_p()
    rc = bkd.lib().bkd_batch_create(ctypes.cast(inst_t, ctypes.c_void_p), 1, 0, bkd.FLAG_DEVICE_PTRS,
                                    ctypes.byref(hnd))
    assert rc == bkd.EINVAL and "not device memory" in bkd.lib().bkd_last_error().decode()


def test_batch_same_alone_and_in_mix_and_under_tunings():
    say("case: alone vs mix, tunings")
    inst = mixed_instances(11, 24)
    with bkd.batch_create(inst) as b:
        bkd.batch_run(b, bkd.Tuning(8, 4, 1))
        ref = [(i.copy(), d.copy()) for i, d in bkd.batch_results(b)]
        for lpt, gpc, solo in ((1, 1, 100000), (3, 2, 64), (32, 3, 2048), (256, 4, 0)):
            bkd.batch_run(b, bkd.Tuning(lpt, gpc, solo))
            for (i, d), (ri, rd) in zip(bkd.batch_results(b), ref):
                assert np.array_equal(i, ri) and np.array_equal(d, rd)
        best, ms = bkd.batch_autotune(b)
        assert 1 <= best.leaves_per_task <= 256 and ms > 0
        bkd.batch_run(b)
        for (i, d), (ri, rd) in zip(bkd.batch_results(b), ref):
            assert np.array_equal(i, ri) and np.array_equal(d, rd)
    for j in (0, 5, 17):
        with bkd.batch_create([inst[j]]) as b:
            bkd.batch_run(b)
            (i, d), = bkd.batch_results(b)
        assert np.array_equal(i, ref[j][0]) and np.array_equal(d, ref[j][1])


@pytest.mark.parametrize("lpt", [1, 8, 64])
def test_batch_round_pieces_match_oracle(lpt):
    # solo_max 1 keeps every instance in rounds to the end, so every leaf scan runs as pieces of
    # at most 32 queries: thousands of queries on two leaves (many pieces per leaf), 4096 leaves
    # (piece codes with the top bit set), and d = 15, k = 32
    say(f"case: batched rounds as pieces, {lpt} pieces per task")
    shapes = [(300, 3, 1, 5000, 5), (65536, 5, 12, 8000, 10), (4000, 15, 5, 3000, 32), (5000, 10, 6, 1, 1)]
    inst = []
    for i, (n, d, h, m, k) in enumerate(shapes):
        P, Q = datagen.batch_instance(41, i, n, m, d)
        inst.append((P, Q, k, h))
    with bkd.batch_create(inst, flags=bkd.FLAG_SQUARED) as b:
        bkd.batch_run(b, bkd.Tuning(lpt, 4, 1))
        res = bkd.batch_results(b)
        st = bkd.batch_stats(b)
    assert st["error"] == 0 and st["rounds"] > 0
    for i, ((P, Q, k, h), (idx, d2)) in enumerate(zip(inst, res)):
        assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q, k)), i


def test_batch_rejects_bad_instances():
    P, Q = datagen.batch_instance(1, 0, 100, 10, 3)
    with pytest.raises(bkd.BkdError) as e:
        bkd.batch_create([(P, Q, 5, 2), (P, Q, 101, 2)])
    assert e.value.code == bkd.EINVAL and "instance 1" in str(e.value)
    with pytest.raises(bkd.BkdError) as e:
        bkd.batch_create([(P, Q, 5, 13)])
    assert e.value.code == bkd.EINVAL


def test_batched_config_sampled_parity():
    # 1024 instances: n = floor(2^U(10,18)), m = floor(2^U(8,16)), d in {3,5,10,15}, k in {1,5,10,32},
    # 4-component mixtures, height floor(log2(n/64)); sampled instances checked against the oracle.
    say("case: batched 1024 instances (sampled)")
    shapes = datagen.batch_shapes()
    inst = []
    for i, s in enumerate(shapes):
        P, Q = datagen.batch_instance(datagen.DEFAULT_SEED, i, s["n"], s["m"], s["d"])
        inst.append((P, Q, s["k"], s["h"]))
    with bkd.batch_create(inst, flags=bkd.FLAG_SQUARED) as b:
        bkd.batch_run(b)
        res = bkd.batch_results(b)
        st = bkd.batch_stats(b)
    say("  stats", st)
    assert st["error"] == 0
    rng = np.random.default_rng(3)
    for i in rng.choice(len(inst), 24, replace=False):
        P, Q, k, h = inst[i]
        rows = rng.choice(len(Q), min(len(Q), 64), replace=False)
        idx, d2 = res[i]
        assert np.array_equal(keys_of(idx[rows], d2[rows]), oracle.brute_f32c(P, Q[rows], k)), i


def test_batch_tuning_cache_roundtrip(tmp_path):
    """The tuning cache keeps one line per batch signature: a new batch of the same shapes
    loads the tuned schedule, another batch finds none, and the results do not depend on it."""
    say("case: tuning cache")
    inst = mixed_instances(29, 12)
    path = str(tmp_path / "tuning.txt")
    with bkd.batch_create(inst) as b:
        best, _ = bkd.batch_autotune(b)
        bkd.batch_tuning_save(b, path)
        bkd.batch_run(b)
        want = [(i.copy(), d.copy()) for i, d in bkd.batch_results(b)]
    with bkd.batch_create(inst) as b2:
        got = bkd.batch_tuning_load(b2, path)
        assert (got.leaves_per_task, got.groups_per_cu, got.solo_max) == \
            (best.leaves_per_task, best.groups_per_cu, best.solo_max)
        bkd.batch_run(b2)
        for (i1, d1), (i2, d2) in zip(want, bkd.batch_results(b2)):
            assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
    with bkd.batch_create(mixed_instances(31, 5)) as b3:
        with pytest.raises(bkd.BkdError) as e:
            bkd.batch_tuning_load(b3, path)
        assert e.value.code == bkd.ENOTFOUND
