"""The temporal reading of the launching loop (dagbound_set_para_launch
PARA_TEMPORAL: spare SMs kept per node, launched nodes chained within the
slot's time) on the GPU against the oracle's, bit-exact: the hand-derived
case, every workload shape and size class, explicit and seeded candidates,
the schedule dump record for record, and switching the reading on a batch.
Expected values come from `oracle` only."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import GOLDEN, check_against_oracle, gpu_eval, mixed_size_batch, say, torch_dev  # noqa: F401
from test_gpu_schedule import gpu_slots, oracle_slots

pytestmark = pytest.mark.gpu
T = oracle.TEMPORAL


def test_temporal_hand_case(torch_dev):
    case = json.load(open(os.path.join(GOLDEN, "temporal_cases.json")))["cases"][0]
    e = np.asarray(case["edges"], np.int32).reshape(-1, 2)
    batch = W.from_dags([(case["n"], e[:, 0], e[:, 1], case["wcet"], case["par"])])
    K = 2
    alloc = np.zeros(K * case["n"], np.uint8)
    alloc[case["n"]:] = case["r"]
    say("temporal: hand case")
    for mode, key in ((oracle.SPATIAL, "spatial"), (T, "temporal")):
        got = gpu_eval(torch_dev, batch, case["M"], K, alloc, para_mode=mode)
        assert [int(got[0][0, 1]), int(got[1][0, 1]), int(got[2][0, 1])] == case["expect"][key]


@pytest.mark.parametrize("k,count,K", [(1, 1000, 16), (2, 2000, 64), (3, 300, 70)])
def test_temporal_workloads(torch_dev, k, count, K):
    wl = W.WORKLOADS[k]
    batch = W.generate_workload(k, count=count, first=11)
    alloc = W.alloc_bytes(batch, wl.num_cus, K, seed=21)
    say("temporal: workload", k, count, "DAGs x", K)
    got = gpu_eval(torch_dev, batch, wl.num_cus, K, alloc, para_mode=T)
    check_against_oracle(batch, wl.num_cus, K, alloc, got, para_mode=T)


@pytest.mark.parametrize("seeded,tuning", [(0, None), (1, None), (0, {"node_lanes": 256}),
                                           (1, {"persistent": 1, "class_streams": 0})])
def test_temporal_mixed_classes(torch_dev, seeded, tuning):
    # node_lanes 256: DAGs of 257-512 nodes on the lane-per-node kernel
    batch = mixed_size_batch()
    K, M = 70, 256
    alloc = W.alloc_bytes(batch, M, K, seed=5)
    say("temporal: mixed size classes, seeded", seeded, "tuning", tuning)
    got = gpu_eval(torch_dev, batch, M, K, alloc, seed=5 if seeded else None, para_mode=T, tuning=tuning)
    check_against_oracle(batch, M, K, alloc, got, para_mode=T)


@pytest.mark.parametrize("M", [256, 8])
def test_temporal_large_dags(torch_dev, M):
    from test_gpu_large import custom_large, large_workload

    batch = W.from_dags(large_workload(3, first=40) + custom_large(7))
    K = 8
    alloc = W.alloc_bytes(batch, M, K, seed=9)
    say("temporal: large DAGs", np.diff(batch.node_off).tolist(), "M", M)
    got = gpu_eval(torch_dev, batch, M, K, alloc, seed=9, para_mode=T)
    check_against_oracle(batch, M, K, alloc, got, para_mode=T)


def test_temporal_small_loads_and_large_loads(torch_dev):
    # loads on both sides of 2^20 (the float paths and the 64-bit ones)
    rng = np.random.default_rng(4)
    base = W.generate_workload(2, count=200, first=5)
    dags = []
    for d in range(base.num_dags):
        n, s, t, w, p = base.dag(d)
        scale = 1 if d % 2 else 5000
        dags.append((n, s, t, np.minimum(w * scale, 2**31 - 1), p))
    batch = W.from_dags(dags)
    for M in (256, 5):
        alloc = W.alloc_bytes(batch, M, 64, seed=int(rng.integers(1, 100)))
        say("temporal: loads up to 5e6, M", M)
        got = gpu_eval(torch_dev, batch, M, 64, alloc, para_mode=T)
        check_against_oracle(batch, M, 64, alloc, got, para_mode=T)


def test_temporal_schedule_dump(torch_dev):
    import paper_2602_20826_amd as db
    from test_gpu_large import custom_large

    batch = W.from_dags([W.generate_workload(2, count=20, first=3).dag(d) for d in range(20)] + custom_large(2)[:2])
    M, K = 64, 4
    alloc = W.alloc_bytes(batch, M, K, seed=2)
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
    db.set_allocations(b, K, db.ALLOC_EXPLICIT, alloc)
    db.set_para_launch(b, db.PARA_TEMPORAL)
    say("temporal: schedule dump")
    for d in range(batch.num_dags):
        n, s, t, w, p = batch.dag(d)
        n0 = int(batch.node_off[d])
        for c in (0, 3):
            r = alloc[K * n0 + c * n: K * n0 + (c + 1) * n] if c > 0 else None
            want = oracle.bound(n, s, t, w, p, M, r, trace=True, para_mode=T)
            rec, terms = db.get_schedule(b, d, c)
            gs, ge = gpu_slots(rec)
            ws, we = oracle_slots(want)
            assert terms == (want.bound, want.cp, want.intf)
            assert gs == ws, (d, c)
            assert {j: sorted(v) for j, v in ge.items()} == {j: sorted(v) for j, v in we.items()}, (d, c)
    b.close()


def test_switching_reading(torch_dev):
    import paper_2602_20826_amd as db

    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2, count=300, first=9)
    K = 32
    alloc = W.alloc_bytes(batch, wl.num_cus, K, seed=3)
    want_s = oracle.bounds_batch(batch, wl.num_cus, K, alloc, threads=8)[0]
    want_t = oracle.bounds_batch(batch, wl.num_cus, K, alloc, threads=8, para_mode=T)[0]
    say("temporal: switching the reading on one batch, with the library graph")
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, wl.num_cus)
    db.set_allocations(b, K, db.ALLOC_EXPLICIT, alloc)
    out = np.empty(batch.num_dags * K, np.int64)
    bi, bb = np.empty(batch.num_dags, np.int32), np.empty(batch.num_dags, np.int64)
    for mode, want in ((db.PARA_TEMPORAL, want_t), (db.PARA_SPATIAL, want_s), (db.PARA_TEMPORAL, want_t)):
        db.set_para_launch(b, mode)
        db.eval_bounds(b, out)
        assert np.array_equal(out.reshape(-1, K), want)
        db.best_allocation(b, bi, bb)
        assert np.array_equal(bb, want.min(1))
    with pytest.raises(db.DagboundError):
        db.set_para_launch(b, 2)
    b.close()


def test_temporal_full_size_sampled(torch_dev):
    # the whole batched-layered workload (100,000 DAGs x 64 explicit
    # candidates) in the temporal reading, a seeded sample of DAGs (and the
    # first and last) on the oracle
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=wl.seed)
    say("temporal: batched-layered full size", batch.num_dags, "DAGs x", wl.K)
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc, terms=False, para_mode=T)
    rng = np.random.default_rng(29)
    sample = np.unique(np.r_[0, rng.integers(0, batch.num_dags, 1500), batch.num_dags - 1])
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got, dags=sample, para_mode=T)
