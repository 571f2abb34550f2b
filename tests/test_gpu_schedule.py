"""GPU schedule dump (dagbound_get_schedule) against the oracle's traced
schedule: every part (member, parallel node launched whole, segment) with
its m, C and load, every slot's members, maxC, sum m, A, R_j and v_R, and
the extra dependencies of Section 4.1, for the paper's cases, small and
large generated DAGs, the paper's rule and explicit or seeded candidates.
Expected values come from `oracle` only."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import GOLDEN, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def gpu_slots(records):
    """Group PART and EDGE records by slot, in the oracle's structure."""
    slots, parts, edges = [], [], {}
    for r in records.tolist():
        if r[0] == 2:
            parts.append(tuple(r[1:8]))
        elif r[0] == 1:
            slots.append((tuple(r[1:8]), parts))
            parts = []
        elif r[0] == 3:
            edges.setdefault(r[1], []).append(tuple(r[1:6]))
        else:
            raise AssertionError(f"bad record tag {r[0]}")
    assert not parts, "parts after the last slot"
    return slots, edges


def oracle_slots(sched):
    slots = [((s.j, s.nP, s.maxC, s.sum_m, s.A, s.R, s.vR),
              [(p.slot, p.node, p.part, p.kind, p.m, p.C, p.load) for p in s.parts]) for s in sched.slots]
    edges = {}
    for e in sched.edges:
        edges.setdefault(e[0], []).append(tuple(e))
    return slots, edges


def check_dag(db, b, batch, d, M, K, alloc, cands):
    n, s, t, w, p = batch.dag(d)
    n0 = int(batch.node_off[d])
    for c in cands:
        r = alloc[K * n0 + c * n: K * n0 + (c + 1) * n] if c > 0 else None
        want = oracle.bound(n, s, t, w, p, M, r, trace=True)
        rec, terms = db.get_schedule(b, d, c, cap=64)
        got_slots, got_edges = gpu_slots(rec)
        want_slots, want_edges = oracle_slots(want)
        assert terms == (want.bound, want.cp, want.intf), (d, c)
        assert len(got_slots) == len(want_slots), (d, c)
        for g, x in zip(got_slots, want_slots):
            assert g == x, (d, c, g, x)
        assert sorted(got_edges) == sorted(want_edges), (d, c)
        for j in want_edges:
            assert sorted(got_edges[j]) == sorted(want_edges[j]), (d, c, j)


def run_batch(torch_dev, batch, M, K, alloc, cands, seed=None, dags=None):
    import paper_2602_20826_amd as db

    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
    if seed is None:
        db.set_allocations(b, K, db.ALLOC_EXPLICIT, alloc)
    else:
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    for d in (range(batch.num_dags) if dags is None else dags):
        check_dag(db, b, batch, d, M, K, alloc, cands)
    b.close()


def test_schedule_paper_cases(torch_dev):
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    cases = [ex] + json.load(open(os.path.join(GOLDEN, "hand_cases.json")))["cases"]
    rng = np.random.default_rng(3)
    for cs in cases:
        e = np.asarray(cs["edges"], np.int32).reshape(-1, 2)
        batch = W.from_dags([(cs["n"], e[:, 0], e[:, 1], cs["wcet"], cs["par"])])
        n, M, K = cs["n"], cs["M"], 3
        alloc = np.zeros(K * n, np.uint8)
        alloc[n:2 * n] = np.asarray(cs.get("r", [0] * n), np.uint8)
        alloc[2 * n:] = W.random_alloc(rng, np.asarray(cs["par"]), M, 0.3)
        say("schedule dump:", cs["name"][:60])
        run_batch(torch_dev, batch, M, K, alloc, [0, 1, 2])


@pytest.mark.parametrize("wk,count,M", [(1, 40, 8), (2, 30, 256), (3, 12, 256)])
def test_schedule_generated(torch_dev, wk, count, M):
    batch = W.generate_workload(wk, count=count, first=7)
    K = 8
    alloc = W.alloc_bytes(batch, M, K, seed=13)
    say("schedule dump: workload", wk, count, "DAGs, explicit and seeded")
    run_batch(torch_dev, batch, M, K, alloc, [0, 1, 5])
    run_batch(torch_dev, batch, M, K, alloc, [0, 3, 7], seed=13)


def test_schedule_large_dags(torch_dev):
    from test_gpu_large import custom_large, large_workload

    batch = W.from_dags(large_workload(2, first=70, max_n=1500) + custom_large(4)[:3])
    M, K = 256, 4
    alloc = W.alloc_bytes(batch, M, K, seed=2)
    say("schedule dump: large DAGs", np.diff(batch.node_off).tolist())
    run_batch(torch_dev, batch, M, K, alloc, [0, 2], seed=2)


def test_schedule_errors(torch_dev):
    import paper_2602_20826_amd as db

    batch = W.generate_workload(1, count=3)
    say("schedule dump errors")
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 8)
    with pytest.raises(db.DagboundError) as e:
        db.get_schedule(b, 0, 0)
    assert e.value.code == -7  # before set_allocations
    db.set_allocations(b, 4, db.ALLOC_SEEDED, None, 1)
    for d, c in [(-1, 0), (3, 0), (0, 4), (0, -1)]:
        with pytest.raises(db.DagboundError) as e:
            db.get_schedule(b, d, c)
        assert e.value.code == -1, (d, c)
    # a buffer too small for the schedule returns the count; the binding grows it
    rec, terms = db.get_schedule(b, 1, 2, cap=1)
    assert len(rec) > 1 and rec[-1][0] in (1, 3)
    b.close()
