"""The schedule run on the GPU as a HIP graph (dagbound_run_schedule), the
counterpart of the paper's case study: every part of the schedule a busy
kernel of m workgroups for C ticks.  With one barrier per slot boundary the
run can take no less than the sum of the slots' longest parts (the critical-
path term) and, launch overheads aside, no more than the bound."""
import json
import os

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import GOLDEN, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

TICK_NS = 50_000
# launch overhead allowance: per slot boundary (a kernel node and an empty
# node) and per run
SLOT_OVERHEAD_NS = 150_000
RUN_OVERHEAD_NS = 1_000_000


def run(db, batch, M, d, c, barriers, reps=10, seed=None):
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
    K = max(c + 1, 2)
    if seed is None:
        db.set_allocations(b, K, db.ALLOC_EXPLICIT, np.zeros(K * int(batch.node_off[-1]), np.uint8))
    else:
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    recs, _ = db.get_schedule(b, d, c)
    slots = int((recs[:, 0] == 1).sum())
    out, terms = db.run_schedule(b, d, c, TICK_NS, barriers=barriers, reps=reps)
    b.close()
    return out, terms, slots


def check_barriers(out, terms, slots):
    bound, cp, intf, parts = terms
    assert bound == cp + intf and parts >= 1
    lo = cp * TICK_NS * 0.97
    hi = bound * TICK_NS + slots * SLOT_OVERHEAD_NS + RUN_OVERHEAD_NS
    assert out.min() >= lo, (out.min(), lo)
    assert np.median(out) <= hi, (np.median(out), hi)


def test_run_worked_example(torch_dev):
    import paper_2602_20826_amd as db

    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    e = np.asarray(ex["edges"], np.int32).reshape(-1, 2)
    batch = W.from_dags([(ex["n"], e[:, 0], e[:, 1], ex["wcet"], ex["par"])])
    say("run schedule: worked example, barriers")
    out, terms, slots = run(db, batch, ex["M"], 0, 0, True)
    assert terms[:3] == (5, 5, 0) and slots == 4
    check_barriers(out, terms, slots)
    say("run schedule: worked example, edges only", np.median(out))
    out2, terms2, _ = run(db, batch, ex["M"], 0, 0, False)
    assert terms2 == terms
    assert out2.min() > 0


@pytest.mark.parametrize("M,seeded", [(8, False), (32, True), (128, False)])
def test_run_generated(torch_dev, M, seeded):
    import paper_2602_20826_amd as db

    batch = W.paper_style(6, 8, 20)
    for d in range(batch.num_dags):
        for c in ([0, 1] if seeded else [0]):
            say("run schedule: evaluation-style DAG", d, "M", M, "candidate", c)
            out, terms, slots = run(db, batch, M, d, c, True, reps=5, seed=3 if seeded else None)
            check_barriers(out, terms, slots)
            out2, _, _ = run(db, batch, M, d, c, False, reps=3, seed=3 if seeded else None)
            assert out2.min() > 0


def test_run_errors(torch_dev):
    import paper_2602_20826_amd as db

    batch = W.paper_style(2, 4, 5)
    say("run schedule: errors")
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 8)
    with pytest.raises(db.DagboundError) as e:
        db.run_schedule(b, 0, 0, TICK_NS)
    assert e.value.code == -7  # before set_allocations
    db.set_allocations(b, 2, db.ALLOC_SEEDED, None, 1)
    for kw in [dict(d=2, c=0, tick_ns=TICK_NS), dict(d=0, c=2, tick_ns=TICK_NS), dict(d=0, c=0, tick_ns=10),
               dict(d=0, c=0, tick_ns=TICK_NS, reps=0)]:
        with pytest.raises(db.DagboundError) as e:
            db.run_schedule(b, **kw)
        assert e.value.code == -1, kw
    b.close()
    # more compute units than the device has
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 4096)
    db.set_allocations(b, 2, db.ALLOC_SEEDED, None, 1)
    with pytest.raises(db.DagboundError) as e:
        db.run_schedule(b, 0, 0, TICK_NS)
    assert e.value.code == -1
    b.close()
