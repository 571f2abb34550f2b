"""dagbound_best_allocation_static (the allocation-free surrogate search)
against dagbound_best_allocation with SURROGATE on the same inputs: two
calls in a row, the second on a smaller batch, bit for bit; and its
argument and state errors."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20826_amd as db

    db.load_library()
    return torch, db


def say(*a):
    print(*a, flush=True)


def test_static_search_matches_allocating_search(env):
    torch, db = env
    wl = W.WORKLOADS[4]
    M, K, seed, top_k = wl.num_cus, 1024, 9, 16
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    big = W.generate_workload(4, count=600, first=7000)
    small = W.generate_workload(4, count=150, first=9000)
    model = db.Model(4)
    batches, refs = [], []
    for dags in (big, small):
        b = db.create_batch(t(dags.node_off), t(dags.edge_off), t(dags.src), t(dags.dst), t(dags.wcet),
                            t(dags.par), M)
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
        idx = torch.empty(dags.num_dags, dtype=torch.int32, device=dev)
        bb = torch.empty(dags.num_dags, dtype=torch.int64, device=dev)
        say("allocating surrogate search,", dags.num_dags, "DAGs")
        db.best_allocation(b, idx, bb, search=db.SEARCH_SURROGATE, top_k=top_k, model=model)
        torch.cuda.synchronize()
        batches.append(b)
        refs.append((idx.cpu().numpy(), bb.cpu().numpy()))
    # two static calls in a row, the second on the smaller batch
    outs = []
    for b, dags in zip(batches, (big, small)):
        idx = torch.full((dags.num_dags,), -1, dtype=torch.int32, device=dev)
        bb = torch.full((dags.num_dags,), -1, dtype=torch.int64, device=dev)
        say("static surrogate search,", dags.num_dags, "DAGs")
        db.best_allocation_static(b, model, top_k, idx, bb)
        torch.cuda.synchronize()
        outs.append((idx.cpu().numpy(), bb.cpu().numpy()))
    for (ri, rb), (gi, gb) in zip(refs, outs):
        assert np.array_equal(ri, gi)
        assert np.array_equal(rb, gb)
        assert np.all(gb > 0)
    # and again on the large batch after the small one (the scratch keeps the
    # last call's lists; nothing may depend on them)
    idx = torch.empty(big.num_dags, dtype=torch.int32, device=dev)
    bb = torch.empty(big.num_dags, dtype=torch.int64, device=dev)
    db.best_allocation_static(batches[0], model, top_k, idx, bb)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), refs[0][0]) and np.array_equal(bb.cpu().numpy(), refs[0][1])
    for b in batches:
        b.close()
    model.close()


def test_static_search_errors(env):
    torch, db = env
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    dags = W.generate_workload(4, count=50, first=11000)
    b = db.create_batch(t(dags.node_off), t(dags.edge_off), t(dags.src), t(dags.dst), t(dags.wcet), t(dags.par),
                        256)
    idx = torch.empty(dags.num_dags, dtype=torch.int32, device=dev)
    bb = torch.empty(dags.num_dags, dtype=torch.int64, device=dev)
    model = db.Model(1)
    with pytest.raises(db.DagboundError) as e:  # no allocations yet
        db.best_allocation_static(b, model, 4, idx, bb)
    assert e.value.code == -7
    db.set_allocations(b, 64, db.ALLOC_SEEDED, None, 3)
    with pytest.raises(db.DagboundError) as e:  # workspace never sized for this batch
        db.best_allocation_static(b, model, 4, idx, bb)
    assert e.value.code == -7
    for bad_k in (0, 64, 256):
        with pytest.raises(db.DagboundError) as e:
            db.best_allocation_static(b, model, bad_k, idx, bb)
        assert e.value.code == -1
    b.close()
    # more list entries than the scratch holds: D x (top_k + 1) above 4 Mi
    many = W.generate_workload(1, count=20000)
    b2 = db.create_batch(many.node_off, many.edge_off, many.src, many.dst, many.wcet, many.par, 8)
    db.set_allocations(b2, 256, db.ALLOC_SEEDED, None, 3)
    i2 = torch.empty(many.num_dags, dtype=torch.int32, device=dev)
    o2 = torch.empty(many.num_dags, dtype=torch.int64, device=dev)
    with pytest.raises(db.DagboundError) as e:
        db.best_allocation_static(b2, model, 255, i2, o2)
    assert e.value.code == -1 and "static scratch" in e.value.message
    b2.close()
    model.close()
