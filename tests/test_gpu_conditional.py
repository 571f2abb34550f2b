"""Conditional DAGs on the GPU (dagbound_eval_conditional) against the CPU
oracle's realization bounds (oracle.cond_bound_max): the hand-derived cases,
random conditional structures on workloads of every size class up to 512
nodes with explicit and seeded candidates, the all-unconditional case
against dagbound_eval_bounds, and the error paths."""
import numpy as np
import pytest

import oracle
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


def random_structure(batch, rng, max_conds=3, max_branches=3, frac=0.5):
    """Per node a conditional id (or -1) and a branch, a few conditionals per DAG."""
    T = int(batch.node_off[-1])
    cond = np.full(T, -1, np.int32)
    br = np.zeros(T, np.int32)
    for d in range(batch.num_dags):
        n0, n1 = int(batch.node_off[d]), int(batch.node_off[d + 1])
        q = int(rng.integers(1, max_conds + 1))
        nb = rng.integers(2, max_branches + 1, q)
        pick = rng.random(n1 - n0) < frac
        cond[n0:n1] = np.where(pick, rng.integers(0, q, n1 - n0), -1)
        for v in range(n0, n1):
            if cond[v] >= 0:
                br[v] = rng.integers(0, nb[cond[v]])
    return cond, br


def check(env, batch, M, K, alloc, seeded_seed, cond, br, label):
    torch, db = env
    D = batch.num_dags
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
    if seeded_seed is None:
        db.set_allocations(b, K, db.ALLOC_EXPLICIT, alloc)
    else:
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seeded_seed)
        alloc = W.alloc_bytes(batch, M, K, seed=seeded_seed)
    got = np.zeros(D * K, np.int64)
    worst = np.zeros(D * K, np.int32)
    say(label, D, "DAGs x", K)
    db.eval_conditional(b, cond, br, got, worst)
    b.close()
    got, worst = got.reshape(D, K), worst.reshape(D, K)
    for d in range(D):
        n, s, t, w, p = batch.dag(d)
        n0 = int(batch.node_off[d])
        rows = alloc[K * n0: K * n0 + K * n].reshape(K, n)
        for c in range(K):
            want = oracle.cond_bound_max(n, s, t, w, p, M, rows[c] if c else None, cond[n0:n0 + n],
                                         br[n0:n0 + n])
            assert (got[d, c], worst[d, c]) == want, (label, d, c)


def test_conditional_hand_cases(env):
    src, dst = np.array([0, 0, 1, 2], np.int32), np.array([1, 2, 3, 3], np.int32)
    cases = [
        # (loads, p, M, candidate 1 bytes, expected (bound, worst) for c = 0 and c = 1)
        ([1, 8, 3, 1], [1, 4, 1, 1], 4, [0, 2, 0, 0], [(5, 1), (6, 0)]),
        ([1, 6, 6, 1], [1, 2, 2, 1], 3, [0, 2, 2, 0], [None, (5, 0)]),
    ]
    torch, db = env
    for w, p, M, r1, want in cases:
        batch = W.from_dags([(4, src, dst, np.array(w, np.int64), np.array(p, np.int32))])
        alloc = np.concatenate([np.zeros(4, np.uint8), np.array(r1, np.uint8)])
        b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
        db.set_allocations(b, 2, db.ALLOC_EXPLICIT, alloc)
        got = np.zeros(2, np.int64)
        worst = np.zeros(2, np.int32)
        db.eval_conditional(b, np.array([-1, 0, 0, -1], np.int32), np.array([0, 0, 1, 0], np.int32), got, worst)
        b.close()
        for c in range(2):
            if want[c] is not None:
                assert (got[c], worst[c]) == want[c], (w, c)
            r = alloc[4 * c: 4 * c + 4] if c else None
            assert (got[c], worst[c]) == oracle.cond_bound_max(4, src, dst, np.array(w), np.array(p), M, r,
                                                                [-1, 0, 0, -1], [0, 0, 1, 0])


@pytest.mark.parametrize("wk,count,K", [(1, 40, 16), (2, 12, 64), (3, 6, 8)])
def test_conditional_matches_oracle_explicit(env, wk, count, K):
    rng = np.random.default_rng(100 + wk)
    batch = W.generate_workload(wk, count=count, first=500)
    if wk == 3:  # keep DAGs of up to 512 nodes (every size class of the per-candidate kernels)
        keep = [d for d in range(batch.num_dags) if batch.dag(d)[0] <= 512]
        batch = batch.subset(keep)
    M = W.WORKLOADS[wk].num_cus
    alloc = W.alloc_bytes(batch, M, K, seed=77)
    cond, br = random_structure(batch, rng)
    check(env, batch, M, K, alloc, None, cond, br, f"conditional explicit wk{wk}")


@pytest.mark.parametrize("wk,count,K", [(1, 30, 8), (4, 4, 4)])
def test_conditional_matches_oracle_seeded(env, wk, count, K):
    rng = np.random.default_rng(200 + wk)
    batch = W.generate_workload(wk, count=count, first=900)
    M = W.WORKLOADS[wk].num_cus
    cond, br = random_structure(batch, rng, max_conds=2, max_branches=4)
    check(env, batch, M, K, None, 31, cond, br, f"conditional seeded wk{wk}")


def test_every_node_unconditional_equals_eval_bounds(env):
    torch, db = env
    batch = W.generate_workload(3, count=300, first=1200)
    keep = [d for d in range(batch.num_dags) if batch.dag(d)[0] <= 512]
    batch = batch.subset(keep)
    M, K = 256, 64
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M)
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, 5)
    T = int(batch.node_off[-1])
    cond = torch.full((T,), -1, dtype=torch.int32, device=dev)
    br = torch.zeros(T, dtype=torch.int32, device=dev)
    got = torch.empty(batch.num_dags * K, dtype=torch.int64, device=dev)
    worst = torch.empty(batch.num_dags * K, dtype=torch.int32, device=dev)
    say("conditional with no conditionals,", batch.num_dags, "DAGs")
    db.eval_conditional(b, cond, br, got, worst)
    want = torch.empty_like(got)
    db.eval_bounds(b, want)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert int(worst.abs().sum()) == 0
    b.close()


def test_conditional_errors(env):
    torch, db = env
    batch = W.generate_workload(1, count=3)
    T = int(batch.node_off[-1])
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 8)
    out = np.zeros(3 * 4, np.int64)
    cond, br = np.full(T, -1, np.int32), np.zeros(T, np.int32)
    with pytest.raises(db.DagboundError) as e:
        db.eval_conditional(b, cond, br, out)
    assert e.value.code == db.E_STATE
    db.set_allocations(b, 4, db.ALLOC_SEEDED, None, 1)
    bad = cond.copy()
    bad[0] = -2
    with pytest.raises(db.DagboundError) as e:
        db.eval_conditional(b, bad, br, out)
    assert e.value.code == db.E_RANGE
    many = np.arange(T, dtype=np.int32) % 13  # 13 conditionals of 2 branches: 8,192 realizations
    with pytest.raises(db.DagboundError) as e:
        db.eval_conditional(b, many, np.ones(T, np.int32), out)
    assert e.value.code == db.E_RANGE
    db.set_para_launch(b, db.PARA_TEMPORAL)
    with pytest.raises(db.DagboundError) as e:
        db.eval_conditional(b, cond, br, out)
    assert e.value.code == db.E_UNSUPPORTED
    b.close()
    big = W.generate_workload(5, count=1)
    Tb = int(big.node_off[-1])
    b = db.create_batch(big.node_off, big.edge_off, big.src, big.dst, big.wcet, big.par, 256)
    db.set_allocations(b, 2, db.ALLOC_SEEDED, None, 1)
    with pytest.raises(db.DagboundError) as e:
        db.eval_conditional(b, np.full(Tb, -1, np.int32), np.zeros(Tb, np.int32), np.zeros(2, np.int64))
    assert e.value.code == db.E_UNSUPPORTED
    b.close()
