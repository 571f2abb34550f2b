"""GPU parity for DAGs above 512 nodes (the large-DAG preprocessing and the
one-wavefront-per-(DAG, candidate) evaluation) against the CPU oracle,
element by element, bit-exact int64.

Inputs come from the seeded generator in `workloads` (the large-compiler
workload and hand-built shapes); expected values come from `oracle` only.
Every test prints the case it runs before touching the GPU.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import check_against_oracle, gpu_eval, mixed_size_batch, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def chain_with_skips(rng, n, skip=7, p=0.5):
    src, dst = [], []
    for i in range(n - 1):
        src.append(i); dst.append(i + 1)
        if i + skip < n and rng.random() < p:
            src.append(i); dst.append(i + skip)
    perm = rng.permutation(n).astype(np.int32)
    return (n, perm[src], perm[dst], rng.integers(1, 10**4, n), rng.integers(1, 128, n))


def wide(rng, n):
    """n independent nodes: every node a source, one residual block."""
    return (n, np.zeros(0, np.int32), np.zeros(0, np.int32), rng.integers(1, 500, n), rng.integers(1, 300, n))


def bipartite(rng, n):
    """n - 1 sources feeding one sink (a join node of in-degree n - 1)."""
    perm = rng.permutation(n).astype(np.int32)
    return (n, perm[:-1], np.full(n - 1, perm[-1], np.int32), rng.integers(1, 2000, n), rng.integers(1, 64, n))


def er(rng, n, p):
    order = rng.permutation(n)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return (n, order[iu[keep]].astype(np.int32), order[ju[keep]].astype(np.int32),
            rng.integers(1, 10**5, n), rng.integers(1, 64, n))


def layered(rng, n, width, p):
    """Layers of 1..width nodes, edges between adjacent layers with prob p
    (every node keeps one predecessor in the previous layer)."""
    layers, v = [], 0
    while v < n:
        w = min(int(rng.integers(1, width + 1)), n - v)
        layers.append(list(range(v, v + w)))
        v += w
    src, dst = [], []
    for a, b in zip(layers, layers[1:]):
        for y in b:
            ps = [x for x in a if rng.random() < p] or [a[int(rng.integers(len(a)))]]
            src += ps
            dst += [y] * len(ps)
    perm = rng.permutation(n).astype(np.int32)
    return (n, perm[np.asarray(src, np.int64)], perm[np.asarray(dst, np.int64)], rng.integers(1, 3000, n),
            rng.integers(1, 128, n))


def large_workload(count, first, max_n=None):
    """DAGs of the large-compiler workload (optionally only those up to max_n nodes)."""
    full = W.generate_workload(5, count=count * (4 if max_n else 1), first=first)
    keep = [d for d in range(full.num_dags) if max_n is None or full.dag(d)[0] <= max_n][:count]
    return [full.dag(d) for d in keep]


def custom_large(seed):
    rng = np.random.default_rng(seed)
    return [chain_with_skips(rng, 900), wide(rng, 700), bipartite(rng, 601), er(rng, 1000, 0.01),
            layered(rng, 1500, 48, 0.3)]


def test_large_division_tables(torch_dev):
    import paper_2602_20826_amd as db

    dags = large_workload(3, first=0) + custom_large(1)
    batch = W.from_dags(dags)
    for M in (256, 8):
        say("large division tables:", batch.num_dags, "DAGs, sizes", np.diff(batch.node_off).tolist(), "M", M)
        b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
        for d in range(batch.num_dags):
            n, s, t, w, p = batch.dag(d)
            want = oracle.division(n, s, t, w, p, M)
            wanc, gof, order, ng = db.get_division(b, d)
            assert wanc.tolist() == want.wanc.tolist(), d
            assert ng == len(want.groups), d
            assert order.tolist() == [v for g in want.groups for v in g], d
        b.close()


@pytest.mark.parametrize("seeded", [0, 1])
def test_large_bounds(torch_dev, seeded):
    dags = large_workload(3, first=10) + custom_large(2)
    batch = W.from_dags(dags)
    M, K = 256, 24
    alloc = W.alloc_bytes(batch, M, K, seed=21)
    say("large bounds:", batch.num_dags, "DAGs x", K, "seeded", seeded)
    got = gpu_eval(torch_dev, batch, M, K, alloc, seed=21 if seeded else None)
    check_against_oracle(batch, M, K, alloc, got)


@pytest.mark.parametrize("M", [1, 8, 65535])
def test_large_compute_units_and_loads(torch_dev, M):
    # loads up to 2^31 - 1 (the exact-division path), and few or many units
    rng = np.random.default_rng(M)
    dags = custom_large(3)[:4]
    n, s, t, w, p = dags[0]
    w = w.copy()
    w[rng.random(n) < 0.2] = 2**31 - 1
    dags[0] = (n, s, t, w, p)
    batch = W.from_dags(dags)
    K = 12
    alloc = W.alloc_bytes(batch, M, K, seed=M + 1)
    say("large DAGs, M", M, "max load", int(batch.wcet.max()))
    got = gpu_eval(torch_dev, batch, M, K, alloc)
    check_against_oracle(batch, M, K, alloc, got)


def mixed_with_large():
    small = mixed_size_batch()
    big = large_workload(3, first=40, max_n=2000)
    dags = [small.dag(d) for d in range(small.num_dags)]
    for i, g in enumerate(big):
        dags.insert(7 + 31 * i, g)
    return W.from_dags(dags)


@pytest.mark.parametrize("classes,streams,seeded", [(1, 1, 0), (1, 0, 1), (0, 1, 0), (0, 0, 1)])
def test_mixed_batch_with_large_dags(torch_dev, classes, streams, seeded):
    # size_classes 0 runs every DAG, small ones included, in the large-DAG kernel
    batch = mixed_with_large()
    sizes = np.diff(batch.node_off)
    assert sizes.max() > 512 and (sizes <= 64).any()
    K, M = 70, 256
    alloc = W.alloc_bytes(batch, M, K, seed=9)
    say("mixed batch with large DAGs:", batch.num_dags, "DAGs, size_classes", classes, "class_streams",
        streams, "seeded", seeded)
    got = gpu_eval(torch_dev, batch, M, K, alloc, seed=9 if seeded else None,
                   tuning={"size_classes": classes, "class_streams": streams})
    check_against_oracle(batch, M, K, alloc, got)


def test_large_determinism(torch_dev):
    batch = W.from_dags(large_workload(2, first=50, max_n=2500))
    M, K = 256, 64
    say("large determinism: two runs")
    a = gpu_eval(torch_dev, batch, M, K, seed=4)
    b = gpu_eval(torch_dev, batch, M, K, seed=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_large_surrogate_search_is_exact_on_its_candidates(torch_dev):
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    batch = W.from_dags(large_workload(4, first=60, max_n=2500))
    M, K, seed, top_k = 256, 512, 7, 16
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M)
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    model = db.Model(4)
    D = batch.num_dags
    cand = torch.empty(D * (top_k + 1), dtype=torch.int32, device=dev)
    say("large surrogate selection and search:", D, "DAGs, K", K, "top", top_k)
    db.model_select(model, b, K, seed, top_k, 32, cand)
    idx = np.empty(D, np.int32)
    bb = np.empty(D, np.int64)
    db.best_allocation(b, idx, bb, search=db.SEARCH_SURROGATE, top_k=top_k, model=model)
    cand = cand.cpu().numpy().reshape(D, top_k + 1)
    b.close()
    model.close()
    # exact bounds of the listed candidates only: their rows of the seeded bytes
    full = W.alloc_bytes(batch, M, K, seed=seed)
    L = top_k + 1
    sub = np.empty(int(batch.node_off[-1]) * L, np.uint8)
    for d in range(D):
        n, n0 = batch.dag(d)[0], int(batch.node_off[d])
        for i, c in enumerate(cand[d]):
            sub[L * n0 + i * n: L * n0 + (i + 1) * n] = full[K * n0 + c * n: K * n0 + (c + 1) * n]
    want, _, _ = oracle.bounds_batch(batch, M, L, sub, threads=8)
    for d in range(D):
        assert cand[d, 0] == 0 and len(set(cand[d, 1:].tolist())) == top_k
        pos = int(np.argmin(want[d]))  # ties: the candidate listed first
        assert bb[d] == want[d, pos] and idx[d] == cand[d, pos], d


def _expect_large(code, dag, M=256):
    import paper_2602_20826_amd as db

    rng = np.random.default_rng(0)
    batch = W.from_dags([chain_with_skips(rng, 600), dag])
    with pytest.raises(db.DagboundError) as e:
        db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
    assert e.value.code == code, e.value.message
    assert "DAG 1" in e.value.message


def test_large_validation_errors(torch_dev):
    from paper_2602_20826_amd import dagbound as B

    say("large validation errors")
    n = 700
    ones = [1] * n
    chain_s, chain_d = list(range(n - 1)), list(range(1, n))
    _expect_large(B.E_CYCLE, (n, chain_s + [n - 1], chain_d + [0], ones, ones))
    _expect_large(B.E_CYCLE, (n, chain_s + [5], chain_d + [5], ones, ones))
    _expect_large(B.E_DUP_EDGE, (n, chain_s + [3], chain_d + [4], ones, ones))
    _expect_large(B.E_RANGE, (n, chain_s + [0], chain_d + [n], ones, ones))
    _expect_large(B.E_RANGE, (n, chain_s, chain_d, [1] * (n - 1) + [0], ones))
    _expect_large(B.E_RANGE, (n, chain_s, chain_d, ones, [1] * (n - 1) + [0]))
    _expect_large(B.E_OVERFLOW, (n, chain_s, chain_d, [2**31 - 1] * n, ones))
    m = 8001
    _expect_large(B.E_UNSUPPORTED, (m, [], [], [1] * m, [1] * m))


def _seeded_rows(batch, dags, M, K, seed, cands=None):
    """Explicit bytes of DAGs `dags` of `batch` (seeded as in the batch, where
    the hash takes the DAG's batch index), for candidates `cands` (default all)."""
    parts = []
    for d in dags:
        one = batch.subset([d])
        n = one.dag(0)[0]
        full = W.alloc_bytes(one, M, K, seed=seed, first=int(d)).reshape(K, n)
        parts.append(full if cands is None else full[np.asarray(cands[d])])
    return np.concatenate([p.ravel() for p in parts])


def test_large_compiler_full_size_sampled(torch_dev):
    # The large-compiler workload at its full size (10,000 DAGs of 1,000-5,000
    # nodes, about 30M nodes and 420M edges): the bench's exact evaluation (64
    # seeded candidates) and the surrogate search over 16,384 seeded
    # candidates with the top 64 verified; sampled DAGs against the oracle.
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    wl = W.WORKLOADS[5]
    say("large-compiler full size: generating", wl.num_dags, "DAGs")
    batch = W.generate_workload(5)
    D, M, K, seed = batch.num_dags, wl.num_cus, 64, 17
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    st = torch.cuda.current_stream(dev)
    say("create_batch + eval_bounds:", D, "DAGs,", int(batch.node_off[-1]), "nodes x", K)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M, stream=st)
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    out = torch.empty(D * K, dtype=torch.int64, device=dev)
    db.eval_bounds(b, out, stream=st)
    idx = torch.empty(D, dtype=torch.int32, device=dev)
    best = torch.empty(D, dtype=torch.int64, device=dev)
    db.best_allocation(b, idx, best, stream=st)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    sample = sorted(set([0, 1, D // 2, D - 1] + rng.choice(D, 6, replace=False).tolist()))
    got = out.view(D, K).cpu().numpy()[sample]
    want, _, _ = oracle.bounds_batch(batch.subset(sample), M, K, _seeded_rows(batch, sample, M, K, seed),
                                     threads=8)
    assert np.array_equal(got, want)
    assert np.array_equal(best.cpu().numpy()[sample], want.min(1))
    assert np.array_equal(idx.cpu().numpy()[sample], want.argmin(1))
    # surrogate search: 16,384 seeded candidates ranked, candidate 0 and the
    # top 64 evaluated exactly
    KS, top_k = wl.K, 64
    say("surrogate search:", KS, "candidates, top", top_k)
    db.set_allocations(b, KS, db.ALLOC_SEEDED, None, seed)
    model = db.Model(2)
    cand = torch.empty(D * (top_k + 1), dtype=torch.int32, device=dev)
    db.model_select(model, b, KS, seed, top_k, 32, cand)
    db.best_allocation(b, idx, best, search=db.SEARCH_SURROGATE, top_k=top_k, model=model, stream=st)
    torch.cuda.synchronize()
    cand = cand.view(D, top_k + 1).cpu().numpy()
    bi, bb = idx.cpu().numpy(), best.cpu().numpy()
    model.close()
    b.close()
    few = sample[:4]
    lists = {d: cand[d] for d in few}
    want, _, _ = oracle.bounds_batch(batch.subset(few), M, top_k + 1,
                                     _seeded_rows(batch, few, M, KS, seed, lists), threads=8)
    for i, d in enumerate(few):
        assert cand[d, 0] == 0 and len(set(cand[d, 1:].tolist())) == top_k
        pos = int(np.argmin(want[i]))
        assert bb[d] == want[i, pos] and bi[d] == cand[d, pos], d


def test_large_eval_in_a_captured_graph(torch_dev):
    # the large-DAG launch (its work counter reset by a kernel) captured with
    # the smaller classes on side streams; every replay equals the eager run
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    batch = mixed_with_large()
    M, K, seed = 256, 40, 31
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    st = torch.cuda.current_stream(dev)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M, stream=st)
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    D = batch.num_dags
    eager = torch.empty(D * K, dtype=torch.int64, device=dev)
    db.eval_bounds(b, eager, stream=st)
    torch.cuda.synchronize()
    out = torch.zeros(D * K, dtype=torch.int64, device=dev)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(st)
    say("capturing eval_bounds with large DAGs")
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            db.eval_bounds(b, out, stream=s)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    for rep in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("replay", rep)
        assert np.array_equal(out.cpu().numpy(), ref), rep
    want, _, _ = oracle.bounds_batch(batch, M, K, W.alloc_bytes(batch, M, K, seed=seed), threads=8)
    assert np.array_equal(ref.reshape(D, K), want)
    del g
    b.close()


@pytest.mark.parametrize("classes,seeded", [(1, 0), (1, 1), (0, 1)])
def test_node_lanes_from_257_nodes(torch_dev, classes, seeded):
    # node_lanes 256: DAGs of 257-512 nodes (and, with one launch, every DAG)
    # run the lane-per-node kernel
    batch = mixed_with_large()
    sizes = np.diff(batch.node_off)
    assert ((sizes > 256) & (sizes <= 512)).any()
    K, M = 70, 256
    alloc = W.alloc_bytes(batch, M, K, seed=19)
    say("node_lanes 256: size_classes", classes, "seeded", seeded)
    got = gpu_eval(torch_dev, batch, M, K, alloc, seed=19 if seeded else None,
                   tuning={"size_classes": classes, "node_lanes": 256})
    check_against_oracle(batch, M, K, alloc, got)


def test_autotune_with_node_lanes(torch_dev):
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    batch = mixed_with_large()
    M, K = 256, 64
    want, _, _ = oracle.bounds_batch(batch, M, K, W.alloc_bytes(batch, M, K, seed=23), threads=8)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    st = torch.cuda.current_stream(dev)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M, stream=st)
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, 23)
    db.set_tuning(b, "autotune", 1)
    for rep in range(2):
        out = torch.full((batch.num_dags * K,), -1, dtype=torch.int64, device=dev)
        say("autotune with node lanes, evaluation", rep)
        db.eval_bounds(b, out, stream=st)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().reshape(batch.num_dags, K), want), rep
    b.close()
