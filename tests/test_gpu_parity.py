"""GPU parity: libdagbound (gfx950 kernels, called through the C-ABI) against
the CPU oracle, element by element, bit-exact int64.

Inputs come from the seeded generator in `workloads`; expected values come
from `oracle` only.  Every test prints the case it runs before touching the
GPU.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20826_amd as db

    db.load_library()
    return torch, torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def gpu_eval(torch_dev, batch, M, K, alloc=None, seed=None, device_ptrs=True, terms=True, tuning=None,
             para_mode=None):
    """Run create_batch / set_allocations / eval_bounds / best_allocation."""
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    D = batch.num_dags
    if device_ptrs:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        stream = torch.cuda.current_stream(dev)
        b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst),
                            t(batch.wcet), t(batch.par), M, stream=stream)
        if para_mode is not None:
            db.set_para_launch(b, para_mode)
        for key, val in (tuning or {}).items():
            db.set_tuning(b, key, val)
        if seed is None:
            a_dev = t(alloc)
            db.set_allocations(b, K, db.ALLOC_EXPLICIT, a_dev)
        else:
            db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
        bounds = torch.empty(D * K, dtype=torch.int64, device=dev)
        cp = torch.empty(D * K, dtype=torch.int64, device=dev) if terms else None
        it = torch.empty(D * K, dtype=torch.int64, device=dev) if terms else None
        db.eval_bounds(b, bounds, cp, it, stream=stream)
        bi = torch.empty(D, dtype=torch.int32, device=dev)
        bb = torch.empty(D, dtype=torch.int64, device=dev)
        db.best_allocation(b, bi, bb, stream=stream)
        torch.cuda.synchronize()
        out = [x.cpu().numpy() if x is not None else None for x in (bounds, cp, it, bi, bb)]
    else:
        b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet,
                            batch.par, M)
        if para_mode is not None:
            db.set_para_launch(b, para_mode)
        for key, val in (tuning or {}).items():
            db.set_tuning(b, key, val)
        if seed is None:
            db.set_allocations(b, K, db.ALLOC_EXPLICIT, alloc)
        else:
            db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
        bounds = np.empty(D * K, np.int64)
        cp = np.empty(D * K, np.int64) if terms else None
        it = np.empty(D * K, np.int64) if terms else None
        db.eval_bounds(b, bounds, cp, it)
        bi = np.empty(D, np.int32)
        bb = np.empty(D, np.int64)
        db.best_allocation(b, bi, bb)
        out = [bounds, cp, it, bi, bb]
    b.close()
    bounds, cp, it, bi, bb = out
    rs = lambda x: None if x is None else x.reshape(D, K)
    return rs(bounds), rs(cp), rs(it), bi, bb


def check_against_oracle(batch, M, K, alloc, got, dags=None, threads=8, para_mode=oracle.SPATIAL):
    bounds, cp, it, bi, bb = got
    idx = np.arange(batch.num_dags) if dags is None else np.asarray(dags)
    wb, wc, wi = oracle.bounds_batch(batch, M, K, alloc, dags=idx, threads=threads, para_mode=para_mode)
    bad = np.argwhere(bounds[idx] != wb)
    assert bad.size == 0, f"{len(bad)} mismatches, first (dag, cand) = {idx[bad[0][0]]}, {bad[0][1]}: " \
                          f"gpu {bounds[idx][tuple(bad[0])]} oracle {wb[tuple(bad[0])]}"
    if cp is not None:
        assert np.array_equal(cp[idx], wc)
        assert np.array_equal(it[idx], wi)
    assert np.array_equal(bb[idx], wb.min(1))
    assert np.array_equal(bi[idx], wb.argmin(1))  # ties to the smallest candidate
    return wb


# ---------------------------------------------------------------- paper cases

def golden_batches():
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    cases = [ex] + json.load(open(os.path.join(GOLDEN, "hand_cases.json")))["cases"]
    for c in cases:
        e = np.asarray(c["edges"], np.int32).reshape(-1, 2)
        yield c, W.from_dags([(c["n"], e[:, 0], e[:, 1], c["wcet"], c["par"])])


@pytest.mark.parametrize("case_i", range(8))
def test_golden_cases(torch_dev, case_i):
    cases = list(golden_batches())
    if case_i >= len(cases):
        pytest.skip("no such case")
    c, batch = cases[case_i]
    M = c["M"]
    K = 3
    rng = np.random.default_rng(case_i)
    n = c["n"]
    alloc = np.zeros(K * n, np.uint8)
    alloc[n:2 * n] = np.asarray(c.get("r", [0] * n), np.uint8)
    alloc[2 * n:] = W.random_alloc(rng, np.asarray(c["par"]), M, 0.3)
    say("golden case", c["name"][:60], "M", M)
    got = gpu_eval(torch_dev, batch, M, K, alloc)
    wb = check_against_oracle(batch, M, K, alloc, got)
    want = c["expect"]["bound"]
    assert got[0][0, 0] == want or "r" in c
    if "r" in c:
        assert got[0][0, 1] == want


def test_division_tables_match_oracle(torch_dev):
    import paper_2602_20826_amd as db

    batch = W.generate_workload(1, count=50)
    cases = list(golden_batches())
    say("division tables: 50 ER DAGs + golden cases")
    for bt, M in [(batch, 8)] + [(b, c["M"]) for c, b in cases]:
        b = db.create_batch(bt.node_off, bt.edge_off, bt.src, bt.dst, bt.wcet, bt.par, M)
        for d in range(bt.num_dags):
            n, s, t, w, p = bt.dag(d)
            want = oracle.division(n, s, t, w, p, M)
            wanc, gof, order, ng = db.get_division(b, d)
            assert wanc.tolist() == want.wanc.tolist()
            assert ng == len(want.groups)
            assert order.tolist() == [v for g in want.groups for v in g]
        b.close()


# ---------------------------------------------------------------- workloads

def test_small_er_workload_full(torch_dev):
    wl = W.WORKLOADS[1]
    batch = W.generate_workload(1)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=101)
    say("small-er workload: 1000 DAGs x 16 candidates, M=8, device pointers")
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc)
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got)


def test_small_er_workload_host_pointers_and_zero_bytes(torch_dev):
    wl = W.WORKLOADS[1]
    batch = W.generate_workload(1, count=300, first=500)
    rng = np.random.default_rng(7)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=5, first=500)
    # some candidates mix the paper's rule (0) with explicit bytes, some
    # exceed p (clamped), some are 255
    mask = rng.random(alloc.shape) < 0.2
    alloc[mask] = 0
    alloc[rng.random(alloc.shape) < 0.05] = 255
    say("small-er 300 DAGs, host pointers, mixed zero / 255 bytes")
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc, device_ptrs=False)
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got)


def test_batched_layered_slice(torch_dev):
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2, count=3000, first=1234)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=9, first=1234)
    say("batched-layered slice: 3000 DAGs x 64, M=256")
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc)
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got)


def test_batched_layered_full_size_sampled(torch_dev):
    # The whole 100,000-DAG batch as the benchmark runs it; the oracle checks
    # every candidate of a seeded sample of DAGs, and every DAG's minimum
    # must not exceed its candidate-0 bound.
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=wl.seed)
    say("batched-layered full size: 100000 DAGs x 64 (sampled check)")
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc, terms=False)
    rng = np.random.default_rng(42)
    sample = np.sort(rng.choice(batch.num_dags, 400, replace=False))
    sample = np.r_[sample, [0, batch.num_dags - 1]]
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got, dags=sample)
    bounds = got[0]
    assert np.all(got[4] <= bounds[:, 0])
    assert np.all(bounds > 0)


@pytest.mark.timeout(600)
def test_persistent_mixed_full_size_sampled(torch_dev):
    # The whole 1,000,000-DAG persistent-mixed batch (about 197M nodes and
    # 1.1G edges) with 256 seeded candidates per DAG, as bench.py runs it with
    # --workload persistent-mixed --seeded; the oracle checks every candidate
    # of a seeded sample of DAGs.
    wl = W.WORKLOADS[3]
    say("persistent-mixed full size: generating", wl.num_dags, "DAGs")
    batch = W.generate_workload(3)
    say("persistent-mixed full size:", batch.num_dags, "DAGs x", wl.K, "seeded (sampled check)")
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, seed=wl.seed, terms=False)
    rng = np.random.default_rng(43)
    sample = np.r_[0, np.sort(rng.choice(batch.num_dags, 120, replace=False)), batch.num_dags - 1]
    parts = [W.alloc_bytes(batch.subset([d]), wl.num_cus, wl.K, seed=wl.seed, first=int(d)) for d in sample]
    sub = batch.subset(sample)
    sub_got = [x[sample] if x is not None else None for x in got]
    check_against_oracle(sub, wl.num_cus, wl.K, np.concatenate(parts), sub_got)
    assert np.all(got[4] <= got[0][:, 0])


def test_seeded_mode_matches_explicit_bytes(torch_dev):
    # The GPU draws seeded candidate bytes itself; the generator draws the
    # same published counter hash into explicit bytes for the oracle.
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2, count=500)
    K = 96  # two tiles, the second ragged
    alloc = W.alloc_bytes(batch, wl.num_cus, K, seed=77)
    say("seeded mode: 500 DAGs x 96")
    got = gpu_eval(torch_dev, batch, wl.num_cus, K, seed=77)
    check_against_oracle(batch, wl.num_cus, K, alloc, got)


@pytest.mark.parametrize("tuning", [{"eval_path": 1}, {"residual_slots": 1}, {"residual_slots": 2},
                                    {"residual_slots": 12}, {"size_classes": 0},
                                    {"size_classes": 0, "residual_slots": 1}],
                         ids=["global-pass-only", "one-slot", "two-slots", "twelve-slots", "one-launch",
                              "one-launch-one-slot"])
def test_second_pass_paths(torch_dev, tuning):
    # The global-memory pass alone, and the first pass with tiny residual
    # tables so that many tiles overflow and are handed over; twelve slots
    # asked of DAGs up to 128 nodes, whose tables hold ten.
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2, count=700, first=50)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=21, first=50)
    say("second pass", tuning)
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc, tuning=tuning)
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got)
    got = gpu_eval(torch_dev, W.generate_workload(1, count=200), 8, 16,
                   W.alloc_bytes(W.generate_workload(1, count=200), 8, 16, seed=2), tuning=tuning)
    check_against_oracle(W.generate_workload(1, count=200), 8, 16,
                         W.alloc_bytes(W.generate_workload(1, count=200), 8, 16, seed=2), got)


def test_overflow_beyond_global_tables(torch_dev):
    # One residual slot: far more than 256 tiles overflow, so the tiles left
    # after the global tables are taken go through the second pass.
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2, count=3000, first=9000)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=8, first=9000)
    say("overflow beyond the global tables: 3000 DAGs, one slot")
    got = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc, tuning={"residual_slots": 1})
    check_against_oracle(batch, wl.num_cus, wl.K, alloc, got)


@pytest.mark.parametrize("top", [(1 << 20) - 1, 1 << 20, 1 << 28])
def test_load_ranges(torch_dev, top):
    # Loads drawn up to `top`: below 2^20 the kernels divide in single
    # precision (exact there), from 2^20 on in integer arithmetic.
    rng = np.random.default_rng(top & 0xFFFF)
    base = W.generate_workload(2, count=300, first=4000)
    dags = []
    for d in range(base.num_dags):
        n, src, dst, _, par = base.dag(d)
        w = rng.integers(top // 2, top + 1, n)
        small = rng.random(n) < 0.3
        w[small] = rng.integers(1, 1000, int(small.sum()))
        dags.append((n, src, dst, w, par))
    batch = W.from_dags(dags)
    assert int(batch.wcet.max()) <= top and int(batch.wcet.max()) > top // 2
    M, K = 256, 64
    alloc = W.alloc_bytes(batch, M, K, seed=4)
    say("load ranges up to", top)
    got = gpu_eval(torch_dev, batch, M, K, alloc)
    check_against_oracle(batch, M, K, alloc, got)


def mixed_size_batch():
    """DAGs of all four size classes (<= 64, 128, 256, 512 nodes), interleaved."""
    a = W.generate_workload(1, count=40)
    b = W.generate_workload(2, count=40, first=300)
    full = W.generate_workload(3, count=300, first=77)
    mid = [d for d in range(full.num_dags) if 128 < full.dag(d)[0] <= 256][:12]
    big = [d for d in range(full.num_dags) if 256 < full.dag(d)[0] <= 400 and len(full.dag(d)[1]) <= 4000][:3]
    dags = []
    for i in range(40):
        dags.append(a.dag(i))
        dags.append(b.dag(i))
        if i < len(mid):
            dags.append(full.dag(mid[i]))
        if i < len(big):
            dags.append(full.dag(big[i]))
    return W.from_dags(dags)


@pytest.mark.parametrize("classes,streams,persistent,seeded",
                         [(1, 1, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (1, 1, 1, 0), (0, 0, 1, 0),
                          (1, 1, 0, 1), (0, 1, 0, 1), (1, 0, 1, 1)])
def test_mixed_size_classes(torch_dev, classes, streams, persistent, seeded):
    # seeded: DAGs above 128 nodes draw their candidate bytes where they use them
    batch = mixed_size_batch()
    sizes = np.diff(batch.node_off)
    assert sizes.max() > 256 and (sizes <= 64).any() and ((sizes > 64) & (sizes <= 128)).any()
    K, M = 70, 256
    alloc = W.alloc_bytes(batch, M, K, seed=5)
    say("mixed size classes:", batch.num_dags, "DAGs, size_classes", classes, "class_streams", streams,
        "persistent", persistent, "seeded", seeded)
    got = gpu_eval(torch_dev, batch, M, K, alloc, seed=5 if seeded else None,
                   tuning={"size_classes": classes, "class_streams": streams, "persistent": persistent})
    check_against_oracle(batch, M, K, alloc, got)


def test_autotune_keeps_results(torch_dev):
    # The autotuning evaluation runs every launch plan; its results and the
    # next evaluation's (with the chosen plan) both match the oracle.
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    batch = mixed_size_batch()
    M, K = 256, 64
    alloc = W.alloc_bytes(batch, M, K, seed=13)
    want, _, _ = oracle.bounds_batch(batch, M, K, alloc, threads=8)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    st = torch.cuda.current_stream(dev)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M, stream=st)
    a_dev = t(alloc)
    db.set_allocations(b, K, db.ALLOC_EXPLICIT, a_dev)
    db.set_tuning(b, "autotune", 1)
    for rep in range(2):
        out = torch.full((batch.num_dags * K,), -1, dtype=torch.int64, device=dev)
        say("autotune evaluation", rep)
        db.eval_bounds(b, out, stream=st)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().reshape(batch.num_dags, K), want), rep
    b.close()


def test_tuning_rejects_bad_keys(torch_dev):
    import paper_2602_20826_amd as db

    batch = W.generate_workload(1, count=2)
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 8)
    for key, val in [("residual_slots", 0), ("residual_slots", 13), ("eval_path", 2), ("size_classes", 2), ("class_streams", 3), ("persistent", 2), ("autotune", -1),
                     ("graph", 2), ("node_lanes", 128), ("nope", 1)]:
        with pytest.raises(db.DagboundError):
            db.set_tuning(b, key, val)
    b.close()


@pytest.mark.parametrize("K", [1, 5, 63, 65, 130])
def test_ragged_candidate_counts(torch_dev, K):
    wl = W.WORKLOADS[1]
    batch = W.generate_workload(1, count=60, first=17)
    alloc = W.alloc_bytes(batch, wl.num_cus, K, seed=K)
    say("ragged K", K)
    got = gpu_eval(torch_dev, batch, wl.num_cus, K, alloc)
    check_against_oracle(batch, wl.num_cus, K, alloc, got)


def test_persistent_mixed_shapes_that_fit(torch_dev):
    # DAGs of the persistent-mixed workload up to the evaluation kernel's LDS
    # budget (uneven sizes, ER and layered, log-uniform loads up to 1e5).
    wl = W.WORKLOADS[3]
    full = W.generate_workload(3, count=400)
    keep = [d for d in range(full.num_dags) if full.dag(d)[0] <= 200 and len(full.dag(d)[1]) <= 3000]
    batch = full.subset(keep[:120])
    K = 64
    alloc = W.alloc_bytes(batch, wl.num_cus, K, seed=3)
    say("persistent-mixed subset:", batch.num_dags, "DAGs x", K)
    got = gpu_eval(torch_dev, batch, wl.num_cus, K, alloc)
    check_against_oracle(batch, wl.num_cus, K, alloc, got)


# ---------------------------------------------------------------- edge cases

def test_edge_cases(torch_dev):
    rng = np.random.default_rng(5)
    dags = [
        (0, [], [], [], []),                                   # empty DAG
        (1, [], [], [7], [3]),                                 # single node
        (5, [], [], [3, 9, 1, 4, 4], [1, 2, 3, 4, 5]),          # no edges
        (4, [0, 1, 2], [1, 2, 3], [5, 5, 5, 5], [1, 1, 1, 1]),  # chain, p = 1
        (3, [0, 0], [1, 2], [2147483647, 2147483647, 1], [1 << 30, 7, 1]),  # largest loads
    ]
    n = 64
    order = rng.permutation(n)
    dags.append((n, order[:-1].astype(np.int32), order[1:].astype(np.int32),
                 rng.integers(1, 100, n), rng.integers(1, 300, n)))   # 64-node chain, ids shuffled
    n = 65
    dags.append((n, np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32),
                 rng.integers(1, 1000, n), rng.integers(1, 300, n)))  # star, crosses a bitset word
    batch = W.from_dags(dags)
    for M in (1, 3, 256, 65535):
        K = 70
        alloc = np.zeros(K * int(batch.node_off[-1]), np.uint8)
        for d in range(batch.num_dags):
            nd = batch.dag(d)[0]
            n0 = int(batch.node_off[d])
            for c in range(1, K):
                alloc[K * n0 + c * nd: K * n0 + (c + 1) * nd] = rng.integers(0, 256, nd)
        say("edge cases M", M)
        got = gpu_eval(torch_dev, batch, M, K, alloc)
        check_against_oracle(batch, M, K, alloc, got)
        assert np.all(got[0][0] == 0) and got[3][0] == 0


def test_empty_batch(torch_dev):
    import paper_2602_20826_amd as db

    say("empty batch")
    b = db.create_batch(np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(0, np.int32),
                        np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0, np.int32), 8)
    db.set_allocations(b, 4, db.ALLOC_EXPLICIT, np.zeros(0, np.uint8))
    db.eval_bounds(b, np.zeros(0, np.int64))
    db.best_allocation(b, np.zeros(0, np.int32), np.zeros(0, np.int64))
    b.close()


def test_largest_dag_that_fits(torch_dev):
    # a 300-node DAG (five 64-bit bitset words) with skip edges
    rng = np.random.default_rng(11)
    n = 300
    src, dst = [], []
    for i in range(n - 1):
        src.append(i); dst.append(i + 1)
        if i + 5 < n and rng.random() < 0.5:
            src.append(i); dst.append(i + 5)
    perm = rng.permutation(n).astype(np.int32)
    batch = W.from_dags([(n, perm[src], perm[dst], rng.integers(1, 10**5, n), rng.integers(1, 64, n))])
    K = 64
    alloc = W.alloc_bytes(batch, 256, K, seed=1)
    say("largest DAG: 300 nodes")
    got = gpu_eval(torch_dev, batch, 256, K, alloc)
    check_against_oracle(batch, 256, K, alloc, got)


def test_determinism(torch_dev):
    wl = W.WORKLOADS[1]
    batch = W.generate_workload(1, count=200)
    alloc = W.alloc_bytes(batch, wl.num_cus, wl.K, seed=1)
    say("determinism: two runs")
    a = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc)
    b = gpu_eval(torch_dev, batch, wl.num_cus, wl.K, alloc)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_best_allocation_ties_pick_smallest(torch_dev):
    wl = W.WORKLOADS[1]
    batch = W.generate_workload(1, count=40)
    K = 20
    # every candidate equal to candidate 1 -> ties everywhere except c = 0
    one = W.alloc_bytes(batch, wl.num_cus, 2, seed=3)
    alloc = np.zeros(K * int(batch.node_off[-1]), np.uint8)
    for d in range(batch.num_dags):
        n = batch.dag(d)[0]
        n0 = int(batch.node_off[d])
        row = one[2 * n0 + n: 2 * n0 + 2 * n]
        for c in range(1, K):
            alloc[K * n0 + c * n: K * n0 + (c + 1) * n] = row
    say("ties")
    got = gpu_eval(torch_dev, batch, wl.num_cus, K, alloc)
    wb = check_against_oracle(batch, wl.num_cus, K, alloc, got)
    assert set(got[3].tolist()) <= {0, 1}


# ---------------------------------------------------------------- errors

def _expect(code, *dag, M=8):
    import paper_2602_20826_amd as db

    batch = W.from_dags([(3, [0], [1], [1, 1, 1], [1, 1, 1]), dag])
    with pytest.raises(db.DagboundError) as e:
        db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
    assert e.value.code == code, e.value.message
    assert "DAG 1" in e.value.message


def test_validation_errors(torch_dev):
    from paper_2602_20826_amd import dagbound as B

    say("validation errors")
    _expect(B.E_CYCLE, 3, [0, 1, 2], [1, 2, 0], [1, 1, 1], [1, 1, 1])
    _expect(B.E_CYCLE, 3, [1], [1], [1, 1, 1], [1, 1, 1])
    _expect(B.E_DUP_EDGE, 3, [0, 0], [1, 1], [1, 1, 1], [1, 1, 1])
    _expect(B.E_RANGE, 3, [0], [3], [1, 1, 1], [1, 1, 1])
    _expect(B.E_RANGE, 3, [-1], [0], [1, 1, 1], [1, 1, 1])
    _expect(B.E_RANGE, 3, [0], [1], [1, 0, 1], [1, 1, 1])
    _expect(B.E_RANGE, 3, [0], [1], [1, 2**31, 1], [1, 1, 1])
    _expect(B.E_RANGE, 3, [0], [1], [1, 1, 1], [1, 0, 1])
    n = 8001
    _expect(B.E_UNSUPPORTED, n, [], [], [1] * n, [1] * n)


def test_state_errors(torch_dev):
    import paper_2602_20826_amd as db
    from paper_2602_20826_amd import dagbound as B

    say("state errors")
    batch = W.generate_workload(1, count=3)
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 8)
    with pytest.raises(db.DagboundError) as e:
        db.eval_bounds(b, np.zeros(3, np.int64))
    assert e.value.code == B.E_STATE
    with pytest.raises(db.DagboundError) as e:
        db.best_allocation(b, np.zeros(3, np.int32), np.zeros(3, np.int64), search=B.SEARCH_SURROGATE)
    assert e.value.code == B.E_ARG
    with pytest.raises(db.DagboundError) as e:
        db.set_allocations(b, 0, B.ALLOC_EXPLICIT, np.zeros(0, np.uint8))
    assert e.value.code == B.E_ARG
    b.close()


def test_eval_bounds_in_a_captured_graph(torch_dev):
    # eval_bounds on device pointers records only kernels and events, so a
    # caller can capture it (here with the class launches on side streams)
    # and replay it; every replay must equal the eager result.
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    batch = mixed_size_batch()
    M, K = 256, 64
    alloc = W.alloc_bytes(batch, M, K, seed=12)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M, stream=torch.cuda.current_stream(dev))
    a_dev = t(alloc)
    db.set_allocations(b, K, db.ALLOC_EXPLICIT, a_dev)
    D = batch.num_dags
    eager = torch.empty(D * K, dtype=torch.int64, device=dev)
    db.eval_bounds(b, eager, stream=torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    out = torch.zeros(D * K, dtype=torch.int64, device=dev)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream(dev))
    say("capturing eval_bounds")
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
    want, _, _ = oracle.bounds_batch(batch, M, K, alloc, threads=8)
    assert np.array_equal(ref.reshape(D, K), want)
    del g
    b.close()


def test_library_graph_replays(torch_dev):
    # set_tuning("graph", 1): eval_bounds records its launches once per
    # (outputs, stream, allocation set, tuning) and replays the graph; every
    # replay and the re-recorded graph after new allocations match the oracle
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    batch = mixed_size_batch()
    M, K = 256, 48
    D = batch.num_dags
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    s = torch.cuda.Stream()
    b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet),
                        t(batch.par), M, stream=s)
    db.set_tuning(b, "graph", 1)
    out = torch.empty(D * K, dtype=torch.int64, device=dev)
    cp = torch.empty(D * K, dtype=torch.int64, device=dev)
    bi = torch.empty(D, dtype=torch.int32, device=dev)
    bb = torch.empty(D, dtype=torch.int64, device=dev)
    for seed in (5, 6):
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
        want, wcp, _ = oracle.bounds_batch(batch, M, K, W.alloc_bytes(batch, M, K, seed=seed), threads=8)
        for rep in range(3):
            say("library graph: seed", seed, "replay", rep)
            with torch.cuda.stream(s):
                out.fill_(-1)
                cp.fill_(-1)
                db.eval_bounds(b, out, cp, stream=s)
                db.best_allocation(b, bi, bb, stream=s)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().reshape(D, K), want), (seed, rep)
            assert np.array_equal(cp.cpu().numpy().reshape(D, K), wcp), (seed, rep)
            assert np.array_equal(bb.cpu().numpy(), want.min(1))
            assert np.array_equal(bi.cpu().numpy(), want.argmin(1))
    b.close()
