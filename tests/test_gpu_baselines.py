"""GPU comparison bounds of Section 5.2 (dagbound_baselines: Greedy,
Greedy + unaware, Graham_para) against the oracle, bit-exact, on the paper's
worked example, the evaluation-style setups of Section 5.1, every benchmark
workload shape (small, batched-layered, persistent-mixed, large DAGs) and
edge cases.  Expected values come from `oracle` only."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import GOLDEN, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def gpu_baselines(torch_dev, batch, M, device_ptrs=True):
    import paper_2602_20826_amd as db

    torch, dev = torch_dev
    D = batch.num_dags
    if device_ptrs:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        stream = torch.cuda.current_stream(dev)
        b = db.create_batch(t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst),
                            t(batch.wcet), t(batch.par), M, stream=stream)
        out = [torch.full((D,), -1, dtype=torch.int64, device=dev) for _ in range(3)]
        db.baselines(b, *out, stream=stream)
        torch.cuda.synchronize()
        got = np.stack([x.cpu().numpy() for x in out], 1)
    else:
        b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, M)
        got = np.stack(db.baselines(b), 1)
    b.close()
    return got


def check(batch, M, got, dags=None, threads=8):
    idx = np.arange(batch.num_dags) if dags is None else np.asarray(dags)
    want = oracle.baselines_batch(batch, M, dags=idx, threads=threads)
    bad = np.argwhere(got[idx] != want)
    assert bad.size == 0, f"{len(bad)} mismatches, first DAG {idx[bad[0][0]]}: gpu {got[idx][bad[0][0]]} " \
                          f"oracle {want[bad[0][0]]}"
    assert np.all(want[:, 1] >= want[:, 0])
    return want


def test_baselines_worked_example(torch_dev):
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    e = np.asarray(ex["edges"], np.int32).reshape(-1, 2)
    batch = W.from_dags([(ex["n"], e[:, 0], e[:, 1], ex["wcet"], ex["par"])])
    say("baselines: worked example")
    got = gpu_baselines(torch_dev, batch, ex["M"])
    assert got.tolist() == [[7, 7, 6]]
    assert gpu_baselines(torch_dev, batch, ex["M"], device_ptrs=False).tolist() == [[7, 7, 6]]


@pytest.mark.parametrize("P,M", [(4, 4), (8, 32), (10, 256), (32, 32)])
def test_baselines_paper_style(torch_dev, P, M):
    batch = W.paper_style(300, P, 20)
    say("baselines: evaluation-style DAGs P", P, "M", M)
    check(batch, M, gpu_baselines(torch_dev, batch, M))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_baselines_workloads(torch_dev, k):
    wl = W.WORKLOADS[k]
    batch = W.generate_workload(k, count=3000 if k < 3 else 600)
    say("baselines: workload", k, batch.num_dags, "DAGs")
    check(batch, wl.num_cus, gpu_baselines(torch_dev, batch, wl.num_cus))
    check(batch, 8, gpu_baselines(torch_dev, batch, 8, device_ptrs=False))


def test_baselines_large_dags(torch_dev):
    from test_gpu_large import custom_large, large_workload

    batch = W.from_dags(large_workload(4, first=20) + custom_large(5))
    say("baselines: large DAGs", np.diff(batch.node_off).tolist())
    for M in (256, 3):
        check(batch, M, gpu_baselines(torch_dev, batch, M))


def test_baselines_full_size_sampled(torch_dev):
    # the whole batched-layered workload on the GPU, a seeded sample of its
    # DAGs (and the first and last) on the oracle
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2)
    say("baselines: batched-layered full size", batch.num_dags, "DAGs")
    got = gpu_baselines(torch_dev, batch, wl.num_cus)
    rng = np.random.default_rng(17)
    sample = np.unique(np.concatenate([[0, batch.num_dags - 1], rng.integers(0, batch.num_dags, 3000)]))
    check(batch, wl.num_cus, got, dags=sample)


def test_baselines_edge_cases(torch_dev):
    import paper_2602_20826_amd as db

    rng = np.random.default_rng(9)
    dags = [
        (0, [], [], [], []),                                   # empty DAG
        (1, [], [], [100], [10]),                              # one node, m^max above M
        (5, [], [], [3, 9, 1, 4, 4], [1, 2, 3, 40, 5]),         # no edges
        (4, [0, 1, 2], [1, 2, 3], [5, 5, 5, 5], [1, 1, 1, 1]),  # chain, p = 1
        (3, [0, 0], [1, 2], [2147483647, 2147483647, 1], [2147483647, 7, 1]),  # largest loads
    ]
    n = 130
    dags.append((n, np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32),
                 rng.integers(1, 1000, n), rng.integers(1, 3000, n)))  # star: 129 successors of one node
    batch = W.from_dags(dags)
    for M in (1, 4, 65535):
        say("baselines: edge cases M", M)
        got = check(batch, M, gpu_baselines(torch_dev, batch, M))
        assert got[0].tolist() == [0, 0, 0]
    # one output only, and none at all
    b = db.create_batch(batch.node_off, batch.edge_off, batch.src, batch.dst, batch.wcet, batch.par, 4)
    only = np.full(batch.num_dags, -1, np.int64)
    db.baselines(b, None, None, only)
    assert np.array_equal(only, oracle.baselines_batch(batch, 4)[:, 2])
    db.baselines(b, None, None, None)
    b.close()
