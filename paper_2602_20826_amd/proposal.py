"""Training and measuring the learned candidate proposal through the C-ABI.

The exact evaluation kernel labels seeded (DAG, candidate) tuples; the
model's own GPU kernels train on them (dagbound_model_train_step); the
search compares, per DAG, the best exact bound found by
  - the paper's rule alone (candidate 0),
  - candidate 0 plus the first `top_k` seeded candidates (plain random),
  - candidate 0 plus the `top_k` candidates the model ranks best,
  - exhaustive exact evaluation of all K candidates.
Everything runs on the current HIP device; torch only holds device memory.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Dict, List, Sequence

import numpy as np

from . import dagbound as db


@dataclass
class Shard:
    """A device-resident group of DAGs with exact labels for K seeded candidates."""

    batch: db.Batch
    K: int
    seed: int
    bounds: object  # torch int64 [D*K] on the device


def _dev_batch(torch, dev, b, M):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    keep = [t(b.node_off), t(b.edge_off), t(b.src), t(b.dst), t(b.wcet), t(b.par)]
    return db.create_batch(*keep, M)


def label_shards(torch, dags, M: int, K: int, seed: int, per_shard: int) -> List[Shard]:
    """Split a workloads.DagBatch into shards of per_shard DAGs and label every
    (DAG, seeded candidate) pair with its exact bound."""
    dev = torch.device("cuda:0")
    shards = []
    for s0 in range(0, dags.num_dags, per_shard):
        sub = dags.subset(range(s0, min(dags.num_dags, s0 + per_shard)))
        b = _dev_batch(torch, dev, sub, M)
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
        out = torch.empty(sub.num_dags * K, dtype=torch.int64, device=dev)
        db.eval_bounds(b, out)
        shards.append(Shard(b, K, seed, out))
    torch.cuda.synchronize()
    return shards


def train(model: db.Model, shards: Sequence[Shard], epochs: int, lr: float = 2e-3,
          lr_end: float = 2e-4) -> List[float]:
    """Adam over the shards in order, epochs times, with a geometric learning
    rate decay from lr to lr_end.  Returns the mean loss of each epoch."""
    total = max(1, epochs * len(shards))
    hist = []
    step = 0
    for _ in range(epochs):
        acc = 0.0
        for sh in shards:
            rate = lr * (lr_end / lr) ** (step / max(1, total - 1))
            acc += db.model_train_step(model, sh.batch, sh.K, sh.seed, sh.bounds, rate)
            step += 1
        hist.append(acc / len(shards))
    return hist


def compare_search(torch, model: db.Model, dags, M: int, K: int, seed: int, top_k: int) -> Dict:
    """Best bounds and DAGs/s of the four searches on a held-out set."""
    dev = torch.device("cuda:0")
    D = dags.num_dags
    b = _dev_batch(torch, dev, dags, M)
    idx = torch.empty(D, dtype=torch.int32, device=dev)
    best_exh = torch.empty(D, dtype=torch.int64, device=dev)
    best_sur = torch.empty(D, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # exhaustive: every candidate evaluated exactly (fresh allocation set, no reuse)
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    t_exh = timed(lambda: db.best_allocation(b, idx, best_exh, stream=stream))
    # surrogate-guided: encoder + head + top_k exact
    db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
    db.best_allocation(b, idx, best_sur, search=db.SEARCH_SURROGATE, top_k=top_k, model=model,
                       stream=stream)  # warm
    t_sur = timed(lambda: db.best_allocation(b, idx, best_sur, search=db.SEARCH_SURROGATE, top_k=top_k,
                                             model=model, stream=stream))
    # paper's rule and plain random: candidates 0..top_k of the same seeded set
    db.set_allocations(b, top_k + 1, db.ALLOC_SEEDED, None, seed)
    small = torch.empty(D * (top_k + 1), dtype=torch.int64, device=dev)
    db.eval_bounds(b, small, stream=stream)
    torch.cuda.synchronize()
    small = small.cpu().numpy().reshape(D, top_k + 1)
    exh = best_exh.cpu().numpy().astype(np.float64)
    sur = best_sur.cpu().numpy().astype(np.float64)
    c0 = small[:, 0].astype(np.float64)
    rnd = small.min(1).astype(np.float64)
    b.close()

    def gap(x):
        g = x / exh - 1.0
        return {"mean": float(g.mean()), "p99": float(np.quantile(g, 0.99)), "max": float(g.max()),
                "exact_frac": float(np.mean(g == 0))}

    return {
        "dags": D, "K": K, "top_k": top_k,
        "exhaustive_dags_per_s": D / t_exh, "surrogate_dags_per_s": D / t_sur,
        "speedup": t_exh / t_sur,
        "gap_surrogate": gap(sur), "gap_paper_rule": gap(c0), "gap_random": gap(rnd),
        "gain_over_paper_rule_mean": float(np.mean(1.0 - sur / c0)),
        "gain_over_random_mean": float(np.mean(1.0 - sur / rnd)),
        "dags_improved_over_paper_rule": int(np.sum(sur < c0)),
    }
