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


def surrogate_lists(torch, model: db.Model, b: db.Batch, K: int, seed: int, top_k: int):
    """The candidate lists a surrogate search of batch `b` evaluates (candidate
    0, then the model's top_k, as dagbound_best_allocation picks them) and
    their exact bounds from dagbound_eval_listed: two host arrays [D, top_k+1]."""
    dev = torch.device("cuda:0")
    D = b.num_dags
    cand = torch.empty(D * (top_k + 1), dtype=torch.int32, device=dev)
    db.model_select(model, b, K, seed, top_k, 32, cand)
    out = torch.empty(D * (top_k + 1), dtype=torch.int64, device=dev)
    db.eval_listed(b, cand, out)
    return cand.view(D, top_k + 1).cpu().numpy(), out.view(D, top_k + 1).cpu().numpy()


def gap_stats(x: np.ndarray, ref: np.ndarray) -> Dict:
    """Relative gap of best bounds x to the reference ref, per DAG."""
    g = x / ref - 1.0
    return {"mean": float(g.mean()), "p99": float(np.quantile(g, 0.99)), "max": float(g.max()),
            "exact_frac": float(np.mean(g == 0)), "within_1pct_frac": float(np.mean(g <= 0.01))}


def compare_search(torch, model: db.Model, dags, M: int, K: int, seed: int, top_k: int,
                   keep_lists: bool = False) -> Dict:
    """Best bounds and DAGs/s of the four searches on a held-out set.  With
    keep_lists, the result also holds the surrogate's candidate lists and
    their exact bounds ("lists", "list_bounds", host arrays [D, top_k+1])."""
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
    lists = surrogate_lists(torch, model, b, K, seed, top_k) if keep_lists else None
    # the encoder's forward pass alone (its layer GEMMs run on MFMA)
    fwd = torch.empty(int(dags.node_off[-1]) * 3, dtype=torch.float32, device=dev)
    t_fwd = timed(lambda: db.model_forward(model, b, fwd, stream=stream))
    del fwd
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
        return gap_stats(x, exh)

    res = {
        "dags": D, "K": K, "top_k": top_k,
        "exhaustive_dags_per_s": D / t_exh, "surrogate_dags_per_s": D / t_sur,
        "speedup": t_exh / t_sur,
        "forward_seconds": t_fwd,
        "forward_gemm_tflops": int(dags.node_off[-1]) * 3 * 2 * 256 * 128 / t_fwd / 1e12,
        "gap_surrogate": gap(sur), "gap_paper_rule": gap(c0), "gap_random": gap(rnd),
        "gain_over_paper_rule_mean": float(np.mean(1.0 - sur / c0)),
        "gain_over_random_mean": float(np.mean(1.0 - sur / rnd)),
        "dags_improved_over_paper_rule": int(np.sum(sur < c0)),
        "dags_improved_over_random": int(np.sum(sur < rnd)),
    }
    if lists is not None:
        res["lists"], res["list_bounds"] = lists
        res["surrogate_best"] = sur
    return res


def compare_budget(torch, model: db.Model, dags, M: int, K: int, seed: int, top_k: int, per_shard: int,
                   exh_dags: int, keep_lists: int = 0) -> Dict:
    """Surrogate-guided search against plain search at the same time budget,
    on DAGs taken per_shard at a time:
      - surrogate: candidate 0 plus the top_k of K seeded candidates ranked by
        the model, evaluated exactly (one best_allocation call, timed);
      - plain: the first K_p seeded candidates (candidate 0 and K_p - 1 random
        ones) evaluated exactly, K_p sized so that this exhaustive search takes
        about the surrogate's time (from the measured rate of a 64-candidate
        evaluation of the same shard), timed;
      - exhaustive over all K candidates on the first exh_dags DAGs of each
        shard, as the reference of the gaps (and timed, for its DAGs/s).
    Returns mean gaps and times.  With keep_lists = n, the result also holds
    the surrogate's candidate lists and their exact bounds for the first n
    DAGs of the first shard ("lists", "list_bounds", "list_best")."""
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    sur_all, plain_all, c0_all, exh_all, sur_s, plain_s, exh_s = [], [], [], [], [], [], []
    kept = None
    kps = []
    for s0 in range(0, dags.num_dags, per_shard):
        sub = dags.subset(range(s0, min(dags.num_dags, s0 + per_shard)))
        D = sub.num_dags
        b = _dev_batch(torch, dev, sub, M)
        idx = torch.empty(D, dtype=torch.int32, device=dev)
        best = torch.empty(D, dtype=torch.int64, device=dev)
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, seed)
        db.best_allocation(b, idx, best, search=db.SEARCH_SURROGATE, top_k=top_k, model=model, stream=st)
        t_sur = timed(lambda: db.best_allocation(b, idx, best, search=db.SEARCH_SURROGATE, top_k=top_k,
                                                 model=model, stream=st))
        sur = best.cpu().numpy().astype(np.float64)
        if keep_lists and s0 == 0:
            cl, bl = surrogate_lists(torch, model, b, K, seed, top_k)
            kept = (cl[:keep_lists], bl[:keep_lists], best.cpu().numpy()[:keep_lists])
        # rate of exact search on this shard, then the plain budget
        db.set_allocations(b, 64, db.ALLOC_SEEDED, None, seed)
        out64 = torch.empty(D * 64, dtype=torch.int64, device=dev)
        db.eval_bounds(b, out64, stream=st)
        t64 = timed(lambda: db.eval_bounds(b, out64, stream=st))
        kp = int(max(top_k + 1, min(K, round(64 * t_sur / t64))))
        db.set_allocations(b, kp, db.ALLOC_SEEDED, None, seed)
        outp = torch.empty(D * kp, dtype=torch.int64, device=dev)
        t_plain = timed(lambda: db.eval_bounds(b, outp, stream=st))
        pl = outp.view(D, kp)
        plain = pl.min(1).values.cpu().numpy().astype(np.float64)
        c0 = pl[:, 0].cpu().numpy().astype(np.float64)
        # exhaustive reference on the first DAGs of the shard
        ne = min(exh_dags, D)
        ex = sub.subset(range(ne))
        be = _dev_batch(torch, dev, ex, M)
        db.set_allocations(be, K, db.ALLOC_SEEDED, None, seed)
        ie = torch.empty(ne, dtype=torch.int32, device=dev)
        bx = torch.empty(ne, dtype=torch.int64, device=dev)
        exh_s.append((ne, timed(lambda: db.best_allocation(be, ie, bx, stream=st))))
        exh_all.append(bx.cpu().numpy().astype(np.float64))
        be.close()
        b.close()
        sur_all.append(sur)
        plain_all.append(plain)
        c0_all.append(c0)
        sur_s.append(t_sur)
        plain_s.append(t_plain)
        kps.append(kp)
    sur, plain, c0 = np.concatenate(sur_all), np.concatenate(plain_all), np.concatenate(c0_all)
    exh = np.concatenate(exh_all)
    first = np.concatenate([np.arange(len(x)) < len(e) for x, e in zip(sur_all, exh_all)])

    def gap(x, ref):
        return gap_stats(x, ref)

    D = len(sur)
    res = {
        "dags": D, "K": K, "top_k": top_k,
        "surrogate_seconds": float(sum(sur_s)), "plain_seconds": float(sum(plain_s)),
        "surrogate_dags_per_s": D / sum(sur_s), "plain_dags_per_s": D / sum(plain_s),
        "exhaustive_dags_per_s": sum(n for n, _ in exh_s) / sum(t for _, t in exh_s),
        "speedup_vs_exhaustive": (D / sum(sur_s)) / (sum(n for n, _ in exh_s) / sum(t for _, t in exh_s)),
        "plain_candidates": kps,
        "surrogate_vs_plain": {"mean": float(np.mean(sur / plain - 1.0)),
                               "better_frac": float(np.mean(sur < plain)),
                               "equal_frac": float(np.mean(sur == plain)),
                               "worse_frac": float(np.mean(sur > plain))},
        "gap_vs_exhaustive_dags": int(first.sum()),
        "gap_surrogate": gap(sur[first], exh),
        "gap_plain": gap(plain[first], exh),
        "gap_paper_rule": gap(c0[first], exh),
        "gain_over_paper_rule_mean": float(np.mean(1.0 - sur / c0)),
        "paper_rule_is_best_frac": float(np.mean(c0[first] == exh)),
    }
    if keep_lists:
        res["lists"], res["list_bounds"], res["list_best"] = kept
    return res
