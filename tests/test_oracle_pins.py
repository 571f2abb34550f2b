"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the expected values come from
the paper's worked example (Sections 3.2, 4.1, 4.2), from schedules derived by
hand from the paper's rules (tests/golden/hand_cases.json, each case with its
derivation), from closed forms of special DAGs, from lower bounds any valid
schedule obeys, from brute-force enumeration of every dispatch order in the
block execution model (Section 2.2), and from structural claims the paper
makes (Sections 3.1, 3.2, 4.1).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def edges_of(case):
    e = np.asarray(case["edges"], np.int32).reshape(-1, 2)
    return e[:, 0].copy(), e[:, 1].copy()


def reachability(n, src, dst):
    """Ancestor matrix by Warshall's transitive closure (independent of the
    oracle's backward search): R[v, u] = u is a transitive predecessor of v."""
    R = np.zeros((n, n), bool)
    for u, v in zip(src, dst):
        R[v, u] = True
    for k in range(n):
        R |= R[:, [k]] & R[[k], :]
    return R


# ---------------------------------------------------------------- worked example

def test_worked_example_division():
    ex = load("worked_example.json")
    src, dst = edges_of(ex)
    d = oracle.division(ex["n"], src, dst, ex["wcet"], ex["par"], ex["M"])
    exp = ex["expect"]
    assert d.theta == exp["theta"]
    blocks = [sorted(np.nonzero(d.block == k)[0].tolist()) for k in range(len(d.theta) + 1)]
    assert blocks == exp["blocks"]
    assert [sorted(g) for g in d.groups] == exp["groups_as_sets"]
    # Eq. 2 checked against a transitive closure computed independently
    R = reachability(ex["n"], src, dst)
    w = np.asarray(ex["wcet"])
    assert d.wanc.tolist() == (w + (R * w[None, :]).sum(1)).tolist()


def test_worked_example_paths_are_in_block_forests():
    # Section 3.1: inside a block each node has at most one in-block
    # predecessor; the local complete paths of the example follow from it.
    ex = load("worked_example.json")
    src, dst = edges_of(ex)
    d = oracle.division(ex["n"], src, dst, ex["wcet"], ex["par"], ex["M"])
    for k, exp_paths in enumerate(ex["expect"]["paths"]):
        members = set(np.nonzero(d.block == k)[0].tolist())
        succ = {v: [t for s, t in zip(src, dst) if s == v and t in members] for v in members}
        has_pred = {t for s, t in zip(src, dst) if s in members and t in members}
        paths = []

        def walk(p):
            nxt = succ[p[-1]]
            if not nxt:
                paths.append(p)
            for t in nxt:
                walk(p + [int(t)])

        for v in sorted(members - has_pred):
            walk([v])
        assert sorted(paths) == sorted(exp_paths)


def test_worked_example_schedule_and_bound():
    ex = load("worked_example.json")
    src, dst = edges_of(ex)
    s = oracle.bound(ex["n"], src, dst, ex["wcet"], ex["par"], ex["M"], trace=True)
    exp = ex["expect"]
    assert s.bound == exp["bound"] == 5  # Section 4.2: R(G) <= 5
    slot2 = s.slots[1]
    members = {p.node: p for p in slot2.parts if p.kind == 0}
    assert {str(k): v.m for k, v in members.items()} == exp["slot2"]["m"]  # m3 = m4 = 2
    # WS_2 = max C * (M - sum m) = 1 * (6 - 4) = 2 (Eq. 6)
    sum_m_members = sum(p.m for p in members.values())
    assert slot2.maxC * (ex["M"] - sum_m_members) == exp["slot2"]["WS"]
    segs = [p for p in slot2.parts if p.kind == 2]
    assert len(segs) == 1
    seg = exp["slot2"]["segment"]
    assert (segs[0].node, segs[0].m, segs[0].load) == (seg["node"], seg["m"], seg["load"])
    # the residual of v2 runs with its own group pi_3 (Section 4.1 example)
    res = [p for p in s.slots[2].parts if p.node == seg["node"]]
    assert len(res) == 1 and res[0].kind == 0 and res[0].load == seg["residual"]
    got_edges = {(a, ap, b, bp) for (_, a, ap, b, bp) in s.edges}
    for e in exp["extra_edges_contain"]:
        assert tuple(e) in got_edges


def test_worked_example_greedy_overload():
    # Section 4.2: under Greedy (m_i = m_i^max, paper mode m^max = C_hat) the
    # concurrent sets {v2,v3,v4} and {v5,v6} ask for more than M SMs.
    ex = load("worked_example.json")
    mmax = np.minimum(np.asarray(ex["par"]), np.asarray(ex["wcet"]))
    for S in ex["expect"]["greedy_overload"]:
        assert mmax[S].sum() > ex["M"]


# ---------------------------------------------------------------- hand cases

@pytest.mark.parametrize("case", load("hand_cases.json")["cases"], ids=lambda c: c["name"][:40])
def test_hand_case(case):
    src, dst = edges_of(case)
    n, M = case["n"], case["M"]
    d = oracle.division(n, src, dst, case["wcet"], case["par"], M)
    exp = case["expect"]
    assert d.groups == exp["groups"]
    s = oracle.bound(n, src, dst, case["wcet"], case["par"], M, case.get("r"), trace=True)
    assert (s.bound, s.cp, s.intf) == (exp["bound"], exp["cp"], exp["intf"])
    assert len(s.slots) == len(exp["slots"])
    for got, want in zip(s.slots, exp["slots"]):
        assert got.R == want["R"] and got.maxC == want["maxC"]
        assert [[p.node, p.kind, p.m, p.C, p.load] for p in got.parts] == want["parts"]
    if "extra_edges_contain" in exp:
        got_edges = {(a, ap, b, bp) for (_, a, ap, b, bp) in s.edges}
        for e in exp["extra_edges_contain"]:
            assert tuple(e) in got_edges
    if "worst_makespan_slot" in exp:
        for sl, want in zip(s.slots, exp["worst_makespan_slot"]):
            ms = [p.m for p in sl.parts]
            Cs = [p.C for p in sl.parts]
            assert oracle.worst_makespan(ms, Cs, [[] for _ in ms], M) == want


# ---------------------------------------------------------------- Eq. 1

def test_exec_time_eq1():
    # Eq. 1, t_min = 1: one wave for m <= M, ceil(m/M) waves above
    assert oracle.exec_time(10, 3, 8) == 4
    assert oracle.exec_time(10, 10, 8) == 2  # two waves of 10/10 -> 2 ticks
    assert oracle.exec_time(1, 5, 8) == 1  # never below t_min
    for load in range(1, 40):
        for m in range(1, 20):
            for M in (1, 4, 8, 16):
                waves = -(-m // M)
                assert oracle.exec_time(load, m, M) == max(1, -(-(waves * load) // m))


# ---------------------------------------------------------------- closed forms

def chain(n, wcet, par):
    src = np.arange(n - 1, dtype=np.int32)
    return src, src + 1


@pytest.mark.parametrize("seed", range(6))
def test_chain_closed_form(seed):
    # A chain has one node per group and nothing to launch beside it; each
    # node runs with m = min(r or p, p, C_hat, M), so the bound is the sum of
    # ceil(C_hat / m); with p = 1 it is the summed WCET.
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 30))
    M = int(rng.integers(1, 20))
    w = rng.integers(1, 200, n)
    p = rng.integers(1, 12, n)
    src, dst = chain(n, w, p)
    r = W.random_alloc(rng, p + 3, 300, zero_frac=0.3)  # some r above p: clamped
    for rr in (None, r):
        b, cp, intf = oracle.bound(n, src, dst, w, p, M, rr)
        mm = np.minimum(np.minimum(p, w), M)
        if rr is not None:
            mm = np.where(rr > 0, np.minimum(mm, rr), mm)
        assert b == int(sum(-(-w // mm)))
        assert intf == 0
    b1, _, _ = oracle.bound(n, src, dst, w, np.ones(n, np.int32), M)
    assert b1 == int(w.sum())


@pytest.mark.parametrize("seed", range(6))
def test_independent_set_closed_form(seed):
    # source -> k unit-parallelism nodes -> sink: groups are the middle nodes
    # in chunks of M by descending load; each chunk runs as long as its
    # largest load.
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(1, 25))
    M = int(rng.integers(1, 9))
    mid = rng.integers(1, 50, k)
    n = k + 2
    src = np.r_[np.zeros(k), np.arange(1, k + 1)].astype(np.int32)
    dst = np.r_[np.arange(1, k + 1), np.full(k, k + 1)].astype(np.int32)
    w = np.r_[[3], mid, [2]].astype(np.int64)
    p = np.ones(n, np.int32)
    b, _, _ = oracle.bound(n, src, dst, w, p, M)
    # Top order: descending W^anc = 3 + load, ties by smaller id (stable sort)
    order = sorted(range(k), key=lambda i: (-int(mid[i]), i))
    expect = 3 + sum(int(mid[order[q]]) for q in range(0, k, M)) + 2
    assert b == expect


@pytest.mark.parametrize("k,M,c", [(1, 8, 5), (2, 8, 3), (4, 8, 7), (8, 8, 7), (2, 16, 15), (4, 4, 1),
                                   (3, 8, 8), (5, 4, 9), (2, 6, 6)])
def test_equal_load_group_closed_form(k, M, c):
    # k | M nodes of equal load c < M, p >= c: Eq. 5 gives each m = min(c, M/k),
    # so the group needs max(1, ceil(k*c/M)) ticks.  With c >= M Rule 2 makes
    # each node a group of its own running on all M SMs: k * ceil(c/M) ticks.
    n = k + 2
    src = np.r_[np.zeros(k), np.arange(1, k + 1)].astype(np.int32)
    dst = np.r_[np.arange(1, k + 1), np.full(k, k + 1)].astype(np.int32)
    w = np.r_[[1], np.full(k, c), [1]].astype(np.int64)
    p = np.r_[[1], np.full(k, c + 5), [1]].astype(np.int32)
    b, cp, intf = oracle.bound(n, src, dst, w, p, M)
    if k == 1:
        assert b == 1 + -(-c // min(c, M)) + 1
    elif c < M:
        assert b == 1 + max(1, -(-(k * c) // M)) + 1
    else:
        assert b == 1 + k * -(-c // M) + 1
    assert intf == 0


# ---------------------------------------------------------------- invariants

def division_invariants(n, src, dst, w, p, M):
    d = oracle.division(n, src, dst, w, p, M)
    R = reachability(n, src, dst) if n <= 400 else None
    # Theta: join nodes, ascending W^anc, ties by smaller id
    indeg = np.bincount(dst, minlength=n)
    joins = sorted(np.nonzero(indeg >= 2)[0].tolist(), key=lambda v: (int(d.wanc[v]), v))
    assert d.theta == joins
    # Eq. 3: blocks
    assigned = np.full(n, -1)
    if R is not None:
        for k, t in enumerate(d.theta):
            anc = np.nonzero(R[t])[0]
            new = anc[assigned[anc] < 0]
            assigned[new] = k
        assigned[assigned < 0] = len(d.theta)
        assert assigned.tolist() == d.block.tolist()
    # in-block in-degree <= 1 (Section 3.1)
    inb = np.zeros(n, int)
    for s, t in zip(src, dst):
        if d.block[s] == d.block[t]:
            inb[t] += 1
    assert inb.max(initial=0) <= 1
    # groups partition V, |pi| <= M, Rule 2, antichains, linear extension
    flat = [v for g in d.groups for v in g]
    assert sorted(flat) == list(range(n))
    gof = np.empty(n, int)
    for j, g in enumerate(d.groups):
        gof[g] = j
        assert 1 <= len(g) <= M
        if len(g) > 1:
            assert all(min(int(p[v]), int(w[v])) < M for v in g)
        if R is not None:
            for a in g:
                for b in g:
                    assert not R[a, b]
        # members in Top order
        assert g == sorted(g, key=lambda v: (-int(d.wanc[v]), v))
    for s, t in zip(src, dst):
        assert gof[s] < gof[t]
    return d


def schedule_invariants(n, src, dst, w, p, M, r):
    s = oracle.bound(n, src, dst, w, p, M, r, trace=True)
    done_load = np.zeros(n, np.int64)
    finished = np.zeros(n, int)
    for sl in s.slots:
        segs = [q for q in sl.parts if q.kind == 2]
        assert len(segs) <= 1  # at most one segmentation per group (Section 4.1)
        for q in sl.parts:
            # m never exceeds the useful parallelism C_hat / t_min (Section 2.2)
            assert 1 <= q.m <= min(M, q.load)
            assert q.C == -(-q.load // q.m)
            assert q.C <= sl.maxC
            done_load[q.node] += q.load
            if q.kind != 2:
                finished[q.node] += 1
        if any(q.kind != 0 for q in sl.parts):
            assert sl.sum_m <= M  # launching only fills spare SMs
        if sl.nP:
            assert sl.R >= sl.maxC
            assert sl.R == sl.maxC or sl.sum_m > M
    assert done_load.tolist() == np.asarray(w).tolist()
    assert finished.tolist() == [1] * n
    assert s.bound == sum(sl.R for sl in s.slots) == s.cp + s.intf
    return s


@pytest.mark.parametrize("k", [1, 2, 3])
def test_invariants_on_workloads(k):
    wl = W.WORKLOADS[k]
    batch = W.generate_workload(k, count=40 if k < 3 else 6)
    rng = np.random.default_rng(k)
    for dgi in range(batch.num_dags):
        n, src, dst, w, p = batch.dag(dgi)
        division_invariants(n, src, dst, w, p, wl.num_cus)
        for rr in (None, W.random_alloc(rng, p, wl.num_cus), W.random_alloc(rng, p, wl.num_cus, 0.5)):
            schedule_invariants(n, src, dst, w, p, wl.num_cus, rr)


@pytest.mark.parametrize("seed", range(40))
def test_invariants_random_small(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 14))
    M = int(rng.integers(1, 10))
    n, src, dst, w, p = W.random_small_dag(rng, n, float(rng.uniform(0.1, 0.6)), 30, 12)
    division_invariants(n, src, dst, w, p, M)
    schedule_invariants(n, src, dst, w, p, M, W.random_alloc(rng, p, M, 0.4))


def longest_path(n, src, dst, weight):
    order = []
    indeg = np.bincount(dst, minlength=n).tolist()
    succ = [[] for _ in range(n)]
    for s, t in zip(src, dst):
        succ[s].append(t)
    q = [v for v in range(n) if indeg[v] == 0]
    while q:
        v = q.pop()
        order.append(v)
        for t in succ[v]:
            indeg[t] -= 1
            if indeg[t] == 0:
                q.append(t)
    dist = [0] * n
    for v in order:
        dist[v] += int(weight[v])
        for t in succ[v]:
            dist[t] = max(dist[t], dist[v])
    return max(dist, default=0)


@pytest.mark.parametrize("seed", range(30))
def test_lower_bounds(seed):
    # Any schedule in the block model needs at least the critical path at
    # full parallelism and the total work spread over M SMs.
    rng = np.random.default_rng(2000 + seed)
    n, src, dst, w, p = W.random_small_dag(rng, int(rng.integers(2, 40)), 0.15, 500, 40)
    M = int(rng.integers(1, 64))
    r = W.random_alloc(rng, p, M, 0.3)
    for rr in (None, r):
        b, _, _ = oracle.bound(n, src, dst, w, p, M, rr)
        fast = -(-w // np.minimum(np.minimum(p, w), M))
        assert b >= longest_path(n, src, dst, fast)
        assert b >= -(-int(w.sum()) // M)


# ---------------------------------------------------------------- brute force

def _check_safe(n, src, dst, w, p, M, r, early_seeds=3, para_mode=oracle.SPATIAL):
    s = oracle.bound(n, src, dst, w, p, M, r, trace=True, para_mode=para_mode)
    m, C, preds = oracle.schedule_parts(s, barriers=True)
    worst = oracle.worst_makespan(m, C, preds, M, node_limit=2_000_000)
    if worst < 0:
        return None
    assert worst <= s.bound
    if all(sl.sum_m <= M for sl in s.slots):
        # Lemma 1 is exact when every group fits: every dispatch order gives
        # the same makespan (the schedule is predictable)
        assert worst == s.bound
    for k in range(early_seeds):
        # early completion never exceeds the bound (sustainability)
        assert oracle.random_makespan(m, C, preds, M, seed=k, early=True) <= s.bound
        if all(sl.sum_m <= M for sl in s.slots):
            # one random dispatch at full durations of a predictable schedule
            # ends exactly at the bound
            assert oracle.random_makespan(m, C, preds, M, seed=k, early=False) == s.bound
    return worst


# Pins of the random dispatcher itself (values derived by hand in the block
# model: part x is m[x] blocks of C[x] ticks, one SM each, started only after
# every predecessor part has finished all its blocks).

def test_random_dispatch_chain_waits_for_predecessors():
    # a chain 3 -> 5 -> 2 ticks runs one part after another on any number of
    # SMs: 10 ticks for every seed (started together they would end at 5)
    for seed in range(10):
        assert oracle.random_makespan([1, 1, 1], [3, 5, 2], [[], [0], [1]], 4, seed, early=False) == 10


def test_random_dispatch_runs_blocks_in_waves():
    # five blocks of 3 ticks on 2 SMs: waves of 2, 2 and 1 blocks, 9 ticks
    for seed in range(10):
        assert oracle.random_makespan([5], [3], [[]], 2, seed, early=False) == 9


def test_random_dispatch_diamond():
    # a (1 block, 2 ticks) -> b (2 blocks, 3 ticks) and c (1 block, 4 ticks)
    # -> d (1 block, 1 tick).  On 3 SMs b and c start together at 2, c ends
    # at 6, d at 7.  On 2 SMs two of the three blocks start at 2: both of b
    # (c runs 5-9, d ends at 10) or one of b with c (b's second block runs
    # 5-8, d ends at 9); the worst order gives 10.
    m, C, preds = [1, 2, 1, 1], [2, 3, 4, 1], [[], [0], [0], [1, 2]]
    for seed in range(10):
        assert oracle.random_makespan(m, C, preds, 3, seed, early=False) == 7
    seen = {oracle.random_makespan(m, C, preds, 2, seed, early=False) for seed in range(60)}
    assert seen == {9, 10}
    assert oracle.worst_makespan(m, C, preds, 2) == 10
    assert oracle.worst_makespan(m, C, preds, 3) == 7


def test_random_early_completion_on_a_chain():
    # with early completion each block runs uniformly 1..C ticks: a chain of
    # four parts of 4 ticks ends between 4 and 16, after 10 ticks on average
    # (four parts of mean 2.5); started together it would end by 4.
    m, C, preds = [1, 1, 1, 1], [4, 4, 4, 4], [[], [0], [1], [2]]
    runs = [oracle.random_makespan(m, C, preds, 4, seed, early=True) for seed in range(400)]
    assert min(runs) >= 4 and max(runs) <= 16
    assert 9.5 <= float(np.mean(runs)) <= 10.5
    assert len(set(runs)) > 5
    # a single block of 1 tick cannot end early
    assert oracle.random_makespan([1], [1], [[]], 1, 0, early=True) == 1


def _worst_by_enumeration(m, C, preds, M):
    """Worst makespan of the block model by plain enumeration (independent
    of the oracle's search): at each instant the work-conserving dispatcher
    starts ready blocks while an SM is free; simultaneous starts are taken
    in nondecreasing part order."""
    n = len(m)
    best = 0

    def dfs(t, started, finished, running, minpart):
        nonlocal best
        ready_any = False
        if len(running) < M:
            for x in range(n):
                if started[x] >= m[x] or any(finished[u] < m[u] for u in preds[x]):
                    continue
                ready_any = True
                if x < minpart:
                    continue
                st = list(started)
                st[x] += 1
                dfs(t, st, finished, running + [(t + C[x], x)], x)
            if ready_any:
                return
        if not running:
            best = max(best, t)
            return
        tn = min(e for e, _ in running)
        fin = list(finished)
        for e, x in running:
            if e == tn:
                fin[x] += 1
        dfs(tn, started, fin, [(e, x) for e, x in running if e != tn], 0)

    dfs(0, [0] * n, [0] * n, [], 0)
    return best


@pytest.mark.parametrize("seed", range(30))
def test_dispatch_search_matches_enumeration(seed):
    # the oracle's search over dispatch orders, against a plain enumeration
    rng = np.random.default_rng(6300 + seed)
    n = int(rng.integers(1, 6))
    M = int(rng.integers(1, 4))
    m = rng.integers(1, 4, n).tolist()
    C = rng.integers(1, 4, n).tolist()
    preds = [[u for u in range(v) if rng.random() < 0.4] for v in range(n)]
    assert oracle.worst_makespan(m, C, preds, M) == _worst_by_enumeration(m, C, preds, M)


@pytest.mark.parametrize("seed", range(60))
def test_bound_safe_against_every_dispatch(seed):
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(2, 8))
    M = int(rng.integers(1, 7))
    n, src, dst, w, p = W.random_small_dag(rng, n, float(rng.uniform(0.15, 0.6)), 6, 6)
    r = W.random_alloc(rng, p, 255, zero_frac=float(rng.uniform(0, 1)))
    _check_safe(n, src, dst, w, p, M, r)
    _check_safe(n, src, dst, w, p, M, None)


@pytest.mark.parametrize("seed", range(60))
def test_temporal_bound_safe_against_every_dispatch(seed):
    # the temporal reading of the launching loop, its chain edges kept inside
    # each slot: no dispatch order ends after the bound
    rng = np.random.default_rng(3500 + seed)
    n = int(rng.integers(2, 8))
    M = int(rng.integers(1, 7))
    n, src, dst, w, p = W.random_small_dag(rng, n, float(rng.uniform(0.15, 0.6)), 6, 6)
    r = W.random_alloc(rng, p, 255, zero_frac=float(rng.uniform(0, 1)))
    _check_safe(n, src, dst, w, p, M, r, para_mode=oracle.TEMPORAL)
    _check_safe(n, src, dst, w, p, M, None, para_mode=oracle.TEMPORAL)


def test_temporal_hand_case():
    case = load("temporal_cases.json")["cases"][0]
    src, dst = edges_of(case)
    args = (case["n"], src, dst, case["wcet"], case["par"], case["M"], np.asarray(case["r"], np.uint8))
    assert list(oracle.bound(*args)) == case["expect"]["spatial"]
    assert list(oracle.bound(*args, para_mode=oracle.TEMPORAL)) == case["expect"]["temporal"]
    s = oracle.bound(*args, trace=True, para_mode=oracle.TEMPORAL)
    chain = sorted([a, b] for (_, a, ap, b, bp) in s.edges if a != 1 and b != 5)
    assert chain == case["expect"]["temporal_chain"]
    sl = s.slots[1]
    want = case["expect"]["temporal_slot2"]
    assert (sl.sum_m, sl.A, sl.maxC, sl.R) == (want["sum_m"], want["A"], want["maxC"], want["R"])


@pytest.mark.parametrize("seed", range(10))
def test_temporal_structure(seed):
    # the temporal reading: parallel parts use at most S SMs each, their C
    # add up to at most the group's maxC, and at most one of them is a
    # segment, the last; with M = 1 there are no spare SMs and both readings
    # agree
    rng = np.random.default_rng(3600 + seed)
    for k in (2, 3):
        batch = W.generate_workload(k, count=6, first=int(rng.integers(0, 1000)))
        M = W.WORKLOADS[k].num_cus
        for d in range(batch.num_dags):
            n, src, dst, w, p = batch.dag(d)
            r = W.random_alloc(rng, p, M, zero_frac=0.5)
            s = oracle.bound(n, src, dst, w, p, M, r, trace=True, para_mode=oracle.TEMPORAL)
            for sl in s.slots:
                members = [q for q in sl.parts if q.kind == 0]
                par = [q for q in sl.parts if q.kind != 0]
                if not par:
                    continue
                S = M - sum(q.m for q in members)
                assert all(q.m <= S for q in par)
                # each takes its target: the candidate byte, else m^max
                for q in par:
                    assert q.m <= p[q.node] and (r[q.node] == 0 or q.m <= r[q.node])
                    assert q.m == S or q.m == min(int(p[q.node]), int(r[q.node]) or int(p[q.node]), q.load) \
                        or q.kind == 2
                assert sum(q.C for q in par) <= sl.maxC
                assert all(q.kind == 1 for q in par[:-1])
            assert oracle.bound(n, src, dst, w, p, 1, r, para_mode=oracle.TEMPORAL) == \
                oracle.bound(n, src, dst, w, p, 1, r)


def test_bound_tight_on_oversubscribed_group():
    # 5 blocks of 2 ticks on 4 SMs: the list-scheduling response 2 + (10-2)/4
    # is reached by the dispatch that leaves one block for the end.
    case = load("hand_cases.json")["cases"][0]
    src, dst = edges_of(case)
    worst = _check_safe(case["n"], src, dst, case["wcet"], case["par"], case["M"], None)
    assert worst == case["expect"]["bound"]


# ---------------------------------------------------------------- comparison bounds (Section 5.2)

def test_baselines_worked_example():
    # Derived by hand from Section 5.2's definitions (the paper prints no
    # value for them on this DAG).  Paper mode p = C_hat and M = 6: every
    # m^max = C_hat <= 6, so Greedy and Greedy + unaware run each node at
    # m = C_hat with C = 1, and the sequential sum over 7 nodes is 7.
    # Graham_para: every unit node takes one tick, the longest path
    # v1 -> v3 -> v5 -> v7 has 4 nodes and vol = sum C_hat = 18, so the bound
    # is 4 + floor(14 / 6) = 6.
    ex = load("worked_example.json")
    src, dst = edges_of(ex)
    assert oracle.baselines(ex["n"], src, dst, ex["wcet"], ex["par"], ex["M"]) == (7, 7, 6)


def test_baselines_single_node():
    # C_hat = 100, p = 10, M = 4: Greedy takes m = 4, C = 25; unaware takes
    # m = 10, ceil(10 / 4) = 3 waves, C = ceil(3 * 100 / 10) = 30; Graham_para
    # has 10 unit nodes of 10 ticks: len 10, vol 100, 10 + floor(90 / 4) = 32.
    assert oracle.baselines(1, [], [], [100], [10], 4) == (25, 30, 32)
    # p above C_hat: with t_min = 1, m^max = C_hat = 3 unit nodes of one tick
    assert oracle.baselines(1, [], [], [3], [8], 4) == (1, 1, 1)
    # p = 1: one SM whatever M
    assert oracle.baselines(1, [], [], [17], [1], 8) == (17, 17, 17)
    # m^max above M in paper mode: C_hat = 9 = p on M = 4 SMs: Greedy m = 4,
    # C = 3; unaware m = 9 in 3 waves of one tick, C = 3; Graham: 9 unit
    # nodes of one tick, 1 + floor(8 / 4) = 3
    assert oracle.baselines(1, [], [], [9], [9], 4) == (3, 3, 3)


@pytest.mark.parametrize("seed", range(4))
def test_baselines_chain_and_antichain(seed):
    rng = np.random.default_rng(6100 + seed)
    # a chain with p = 1: every analysis runs the nodes one after another
    k = int(rng.integers(1, 12))
    w = rng.integers(1, 50, k).astype(np.int64)
    src = np.arange(k - 1, dtype=np.int32)
    dst = src + 1
    total = int(w.sum())
    assert oracle.baselines(k, src, dst, w, np.ones(k, np.int32), int(rng.integers(1, 9))) == (total,) * 3
    # n independent unit nodes on M SMs: the sequential analyses give n;
    # Graham's bound 1 + floor((n - 1) / M) = ceil(n / M), the optimum
    n = int(rng.integers(1, 40))
    M = int(rng.integers(1, 9))
    got = oracle.baselines(n, [], [], np.ones(n, np.int64), np.ones(n, np.int32), M)
    assert got == (n, n, -(-n // M))


@pytest.mark.parametrize("seed", range(40))
def test_graham_para_safe_against_every_dispatch(seed):
    # Graham's theorem: no work-conserving dispatch of the expanded DAG (node
    # v as m^max blocks of ceil(C_hat / m^max) ticks, Section 2.2's block
    # model) ends after the bound; checked over every dispatch by brute
    # force.  Greedy + unaware never beats Greedy (more waves, never fewer).
    rng = np.random.default_rng(6200 + seed)
    n = int(rng.integers(1, 7))
    M = int(rng.integers(1, 5))
    n, src, dst, w, p = W.random_small_dag(rng, n, float(rng.uniform(0.2, 0.6)), 5, 3)
    greedy, unaware, graham = oracle.baselines(n, src, dst, w, p, M)
    assert unaware >= greedy
    mm = np.minimum(p, w)
    C = -(-w // mm)
    preds = [[] for _ in range(n)]
    for a, b in zip(src, dst):
        preds[int(b)].append(int(a))
    worst = oracle.worst_makespan(mm, C, preds, M, node_limit=2_000_000)
    if worst >= 0:
        assert worst <= graham
    for k in range(3):
        assert oracle.random_makespan(mm, C, preds, M, seed=k, early=False) <= graham
    # the bound is at least the longest path of the expanded DAG
    L = np.zeros(n, np.int64)
    R = reachability(n, src, dst)
    for v in sorted(range(n), key=lambda v: R[v].sum()):
        L[v] = C[v] + max([L[u] for u in preds[v]], default=0)
    assert graham >= L.max()


# ---------------------------------------------------------------- input checks

def test_rejects_bad_inputs():
    w = [1, 1, 1]
    p = [1, 1, 1]
    with pytest.raises(oracle.OracleError) as e:
        oracle.bound(3, [0, 1, 2], [1, 2, 0], w, p, 4)
    assert e.value.code == oracle.E_CYCLE
    with pytest.raises(oracle.OracleError) as e:
        oracle.bound(3, [0, 0], [1, 1], w, p, 4)
    assert e.value.code == oracle.E_DUP_EDGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.bound(3, [1], [1], w, p, 4)
    assert e.value.code == oracle.E_CYCLE
    with pytest.raises(oracle.OracleError) as e:
        oracle.bound(3, [0], [3], w, p, 4)
    assert e.value.code == oracle.E_RANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.bound(3, [0], [1], [1, 0, 1], p, 4)
    assert e.value.code == oracle.E_RANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.bound(3, [0], [1], w, [1, 1, 0], 4)
    assert e.value.code == oracle.E_RANGE
    assert oracle.bound(0, [], [], [], [], 4) == (0, 0, 0)


# ---------------------------------------------------------------- conditional DAGs
# (the paper's future work): the schedule of the DAG with every branch
# present; in one realization only the chosen branches' nodes execute, and
# each slot's response is Lemma 1 over its executed parts.

def test_conditional_hand_cases():
    # s -> a | b -> t with a and b the two branches of one conditional.
    #   M = 4, loads (1, 8, 3, 1), p = (1, 4, 1, 1), candidate byte 2 for a.
    #   Groups {s}, {a} (Rule 2: m^max(a) = 4 >= M), {b}, {t}.  Slot 2: a runs
    #   on 2 SMs (C = 4), S = 2, and b is launched beside it whole (m = 1,
    #   C = 3 <= maxC); slot 3 is then empty.  Full bound 1 + 4 + 0 + 1 = 6.
    #   Realization "a": slot 2 holds a (4): 6.  Realization "b": slot 2
    #   holds only b's parallel part (3): 1 + 3 + 0 + 1 = 5.
    src, dst = np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3])
    w, p = np.array([1, 8, 3, 1]), np.array([1, 4, 1, 1])
    r = np.array([0, 2, 0, 0], np.uint8)
    cond, br = [-1, 0, 0, -1], [0, 0, 1, 0]
    assert oracle.bound(4, src, dst, w, p, 4, r)[0] == 6
    masks = oracle.realizations(cond, br)
    assert [m.tolist() for m in masks] == [[1, 1, 0, 1], [1, 0, 1, 1]]
    assert oracle.cond_bound(4, src, dst, w, p, 4, r, masks[0]) == (6, 6, 0)
    assert oracle.cond_bound(4, src, dst, w, p, 4, r, masks[1]) == (5, 5, 0)
    assert oracle.cond_bound_max(4, src, dst, w, p, 4, r, cond, br) == (6, 0)
    # with the paper's rule a runs on all 4 SMs (C = 2), b has its own slot
    # (m = 1, C = 3): full 1 + 2 + 3 + 1 = 7; each realization skips one of
    # the two middle slots: 1 + 2 + 0 + 1 = 4 and 1 + 0 + 3 + 1 = 5.
    assert oracle.bound(4, src, dst, w, p, 4)[0] == 7
    assert oracle.cond_bound(4, src, dst, w, p, 4, None, masks[0])[0] == 4
    assert oracle.cond_bound(4, src, dst, w, p, 4, None, masks[1])[0] == 5
    assert oracle.cond_bound_max(4, src, dst, w, p, 4, None, cond, br) == (5, 1)


def test_conditional_oversubscribed_slot_that_fits_once_branches_are_skipped():
    # M = 3; s -> x, y -> t, x and y the two branches; loads (1, 6, 6, 1),
    # p = (1, 2, 2, 1), candidate bytes 2 for x and y.  One group {x, y}
    # (m^max = 2 < M, no Rule 2): m = 2 + 2 = 4 > 3, C = 3 each, A = 12, so
    # the slot takes 3 + floor((12 - 3) / 3) = 6; full bound 1 + 6 + 1 = 8.
    # With one branch the slot holds 2 SMs for 3 ticks: 1 + 3 + 1 = 5.
    src, dst = np.array([0, 0, 1, 2]), np.array([1, 2, 3, 3])
    w, p = np.array([1, 6, 6, 1]), np.array([1, 2, 2, 1])
    r = np.array([0, 2, 2, 0], np.uint8)
    assert oracle.bound(4, src, dst, w, p, 3, r) == (8, 5, 3)
    for m in oracle.realizations([-1, 0, 0, -1], [0, 0, 1, 0]):
        assert oracle.cond_bound(4, src, dst, w, p, 3, r, m) == (5, 5, 0)


def test_conditional_realization_order():
    # two conditionals of 2 and 3 branches: 6 realizations, conditional 0
    # the least significant digit
    cond, br = [0, 0, 1, 1, 1, -1], [0, 1, 0, 1, 2, 0]
    masks = [m.tolist() for m in oracle.realizations(cond, br)]
    assert masks == [[1, 0, 1, 0, 0, 1], [0, 1, 1, 0, 0, 1], [1, 0, 0, 1, 0, 1],
                     [0, 1, 0, 1, 0, 1], [1, 0, 0, 0, 1, 1], [0, 1, 0, 0, 1, 1]]
    assert [m.tolist() for m in oracle.realizations([-1, -1], [0, 0])] == [[1, 1]]


@pytest.mark.parametrize("seed", range(20))
def test_conditional_every_node_executed_is_the_bound(seed):
    rng = np.random.default_rng(5100 + seed)
    n, src, dst, w, p = W.random_small_dag(rng, int(rng.integers(2, 40)), 0.15, 500, 40)
    M = int(rng.integers(1, 64))
    r = W.random_alloc(rng, p, M, 0.3)
    for rr in (None, r):
        assert oracle.cond_bound(n, src, dst, w, p, M, rr, np.ones(n, np.uint8)) == \
            oracle.bound(n, src, dst, w, p, M, rr)


@pytest.mark.parametrize("seed", range(20))
def test_conditional_bound_is_monotone_in_the_executed_set(seed):
    rng = np.random.default_rng(5200 + seed)
    n, src, dst, w, p = W.random_small_dag(rng, int(rng.integers(2, 30)), 0.2, 300, 30)
    M = int(rng.integers(1, 32))
    r = W.random_alloc(rng, p, M, 0.3)
    full = oracle.bound(n, src, dst, w, p, M, r)[0]
    for _ in range(5):
        big = (rng.random(n) < 0.7).astype(np.uint8)
        small = big & (rng.random(n) < 0.6).astype(np.uint8)
        bs = oracle.cond_bound(n, src, dst, w, p, M, r, small)[0]
        bb = oracle.cond_bound(n, src, dst, w, p, M, r, big)[0]
        assert 0 <= bs <= bb <= full
    assert oracle.cond_bound(n, src, dst, w, p, M, r, np.zeros(n, np.uint8))[0] == 0


def _executed_parts(sched, xm):
    """Part DAG of the executed parts of a traced schedule: one barrier
    between consecutive slots that keep a part (empty slots pass at once)."""
    parts = [q for s in sched.slots for q in s.parts if xm[q.node]]
    m = [q.m for q in parts]
    C = [q.C for q in parts]
    by_slot = {}
    for i, q in enumerate(parts):
        by_slot.setdefault(q.slot, []).append(i)
    preds = [[] for _ in parts]
    slots = sorted(by_slot)
    for a, b in zip(slots, slots[1:]):
        for x in by_slot[b]:
            preds[x] = list(by_slot[a])
    return m, C, preds, by_slot


@pytest.mark.parametrize("seed", range(40))
def test_conditional_bound_safe_against_every_dispatch(seed):
    # every work-conserving dispatch of the executed blocks (one barrier per
    # slot boundary) ends by the realization's bound, and exactly at it when
    # no slot's executed parts oversubscribe M
    rng = np.random.default_rng(5300 + seed)
    n, src, dst, w, p = W.random_small_dag(rng, int(rng.integers(3, 8)), 0.3, 6, 4)
    M = int(rng.integers(1, 6))
    r = W.random_alloc(rng, p, M, 0.4)
    cond = np.where(rng.random(n) < 0.6, rng.integers(0, 2, n), -1)
    br = rng.integers(0, 2, n)
    s = oracle.bound(n, src, dst, w, p, M, r, trace=True)
    checked = 0
    for xm in oracle.realizations(cond, br):
        b = oracle.cond_bound(n, src, dst, w, p, M, r, xm)[0]
        m, C, preds, by_slot = _executed_parts(s, xm)
        worst = oracle.worst_makespan(m, C, preds, M, node_limit=2_000_000) if m else 0
        if worst < 0:
            continue
        assert worst <= b
        if all(sum(m[i] for i in idx) <= M for idx in by_slot.values()):
            assert worst == b
        checked += 1
    assert checked > 0
