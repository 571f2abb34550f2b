"""CPU oracle for the DAG makespan bound -- TEST INFRASTRUCTURE ONLY.

Python bindings of ``oracle.c`` (plain C, int64), the slow step-by-step
reference the GPU library is checked against.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the
library never does.

The C code follows the paper's Algorithm 1 (sub-graph division), Algorithm 2
(scheduling) and Lemma 1 / Theorem 1 (the bound); its header lists the
readings taken where the paper is informal.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DAGBOUND_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_CYCLE, E_RANGE, E_DUP_EDGE, E_OOM, E_OVERFLOW = 0, -1, -2, -3, -4, -5, -8

_lib: Optional[ctypes.CDLL] = None


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-Wall", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_exec_time.restype = ctypes.c_int64
        lib.oracle_exec_time.argtypes = [ctypes.c_int64] * 3
        lib.oracle_division.restype = ctypes.c_int
        lib.oracle_division.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int] + [P] * 7
        lib.oracle_bound.restype = ctypes.c_int
        lib.oracle_bound.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int, P, P, P,
                                     ctypes.c_int64, P, ctypes.c_int]
        lib.oracle_bounds_dag.restype = ctypes.c_int
        lib.oracle_bounds_dag.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int,
                                          ctypes.c_int, P, P, P, P, ctypes.c_int]
        lib.oracle_baselines.restype = ctypes.c_int
        lib.oracle_baselines.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int, P]
        lib.oracle_worst_makespan.restype = ctypes.c_int64
        lib.oracle_worst_makespan.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int64]
        lib.oracle_cond_bound.restype = ctypes.c_int
        lib.oracle_cond_bound.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int, P, P, P]
        lib.oracle_random_makespan.restype = ctypes.c_int64
        lib.oracle_random_makespan.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P,
                                               ctypes.c_uint64, ctypes.c_int]
        _lib = lib
    return _lib


def _arr(x, dt):
    a = np.ascontiguousarray(np.asarray(x, dtype=dt))
    return a, (a.ctypes.data if a.size else None)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}")
        self.code = code


def exec_time(load: int, m: int, M: int) -> int:
    """Eq. 1 with t_min = 1 in integer ticks."""
    return int(_load().oracle_exec_time(load, m, M))


@dataclass
class Division:
    wanc: np.ndarray      # Eq. 2, per node
    theta: List[int]      # join nodes in Theta order
    block: np.ndarray     # block index per node (len(theta) = residual)
    groups: List[List[int]]  # Pi, members of each group in Top order


def division(n, src, dst, wcet, par, M) -> Division:
    """Sub-graph division (Algorithm 1) of one DAG."""
    lib = _load()
    s, sp = _arr(src, np.int32)
    t, tp = _arr(dst, np.int32)
    w, wp = _arr(wcet, np.int64)
    p, pp = _arr(par, np.int32)
    wanc = np.zeros(max(n, 1), np.int64)
    theta = np.zeros(max(n, 1), np.int32)
    block = np.zeros(max(n, 1), np.int32)
    gof = np.zeros(max(n, 1), np.int32)
    gmem = np.zeros(max(n, 1), np.int32)
    goff = np.zeros(n + 1, np.int32)
    counts = np.zeros(2, np.int32)
    rc = lib.oracle_division(n, len(s), sp, tp, wp, pp, M, wanc.ctypes.data, theta.ctypes.data,
                             block.ctypes.data, gof.ctypes.data, gmem.ctypes.data,
                             goff.ctypes.data, counts.ctypes.data)
    if rc != OK:
        raise OracleError(rc)
    nt, ng = int(counts[0]), int(counts[1])
    groups = [list(map(int, gmem[goff[j]:goff[j + 1]])) for j in range(ng)]
    return Division(wanc[:n].copy(), list(map(int, theta[:nt])), block[:n].copy(), groups)


@dataclass
class Part:
    slot: int
    node: int
    part: int
    kind: int  # 0 member, 1 parallel node launched whole, 2 parallel segment
    m: int
    C: int
    load: int


@dataclass
class Slot:
    j: int
    nP: int
    maxC: int
    sum_m: int
    A: int
    R: int
    vR: int
    parts: List[Part]


@dataclass
class Schedule:
    bound: int
    cp: int
    intf: int
    slots: List[Slot]
    edges: List[Tuple[int, int, int, int, int]]  # (slot, from node, from part, to node, to part)


SPATIAL, TEMPORAL = 0, 1


def bound(n, src, dst, wcet, par, M, r=None, trace: bool = False, para_mode: int = SPATIAL):
    """Bound of one DAG under candidate r (None: the paper's rule for all
    nodes).  Returns (bound, cp, intf), or a Schedule when trace=True.
    para_mode: SPATIAL (the launching loop's spare SMs shrink per node) or
    TEMPORAL (the launched nodes run one after another on the spare SMs
    within the slot's time)."""
    lib = _load()
    s, sp = _arr(src, np.int32)
    t, tp = _arr(dst, np.int32)
    w, wp = _arr(wcet, np.int64)
    p, pp = _arr(par, np.int32)
    if r is not None:
        rr, rp = _arr(r, np.uint8)
    else:
        rp = None
    out = np.zeros(3, np.int64)
    cap = 0
    buf = None
    ntr = np.zeros(1, np.int64)
    if trace:
        cap = 64 * (n + 4) * (n + 4) + 1024
        buf = np.zeros(cap * 8, np.int64)
    rc = lib.oracle_bound(n, len(s), sp, tp, wp, pp, M, rp, out.ctypes.data,
                          buf.ctypes.data if buf is not None else None, cap, ntr.ctypes.data, int(para_mode))
    if rc != OK:
        raise OracleError(rc)
    if not trace:
        return int(out[0]), int(out[1]), int(out[2])
    nrec = int(ntr[0])
    if nrec > cap:
        raise RuntimeError("trace buffer too small")
    recs = buf[: nrec * 8].reshape(nrec, 8)
    slots: List[Slot] = []
    pending: List[Part] = []
    edges = []
    for rec in recs:
        tag = int(rec[0])
        if tag == 2:
            pending.append(Part(int(rec[1]), int(rec[2]), int(rec[3]), int(rec[4]), int(rec[5]),
                                int(rec[6]), int(rec[7])))
        elif tag == 1:
            slots.append(Slot(int(rec[1]), int(rec[2]), int(rec[3]), int(rec[4]), int(rec[5]),
                              int(rec[6]), int(rec[7]), pending))
            pending = []
        elif tag == 3:
            edges.append((int(rec[1]), int(rec[2]), int(rec[3]), int(rec[4]), int(rec[5])))
    return Schedule(int(out[0]), int(out[1]), int(out[2]), slots, edges)


def cond_bound(n, src, dst, wcet, par, M, r, xmask) -> Tuple[int, int, int]:
    """Bound of one realization of a conditional DAG (spatial reading): the
    schedule of the DAG with every branch present, each slot's response
    from the parts of the nodes with xmask[v] != 0 (oracle_cond_bound).
    Returns (bound, cp, intf)."""
    lib = _load()
    s, sp = _arr(src, np.int32)
    t, tp = _arr(dst, np.int32)
    w, wp = _arr(wcet, np.int64)
    p, pp = _arr(par, np.int32)
    rp = _arr(r, np.uint8)[1] if r is not None else None
    x, xp = _arr(xmask, np.uint8)
    out = np.zeros(3, np.int64)
    rc = lib.oracle_cond_bound(n, len(s), sp, tp, wp, pp, M, rp, xp, out.ctypes.data)
    if rc != OK:
        raise OracleError(rc)
    return int(out[0]), int(out[1]), int(out[2])


def realizations(cond_of, branch_of) -> List[np.ndarray]:
    """Every realization of a conditional DAG as an execution mask, in
    mixed-radix order: node v with cond_of[v] = q >= 0 runs only in the
    realizations whose digit q equals branch_of[v] (conditional 0 is the
    least significant digit, each conditional has max branch + 1
    branches); nodes with cond_of[v] < 0 always run."""
    cond_of = np.asarray(cond_of, np.int64)
    branch_of = np.asarray(branch_of, np.int64)
    nc = int(cond_of.max()) + 1 if len(cond_of) and cond_of.max() >= 0 else 0
    nb = [int(branch_of[cond_of == q].max()) + 1 if np.any(cond_of == q) else 1 for q in range(nc)]
    total = int(np.prod(nb)) if nc else 1
    out = []
    for rho in range(total):
        digit, rest = [], rho
        for q in range(nc):
            digit.append(rest % nb[q])
            rest //= nb[q]
        m = np.ones(len(cond_of), np.uint8)
        for v in range(len(cond_of)):
            if cond_of[v] >= 0 and branch_of[v] != digit[cond_of[v]]:
                m[v] = 0
        out.append(m)
    return out


def cond_bound_max(n, src, dst, wcet, par, M, r, cond_of, branch_of) -> Tuple[int, int]:
    """The conditional DAG's bound: the largest realization bound, and the
    first realization (mixed-radix index) that reaches it."""
    best, arg = -1, -1
    for rho, m in enumerate(realizations(cond_of, branch_of)):
        b = cond_bound(n, src, dst, wcet, par, M, r, m)[0]
        if b > best:
            best, arg = b, rho
    return best, arg


def bounds_dag(n, src, dst, wcet, par, M, K, alloc_dag,
               para_mode: int = SPATIAL) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """All K candidates of one DAG; alloc_dag holds K*n bytes ((c, v) at
    c*n + v), candidate 0's bytes ignored."""
    lib = _load()
    s, sp = _arr(src, np.int32)
    t, tp = _arr(dst, np.int32)
    w, wp = _arr(wcet, np.int64)
    p, pp = _arr(par, np.int32)
    a, ap = _arr(alloc_dag, np.uint8)
    b = np.zeros(K, np.int64)
    cp = np.zeros(K, np.int64)
    it = np.zeros(K, np.int64)
    rc = lib.oracle_bounds_dag(n, len(s), sp, tp, wp, pp, M, K, ap, b.ctypes.data,
                               cp.ctypes.data, it.ctypes.data, int(para_mode))
    if rc != OK:
        raise OracleError(rc)
    return b, cp, it


def bounds_batch(batch, M: int, K: int, alloc: np.ndarray, dags: Optional[Sequence[int]] = None,
                 threads: int = 1, para_mode: int = SPATIAL):
    """Bounds of DAGs `dags` (default: all) of a workloads.DagBatch with the
    explicit candidate bytes `alloc` (layout K*node_off[d] + c*N_d + v).
    Returns (bounds, cp, intf), each [len(dags), K]."""
    idx = list(range(batch.num_dags)) if dags is None else list(dags)
    out_b = np.zeros((len(idx), K), np.int64)
    out_c = np.zeros((len(idx), K), np.int64)
    out_i = np.zeros((len(idx), K), np.int64)

    def one(i):
        d = idx[i]
        n, s, t, w, p = batch.dag(d)
        n0 = int(batch.node_off[d])
        a = alloc[K * n0: K * n0 + K * n]
        out_b[i], out_c[i], out_i[i] = bounds_dag(n, s, t, w, p, M, K, a, para_mode)

    if threads <= 1:
        for i in range(len(idx)):
            one(i)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(idx))))
    return out_b, out_c, out_i


def baselines(n, src, dst, wcet, par, M) -> Tuple[int, int, int]:
    """The comparison bounds of Section 5.2 for one DAG: (Greedy,
    Greedy + unaware, Graham_para)."""
    lib = _load()
    s, sp = _arr(src, np.int32)
    t, tp = _arr(dst, np.int32)
    w, wp = _arr(wcet, np.int64)
    p, pp = _arr(par, np.int32)
    out = np.zeros(3, np.int64)
    rc = lib.oracle_baselines(n, len(s), sp, tp, wp, pp, M, out.ctypes.data)
    if rc != OK:
        raise OracleError(rc)
    return int(out[0]), int(out[1]), int(out[2])


def baselines_batch(batch, M: int, dags: Optional[Sequence[int]] = None, threads: int = 1) -> np.ndarray:
    """Comparison bounds of DAGs `dags` (default: all) of a workloads.DagBatch,
    as an array [len(dags), 3] of (Greedy, Greedy + unaware, Graham_para)."""
    idx = list(range(batch.num_dags)) if dags is None else list(dags)
    out = np.zeros((len(idx), 3), np.int64)

    def one(i):
        n, s, t, w, p = batch.dag(idx[i])
        out[i] = baselines(n, s, t, w, p, M)

    if threads <= 1:
        for i in range(len(idx)):
            one(i)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(idx))))
    return out


def worst_makespan(parts_m, parts_C, preds: Sequence[Sequence[int]], M: int, node_limit: int = 0) -> int:
    """Worst makespan over every work-conserving dispatch of blocks (each part
    x is m[x] blocks of C[x] ticks; preds[x] lists parts that must finish
    first).  -1 if node_limit was hit."""
    lib = _load()
    m, mp = _arr(parts_m, np.int64)
    C, Cp = _arr(parts_C, np.int64)
    off = np.zeros(len(preds) + 1, np.int32)
    flat = []
    for i, ps in enumerate(preds):
        flat.extend(ps)
        off[i + 1] = len(flat)
    fl, flp = _arr(flat if flat else [0], np.int32)
    return int(lib.oracle_worst_makespan(len(preds), M, mp, Cp, off.ctypes.data, flp, node_limit))


def random_makespan(parts_m, parts_C, preds, M: int, seed: int, early: bool) -> int:
    lib = _load()
    m, mp = _arr(parts_m, np.int64)
    C, Cp = _arr(parts_C, np.int64)
    off = np.zeros(len(preds) + 1, np.int32)
    flat = []
    for i, ps in enumerate(preds):
        flat.extend(ps)
        off[i + 1] = len(flat)
    fl, flp = _arr(flat if flat else [0], np.int32)
    return int(lib.oracle_random_makespan(len(preds), M, mp, Cp, off.ctypes.data, flp,
                                          ctypes.c_uint64(seed), int(early)))


def schedule_parts(sched: Schedule, barriers: bool = True, src=None, dst=None):
    """Turn a traced schedule into the part DAG of the block model.

    With barriers, every part of slot j waits for every part of slot j-1
    (one barrier per slot boundary), and the recorded dependencies inside a
    slot (the chain of the temporal reading) are kept.  Without them, the parts keep only the
    original edges (mapped to the first/last part of each node), the chain
    between consecutive parts of a segmented node and the extra dependencies
    of Section 4.1.  Returns (m, C, preds)."""
    parts = [p for s in sched.slots for p in s.parts]
    index = {(p.node, p.part): i for i, p in enumerate(parts)}
    m = [p.m for p in parts]
    C = [p.C for p in parts]
    preds: List[set] = [set() for _ in parts]
    if barriers:
        by_slot = {}
        for i, p in enumerate(parts):
            by_slot.setdefault(p.slot, []).append(i)
        slots = sorted(by_slot)
        for a, b in zip(slots, slots[1:]):
            for x in by_slot[b]:
                preds[x].update(by_slot[a])
        # dependencies inside one slot: the chain of the temporal reading
        for (_, a, ap, b, bp) in sched.edges:
            if (a, ap) in index and (b, bp) in index:
                ia, ib = index[(a, ap)], index[(b, bp)]
                if parts[ia].slot == parts[ib].slot:
                    preds[ib].add(ia)
    else:
        last = {}
        first = {}
        for i, p in enumerate(parts):
            first.setdefault(p.node, i)
            last[p.node] = i
        for i, p in enumerate(parts):
            if p.part > 0:
                preds[i].add(index[(p.node, p.part - 1)])
        for u, v in zip(src, dst):
            preds[first[int(v)]].add(last[int(u)])
        for (_, a, ap, b, bp) in sched.edges:
            if (a, ap) in index and (b, bp) in index:
                preds[index[(b, bp)]].add(index[(a, ap)])
    return m, C, [sorted(s) for s in preds]
