"""Seeded synthetic DAG-task workloads (input generation only).

This module draws random DAG tasks and candidate allocations.  It contains
none of the bound's arithmetic; the CPU oracle and the GPU library both take
its arrays as inputs.  The generator itself is C (``gen.c``), built into
``libwl.so`` next to this file.

Workload shapes follow the task model of the paper (DAG ``G=(V,E)``, per-node
load in integer ticks with ``t_min = 1`` and a maximum parallelism, ``M``
compute units; Section 2).  One source and one sink node are added to every
generated DAG (the paper assumes a single source and sink, Section 2.1).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwl.so")
GPU_LIB_PATH = os.path.join(_HERE, "libwlgpu.so")
BASE_SEED = 0x2602208260000000


class _Spec(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int32),
        ("nmin", ctypes.c_int32),
        ("nmax", ctypes.c_int32),
        ("n_logu", ctypes.c_int32),
        ("width_max", ctypes.c_int32),
        ("skip_min", ctypes.c_int32),
        ("skip_max", ctypes.c_int32),
        ("wcet_kind", ctypes.c_int32),
        ("pmin", ctypes.c_int32),
        ("pmax", ctypes.c_int32),
        ("add_src_sink", ctypes.c_int32),
        ("permute_ids", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("p_er", ctypes.c_double),
        ("p_adj", ctypes.c_double),
        ("p_skip", ctypes.c_double),
        ("wmin", ctypes.c_int64),
        ("wmax", ctypes.c_int64),
        ("mu", ctypes.c_double),
        ("sigma", ctypes.c_double),
    ]


SHAPE_ER, SHAPE_LAYERED, SHAPE_MIXED = 0, 1, 2
WCET_UNIFORM, WCET_LOGUNIFORM, WCET_LOGNORMAL = 0, 1, 2


@dataclasses.dataclass(frozen=True)
class Spec:
    """Shape and distributions of one synthetic workload."""

    shape: int
    nmin: int
    nmax: int
    n_logu: bool = False
    p_er: float = 0.0
    width_max: int = 1
    p_adj: float = 0.0
    p_skip: float = 0.0
    skip_min: int = 2
    skip_max: int = 8
    wcet_kind: int = WCET_UNIFORM
    wmin: int = 1
    wmax: int = 100
    mu: float = 0.0
    sigma: float = 1.0
    pmin: int = 1
    pmax: int = 8
    add_src_sink: bool = True
    permute_ids: bool = True

    def to_c(self) -> _Spec:
        return _Spec(
            shape=self.shape, nmin=self.nmin, nmax=self.nmax, n_logu=int(self.n_logu),
            width_max=self.width_max, skip_min=self.skip_min, skip_max=self.skip_max,
            wcet_kind=self.wcet_kind, pmin=self.pmin, pmax=self.pmax,
            add_src_sink=int(self.add_src_sink), permute_ids=int(self.permute_ids), pad0=0,
            p_er=self.p_er, p_adj=self.p_adj, p_skip=self.p_skip, wmin=self.wmin,
            wmax=self.wmax, mu=self.mu, sigma=self.sigma,
        )


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named workload: DAG spec, batch size, compute units and candidates."""

    name: str
    spec: Spec
    num_dags: int
    num_cus: int
    K: int
    seed: int


# The five synthetic workloads of the benchmark plan.
WORKLOADS: Dict[int, Workload] = {
    1: Workload(
        "small-er: 1000 DAGs, ER p=0.2, 10-20 nodes, WCET 1-100, par 1-8, M=8, K=16",
        Spec(SHAPE_ER, 10, 20, p_er=0.2, wcet_kind=WCET_UNIFORM, wmin=1, wmax=100, pmin=1, pmax=8),
        1000, 8, 16, BASE_SEED + 1),
    2: Workload(
        "batched-layered: 100k DAGs, layered width 1-16 p=0.3, 20-100 nodes, WCET 1-1000, par 1-32, M=256, K=64",
        Spec(SHAPE_LAYERED, 20, 100, width_max=16, p_adj=0.3, wcet_kind=WCET_UNIFORM, wmin=1,
             wmax=1000, pmin=1, pmax=32),
        100_000, 256, 64, BASE_SEED + 2),
    3: Workload(
        "persistent-mixed: 1M DAGs, ER p=0.05 / layered width 1-32 p=0.3, 50-500 nodes log-uniform, WCET log-uniform 1-1e5, par 1-64, M=256, K=256",
        Spec(SHAPE_MIXED, 50, 500, n_logu=True, p_er=0.05, width_max=32, p_adj=0.3,
             wcet_kind=WCET_LOGUNIFORM, wmin=1, wmax=100_000, pmin=1, pmax=64),
        1_000_000, 256, 256, BASE_SEED + 3),
    4: Workload(
        "learned-proposal: 100k held-out DAGs of the persistent-mixed shape, K=4096 seeded",
        Spec(SHAPE_MIXED, 50, 500, n_logu=True, p_er=0.05, width_max=32, p_adj=0.3,
             wcet_kind=WCET_LOGUNIFORM, wmin=1, wmax=100_000, pmin=1, pmax=64),
        100_000, 256, 4096, BASE_SEED + 4),
    5: Workload(
        "large-compiler: 10k DAGs, layered width 1-64 p=0.3 + skip 2-8 layers p=0.02, 1000-5000 nodes, lognormal(3,1.5) WCET, par 1-128, M=256, K=16384 seeded",
        Spec(SHAPE_LAYERED, 1000, 5000, width_max=64, p_adj=0.3, p_skip=0.02, skip_min=2,
             skip_max=8, wcet_kind=WCET_LOGNORMAL, mu=3.0, sigma=1.5, pmin=1, pmax=128),
        10_000, 256, 16384, BASE_SEED + 5),
}


@dataclasses.dataclass
class DagBatch:
    """Host arrays of a DAG batch in the library's ingest layout."""

    node_off: np.ndarray  # int64 [D+1]
    edge_off: np.ndarray  # int64 [D+1]
    src: np.ndarray  # int32 [E]  DAG-local ids
    dst: np.ndarray  # int32 [E]
    wcet: np.ndarray  # int64 [N]
    par: np.ndarray  # int32 [N]

    @property
    def num_dags(self) -> int:
        return int(self.node_off.shape[0] - 1)

    def dag(self, d: int):
        """Return (n, src, dst, wcet, par) of DAG d (views)."""
        n0, n1 = int(self.node_off[d]), int(self.node_off[d + 1])
        e0, e1 = int(self.edge_off[d]), int(self.edge_off[d + 1])
        return n1 - n0, self.src[e0:e1], self.dst[e0:e1], self.wcet[n0:n1], self.par[n0:n1]

    def subset(self, idx) -> "DagBatch":
        """A new batch holding DAGs idx (in that order)."""
        parts = [self.dag(int(d)) for d in idx]
        return from_dags(parts)


_lib: Optional[ctypes.CDLL] = None


def build(force: bool = False, gpu: bool = True) -> str:
    """Compile gen.c into libwl.so (gcc, OpenMP) and, with `gpu`, the
    device-side byte generator gen_gpu.hip into libwlgpu.so (hipcc, gfx950)."""
    import subprocess

    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    gsrc = os.path.join(_HERE, "gen_gpu.hip")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if gpu and os.path.exists(hipcc) and (force or not os.path.exists(GPU_LIB_PATH)
                                          or os.path.getmtime(GPU_LIB_PATH) < os.path.getmtime(gsrc)):
        tmp = GPU_LIB_PATH + ".tmp"
        arch = os.environ.get("DAGBOUND_OFFLOAD_ARCH", "gfx950")
        subprocess.check_call([hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={arch}",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, gsrc])
        os.replace(tmp, GPU_LIB_PATH)
    return LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.wl_batch_generate.restype = ctypes.c_void_p
        lib.wl_batch_generate.argtypes = [ctypes.POINTER(_Spec), ctypes.c_uint64, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int32]
        lib.wl_batch_nodes.restype = ctypes.c_int64
        lib.wl_batch_nodes.argtypes = [ctypes.c_void_p]
        lib.wl_batch_edges.restype = ctypes.c_int64
        lib.wl_batch_edges.argtypes = [ctypes.c_void_p]
        lib.wl_batch_take.restype = None
        lib.wl_batch_take.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6 + [ctypes.c_int32]
        lib.wl_batch_free.restype = None
        lib.wl_batch_free.argtypes = [ctypes.c_void_p]
        lib.wl_alloc_bytes.restype = None
        lib.wl_alloc_bytes.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]
        lib.wl_alloc_bytes_list.restype = None
        lib.wl_alloc_bytes_list.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        _lib = lib
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def generate(spec: Spec, seed: int, count: int, first: int = 0) -> DagBatch:
    """Generate DAGs first .. first+count-1 of the seeded stream of `spec`."""
    lib = _load()
    cs = spec.to_c()
    h = lib.wl_batch_generate(ctypes.byref(cs), ctypes.c_uint64(seed & (2**64 - 1)), first, count,
                              _threads())
    if not h:
        raise MemoryError("DAG generation failed")
    nn, ne = lib.wl_batch_nodes(h), lib.wl_batch_edges(h)
    b = DagBatch(np.empty(count + 1, np.int64), np.empty(count + 1, np.int64),
                 np.empty(ne, np.int32), np.empty(ne, np.int32), np.empty(nn, np.int64),
                 np.empty(nn, np.int32))
    lib.wl_batch_take(h, _ptr(b.node_off), _ptr(b.edge_off), _ptr(b.src), _ptr(b.dst),
                      _ptr(b.wcet), _ptr(b.par), _threads())
    return b


def generate_workload(k: int, count: Optional[int] = None, first: int = 0) -> DagBatch:
    w = WORKLOADS[k]
    return generate(w.spec, w.seed, w.num_dags if count is None else count, first)


def alloc_bytes(batch: DagBatch, num_cus: int, K: int, seed: int, first: int = 0) -> np.ndarray:
    """Explicit candidate bytes: (d, c, v) at K*node_off[d] + c*N_d + v.

    Candidate 0 is all zeros (the method's own rule); candidate c >= 1 draws
    r_v uniformly in 1..min(p_v, M, 255) from a counter-based hash of
    (seed, first+d, c, v)."""
    lib = _load()
    out = np.empty(int(batch.node_off[-1]) * K, np.uint8)
    lib.wl_alloc_bytes(ctypes.c_uint64(seed & (2**64 - 1)), first, batch.num_dags,
                       _ptr(batch.node_off), _ptr(batch.par), num_cus, K, _ptr(out), _threads())
    return out


_gpu_lib: Optional[ctypes.CDLL] = None


def alloc_bytes_device(node_off_dev, par_dev, count: int, max_n: int, num_cus: int, K: int, seed: int,
                       out_dev, stream=None, first: int = 0) -> None:
    """The bytes of `alloc_bytes` written by a GPU kernel straight into the
    device tensor `out_dev` (uint8, K * N), from device tensors `node_off_dev`
    (int64, count + 1) and `par_dev` (int32, N), on `stream` (a torch stream
    or None for the current one).  Same values as `alloc_bytes` for DAGs
    first .. first + count - 1."""
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(GPU_LIB_PATH):
            raise ImportError(f"{GPU_LIB_PATH} is not built (workloads.build())")
        lib = ctypes.CDLL(GPU_LIB_PATH)
        lib.wl_alloc_bytes_device.restype = ctypes.c_int
        lib.wl_alloc_bytes_device.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_void_p]
        _gpu_lib = lib
    import torch

    assert out_dev.dtype == torch.uint8 and node_off_dev.dtype == torch.int64 and par_dev.dtype == torch.int32
    total = int(node_off_dev[-1].item() - node_off_dev[0].item())
    assert out_dev.numel() >= total * K and par_dev.numel() >= total
    st = stream if stream is not None else torch.cuda.current_stream(out_dev.device)
    rc = _gpu_lib.wl_alloc_bytes_device(ctypes.c_uint64(seed & (2**64 - 1)), first, count,
                                        node_off_dev.data_ptr(), par_dev.data_ptr(), num_cus, K, max_n,
                                        out_dev.data_ptr(), ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"wl_alloc_bytes_device failed: hipError {rc}")


def alloc_bytes_list(batch: DagBatch, num_cus: int, cand: np.ndarray, seed: int, first: int = 0) -> np.ndarray:
    """Bytes of listed candidates: `cand` [D, L] candidate ids per DAG; row i
    of DAG d holds the bytes `alloc_bytes` gives candidate cand[d, i] (all
    zero for candidate 0), at L*node_off[d] + i*N_d + v."""
    lib = _load()
    cand = np.ascontiguousarray(np.asarray(cand, np.int32))
    assert cand.ndim == 2 and cand.shape[0] == batch.num_dags
    L = cand.shape[1]
    out = np.empty(int(batch.node_off[-1]) * L, np.uint8)
    lib.wl_alloc_bytes_list(ctypes.c_uint64(seed & (2**64 - 1)), first, batch.num_dags, _ptr(batch.node_off),
                            _ptr(batch.par), num_cus, L, _ptr(cand), _ptr(out), _threads())
    return out


def from_dags(dags) -> DagBatch:
    """Pack a list of (n, src, dst, wcet, par) into a DagBatch."""
    node_off = [0]
    edge_off = [0]
    for n, s, t, w, p in dags:
        node_off.append(node_off[-1] + int(n))
        edge_off.append(edge_off[-1] + len(s))
    cat = lambda xs, dt: (np.concatenate([np.asarray(x, dt) for x in xs]) if xs else np.empty(0, dt))
    return DagBatch(np.asarray(node_off, np.int64), np.asarray(edge_off, np.int64),
                    cat([d[1] for d in dags], np.int32), cat([d[2] for d in dags], np.int32),
                    cat([d[3] for d in dags], np.int64), cat([d[4] for d in dags], np.int32))


# Seed of the evaluation-style workloads (Section 5.1's setups).
PAPER_STYLE_SEED = BASE_SEED + 6


def paper_style(count: int, P: int, c_avg: int, depth=(5, 8), p_adj: float = 0.3,
                seed: int = PAPER_STYLE_SEED) -> DagBatch:
    """DAGs shaped like the evaluation's synthetic setups (Section 5.1): the
    number of layers is drawn in depth[0]..depth[1], the first layer is one
    source node and every later layer has U{2..P} nodes; each node of a layer
    takes one predecessor drawn from the layer before and every other pair of
    adjacent-layer nodes is an edge with probability p_adj; one sink follows
    every node left without a successor.  Loads are uniform in
    1..2*c_avg - 1 (mean c_avg) and the maximum parallelism is the load
    itself (t_min = 1, so m^max = C_hat).  DAG d draws from its own stream
    (seed, d); ids are in layer order."""
    dags = []
    for d in range(count):
        rng = np.random.default_rng([seed & (2**63 - 1), P, c_avg, depth[0], depth[1], d])
        layers = int(rng.integers(depth[0], depth[1] + 1))
        widths = [1] + [int(x) for x in rng.integers(2, P + 1, layers - 1)]
        first = np.cumsum([0] + widths)
        src, dst = [], []
        for l in range(1, layers):
            prev = np.arange(first[l - 1], first[l])
            for v in range(first[l], first[l + 1]):
                parent = int(prev[rng.integers(0, len(prev))])
                for u in prev:
                    if u == parent or rng.random() < p_adj:
                        src.append(int(u))
                        dst.append(v)
        n = int(first[-1]) + 1
        sink = n - 1
        has_succ = np.zeros(n, bool)
        has_succ[np.asarray(src, np.int64)] = True
        for u in range(sink):
            if not has_succ[u]:
                src.append(u)
                dst.append(sink)
        wcet = rng.integers(1, 2 * c_avg, n).astype(np.int64)
        dags.append((n, np.asarray(src, np.int32), np.asarray(dst, np.int32), wcet, wcet.astype(np.int32)))
    return from_dags(dags)


def random_small_dag(rng: np.random.Generator, n: int, p_edge: float, wmax: int, pmax: int):
    """A tiny random DAG for brute-force tests: edges follow a random order."""
    order = rng.permutation(n)
    src, dst = [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p_edge:
                src.append(int(order[i]))
                dst.append(int(order[j]))
    wcet = rng.integers(1, wmax + 1, n)
    par = rng.integers(1, pmax + 1, n)
    return n, np.asarray(src, np.int32), np.asarray(dst, np.int32), wcet.astype(np.int64), par.astype(np.int32)


def random_alloc(rng: np.random.Generator, par, M: int, zero_frac: float = 0.0) -> np.ndarray:
    """One candidate vector r in {0..255}: 0 (the method's rule) with
    probability zero_frac, else uniform in 1..min(p_v, M, 255)."""
    par = np.asarray(par)
    hi = np.minimum(np.minimum(par, M), 255)
    r = rng.integers(1, hi + 1)
    if zero_frac > 0:
        r[rng.random(len(par)) < zero_frac] = 0
    return r.astype(np.uint8)
