"""Python binding of libdagbound (include/dagbound.h): argument marshalling only.

Every step of the bound runs in the library's gfx950 kernels; this module
turns numpy arrays (host memory) or torch tensors (device memory of the
current HIP device, or host) into pointers and status codes into exceptions.
It fails loudly when the library is not built: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Any, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdagbound.so")

OK, E_ARG, E_CYCLE, E_RANGE, E_DUP_EDGE, E_OOM, E_DEVICE, E_STATE, E_OVERFLOW, E_UNSUPPORTED, E_IO = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10)
PTR_HOST, PTR_DEVICE = 0, 1
ALLOC_EXPLICIT, ALLOC_SEEDED = 0, 1
SEARCH_EXHAUSTIVE, SEARCH_SURROGATE = 0, 1
PARA_SPATIAL, PARA_TEMPORAL = 0, 1
MAX_NODES_PER_DAG = 8000
MAX_CANDIDATES = 1 << 22
MODEL_PARAMS = 100356

# Every symbol include/dagbound.h declares.
EXPORTS = (
    "dagbound_create_batch", "dagbound_set_allocations", "dagbound_eval_bounds",
    "dagbound_best_allocation", "dagbound_best_allocation_static", "dagbound_eval_listed",
    "dagbound_eval_conditional", "dagbound_get_division", "dagbound_get_schedule", "dagbound_baselines", "dagbound_run_schedule",
    "dagbound_set_para_launch",
    "dagbound_set_tuning",
    "dagbound_destroy_batch", "dagbound_model_create", "dagbound_model_destroy",
    "dagbound_model_params", "dagbound_model_forward", "dagbound_model_train_step",
    "dagbound_model_select", "dagbound_model_save", "dagbound_model_load",
    "dagbound_shutdown", "dagbound_last_error", "dagbound_version",
)

_lib: Optional[ctypes.CDLL] = None
# Live handles, closed in order at interpreter exit (while the HIP runtime is
# still up), before the library releases its process-wide resources.
_live: "weakref.WeakSet" = weakref.WeakSet()


def _close_all() -> None:
    if _lib is None:
        return
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass
    _lib.dagbound_shutdown()


atexit.register(_close_all)


class DagboundError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"libdagbound status {code}: {message}")
        self.code = code
        self.message = message


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdagbound.so (built by paper_2602_20826_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    P, I32, U32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    lib.dagbound_create_batch.restype = I32
    lib.dagbound_create_batch.argtypes = [I32, P, P, P, P, P, P, I32, U32, P, ctypes.POINTER(P)]
    lib.dagbound_set_allocations.restype = I32
    lib.dagbound_set_allocations.argtypes = [P, I32, U32, P, U64, U32]
    lib.dagbound_eval_bounds.restype = I32
    lib.dagbound_eval_bounds.argtypes = [P, P, P, P, U32, P]
    lib.dagbound_eval_listed.restype = I32
    lib.dagbound_eval_listed.argtypes = [P, I32, P, P, P, P, U32, P]
    lib.dagbound_eval_conditional.restype = I32
    lib.dagbound_eval_conditional.argtypes = [P, P, P, P, P, U32, P]
    lib.dagbound_model_save.restype = I32
    lib.dagbound_model_save.argtypes = [P, ctypes.c_char_p]
    lib.dagbound_model_load.restype = I32
    lib.dagbound_model_load.argtypes = [P, ctypes.c_char_p]
    lib.dagbound_shutdown.restype = None
    lib.dagbound_shutdown.argtypes = []
    lib.dagbound_best_allocation.restype = I32
    lib.dagbound_best_allocation.argtypes = [P, U32, I32, P, P, P, U32, P]
    lib.dagbound_best_allocation_static.restype = I32
    lib.dagbound_best_allocation_static.argtypes = [P, P, I32, P, P, P]
    lib.dagbound_get_division.restype = I32
    lib.dagbound_get_division.argtypes = [P, I32, P, P, P, P]
    lib.dagbound_get_schedule.restype = I32
    lib.dagbound_get_schedule.argtypes = [P, I32, I32, P, ctypes.c_int64, P, P]
    lib.dagbound_set_para_launch.restype = I32
    lib.dagbound_set_para_launch.argtypes = [P, U32]
    lib.dagbound_run_schedule.restype = I32
    lib.dagbound_run_schedule.argtypes = [P, I32, I32, ctypes.c_int64, I32, I32, P, P]
    lib.dagbound_baselines.restype = I32
    lib.dagbound_baselines.argtypes = [P, P, P, P, U32, P]
    lib.dagbound_set_tuning.restype = I32
    lib.dagbound_set_tuning.argtypes = [P, ctypes.c_char_p, ctypes.c_int64]
    lib.dagbound_destroy_batch.restype = None
    lib.dagbound_destroy_batch.argtypes = [P]
    lib.dagbound_last_error.restype = ctypes.c_char_p
    lib.dagbound_last_error.argtypes = []
    lib.dagbound_model_create.restype = I32
    lib.dagbound_model_create.argtypes = [U64, ctypes.POINTER(P)]
    lib.dagbound_model_destroy.restype = None
    lib.dagbound_model_destroy.argtypes = [P]
    lib.dagbound_model_params.restype = I32
    lib.dagbound_model_params.argtypes = [P, P, P, P, P]
    lib.dagbound_model_forward.restype = I32
    lib.dagbound_model_forward.argtypes = [P, P, P, U32, P]
    lib.dagbound_model_train_step.restype = I32
    lib.dagbound_model_train_step.argtypes = [P, P, I32, U64, P, ctypes.c_float, P, U32, P]
    lib.dagbound_model_select.restype = I32
    lib.dagbound_model_select.argtypes = [P, P, I32, U64, I32, I32, P, P, U32, P]
    lib.dagbound_version.restype = ctypes.c_char_p
    lib.dagbound_version.argtypes = []
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().dagbound_last_error().decode()


def version() -> str:
    return load_library().dagbound_version().decode()


def _check(rc: int) -> None:
    if rc != OK:
        raise DagboundError(rc, last_error())


def _is_torch(x: Any) -> bool:
    return type(x).__module__.startswith("torch")


_NP = {"int64": np.int64, "int32": np.int32, "uint8": np.uint8, "float32": np.float32}


def _marshal(arrays: Sequence[Tuple[Any, str]]):
    """Pointers for (array, dtype name) pairs; all must live in one kind of
    memory.  Returns (pointers, ptr_kind, keepalive)."""
    kinds = set()
    ptrs = []
    keep = []
    for a, dt in arrays:
        if a is None:
            ptrs.append(None)
            continue
        if _is_torch(a):
            import torch

            want = getattr(torch, dt)
            if a.dtype != want:
                raise TypeError(f"expected a {dt} tensor, got {a.dtype}")
            if not a.is_contiguous():
                raise ValueError("tensors must be contiguous")
            kinds.add(PTR_DEVICE if a.is_cuda else PTR_HOST)
            ptrs.append(a.data_ptr() if a.numel() else None)
            keep.append(a)
        else:
            arr = np.asarray(a)
            if arr.dtype != _NP[dt]:
                raise TypeError(f"expected {dt}, got {arr.dtype}")
            if not arr.flags.c_contiguous:
                raise ValueError("arrays must be C-contiguous")
            kinds.add(PTR_HOST)
            ptrs.append(arr.ctypes.data if arr.size else None)
            keep.append(arr)
    if len(kinds) > 1:
        raise ValueError("all arrays of one call must be in the same memory (host or device)")
    return ptrs, (kinds.pop() if kinds else PTR_HOST), keep


def _stream_ptr(stream, arrays: Sequence[Any] = ()) -> Optional[int]:
    """The hipStream_t of `stream` (a torch stream or a raw handle).  With
    None and a device tensor among `arrays`, torch's current stream of that
    tensor's device, so the call is ordered after the work that produced it
    (for torch's default stream that is the NULL stream: the call then
    waits for its work)."""
    if stream is None:
        for a in arrays:
            if a is not None and _is_torch(a) and a.is_cuda:
                import torch

                stream = torch.cuda.current_stream(a.device)
                break
        else:
            return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream) or None


class Batch:
    """Owning handle of a dagbound_batch."""

    def __init__(self, handle: int, num_dags: int, node_off_host: np.ndarray):
        self.handle = handle
        self.num_dags = num_dags
        self.node_off = node_off_host
        self.K = 0
        _live.add(self)

    def close(self) -> None:
        if self.handle:
            load_library().dagbound_destroy_batch(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # at interpreter exit the atexit hook has closed every live handle
        # (and module globals such as sys may already be gone)
        if not self.handle or sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def create_batch(node_off, edge_off, edge_src, edge_dst, wcet, max_par, num_cus: int,
                 stream=None) -> Batch:
    """dagbound_create_batch: ingest and preprocess a batch of DAG tasks."""
    lib = load_library()
    (p_no, p_eo, p_s, p_t, p_w, p_p), kind, keep = _marshal(
        [(node_off, "int64"), (edge_off, "int64"), (edge_src, "int32"), (edge_dst, "int32"),
         (wcet, "int64"), (max_par, "int32")])
    num_dags = int(len(node_off)) - 1
    out = ctypes.c_void_p()
    _check(lib.dagbound_create_batch(num_dags, p_no, p_eo, p_s, p_t, p_w, p_p, int(num_cus), kind,
                                     _stream_ptr(stream, keep), ctypes.byref(out)))
    if _is_torch(node_off):
        no = node_off.detach().cpu().numpy()
    else:
        no = np.asarray(node_off)
    return Batch(out.value, num_dags, no.astype(np.int64))


def set_allocations(batch: Batch, K: int, mode: int = ALLOC_EXPLICIT, alloc=None, seed: int = 0) -> None:
    """dagbound_set_allocations: explicit bytes (host array or device tensor) or a seed."""
    lib = load_library()
    (p_a,), kind, keep = _marshal([(alloc, "uint8")])
    _check(lib.dagbound_set_allocations(ctypes.c_void_p(batch.handle), int(K), int(mode), p_a,
                                        ctypes.c_uint64(seed & (2**64 - 1)), kind))
    batch.K = int(K)
    batch._alloc_keep = keep  # explicit device bytes are read in place later


def eval_bounds(batch: Batch, bounds, cp_term=None, intf_term=None, stream=None) -> None:
    """dagbound_eval_bounds: bounds[d*K + c] (+ optional terms), written in place."""
    lib = load_library()
    (p_b, p_c, p_i), kind, keep = _marshal([(bounds, "int64"), (cp_term, "int64"), (intf_term, "int64")])
    _check(lib.dagbound_eval_bounds(ctypes.c_void_p(batch.handle), p_b, p_c, p_i, kind,
                                    _stream_ptr(stream, keep)))


def eval_listed(batch: Batch, cand, bounds, cp_term=None, intf_term=None, stream=None) -> None:
    """dagbound_eval_listed: bounds[d*L + i] of candidate cand[d*L + i] of DAG
    d (int32 ids, L per DAG), written in place; waits for its work."""
    lib = load_library()
    (p_l, p_b, p_c, p_i), kind, keep = _marshal([(cand, "int32"), (bounds, "int64"), (cp_term, "int64"),
                                                 (intf_term, "int64")])
    n = int(np.prod(np.shape(cand))) if not _is_torch(cand) else cand.numel()
    if batch.num_dags == 0 or n % batch.num_dags:
        raise ValueError("cand must hold L entries per DAG")
    _check(lib.dagbound_eval_listed(ctypes.c_void_p(batch.handle), n // batch.num_dags, p_l, p_b, p_c, p_i,
                                    kind, _stream_ptr(stream, keep)))


def baselines(batch: Batch, greedy=None, greedy_unaware=None, graham_para=None, stream=None):
    """dagbound_baselines: the comparison bounds of Section 5.2 per DAG,
    written in place into the given [D] int64 arrays; with none given, host
    arrays are allocated and returned as (greedy, greedy_unaware, graham_para)."""
    lib = load_library()
    if greedy is None and greedy_unaware is None and graham_para is None:
        greedy, greedy_unaware, graham_para = (np.zeros(batch.num_dags, np.int64) for _ in range(3))
    (p_g, p_u, p_h), kind, keep = _marshal([(greedy, "int64"), (greedy_unaware, "int64"),
                                            (graham_para, "int64")])
    _check(lib.dagbound_baselines(ctypes.c_void_p(batch.handle), p_g, p_u, p_h, kind, _stream_ptr(stream, keep)))
    return greedy, greedy_unaware, graham_para


def set_para_launch(batch: Batch, mode: int) -> None:
    """dagbound_set_para_launch: PARA_SPATIAL or PARA_TEMPORAL reading of the
    launching loop for the batch's later evaluations."""
    _check(load_library().dagbound_set_para_launch(ctypes.c_void_p(batch.handle), int(mode)))


def run_schedule(batch: Batch, d: int, c: int, tick_ns: int, barriers: bool = True, reps: int = 10):
    """dagbound_run_schedule: (makespan_ns [reps] int64, (bound, cp, intf,
    parts)) of DAG d's schedule under candidate c run as a HIP graph."""
    out = np.zeros(reps, np.int64)
    terms = np.zeros(4, np.int64)
    _check(load_library().dagbound_run_schedule(ctypes.c_void_p(batch.handle), int(d), int(c), int(tick_ns),
                                                int(bool(barriers)), int(reps), out.ctypes.data, terms.ctypes.data))
    return out, tuple(int(x) for x in terms)


def best_allocation(batch: Batch, best_idx, best_bound, search: int = SEARCH_EXHAUSTIVE,
                    top_k: int = 0, model=None, stream=None) -> None:
    """dagbound_best_allocation: per-DAG argmin candidate and its bound."""
    lib = load_library()
    (p_i, p_b), kind, keep = _marshal([(best_idx, "int32"), (best_bound, "int64")])
    mh = ctypes.c_void_p(model.handle) if model is not None else None
    _check(lib.dagbound_best_allocation(ctypes.c_void_p(batch.handle), int(search), int(top_k),
                                        mh, p_i, p_b, kind, _stream_ptr(stream, keep)))


def eval_conditional(batch: Batch, cond_of, branch_of, bounds, worst=None, stream=None) -> None:
    """dagbound_eval_conditional: bounds[d*K + c] the largest realization
    bound of conditional DAG d under candidate c (and the first realization
    reaching it in worst)."""
    lib = load_library()
    (pc, pb, po, pw), kind, keep = _marshal([(cond_of, "int32"), (branch_of, "int32"), (bounds, "int64"),
                                             (worst, "int32")])
    _check(lib.dagbound_eval_conditional(ctypes.c_void_p(batch.handle), pc, pb, po, pw, kind,
                                         _stream_ptr(stream, keep)))


def best_allocation_static(batch: Batch, model, top_k: int, best_idx, best_bound, stream=None) -> None:
    """dagbound_best_allocation_static: the surrogate search without device
    allocation (device tensors only; the model's workspace must already be
    sized for the batch by an allocating call)."""
    lib = load_library()
    (p_i, p_b), kind, keep = _marshal([(best_idx, "int32"), (best_bound, "int64")])
    if kind != PTR_DEVICE:
        raise DagboundError(E_ARG, "best_allocation_static takes device tensors")
    _check(lib.dagbound_best_allocation_static(ctypes.c_void_p(batch.handle), ctypes.c_void_p(model.handle),
                                               int(top_k), p_i, p_b, _stream_ptr(stream, keep)))


class Model:
    """Owning handle of a dagbound_model (learned candidate proposal)."""

    def __init__(self, seed: int = 0):
        out = ctypes.c_void_p()
        _check(load_library().dagbound_model_create(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.byref(out)))
        self.handle = out.value
        _live.add(self)

    def close(self) -> None:
        if self.handle:
            load_library().dagbound_model_destroy(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        if not self.handle or sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def save(self, path: str) -> None:
        """dagbound_model_save: parameters, Adam moments and step to `path`."""
        _check(load_library().dagbound_model_save(ctypes.c_void_p(self.handle), os.fsencode(path)))

    def load(self, path: str) -> None:
        """dagbound_model_load: parameters, Adam moments and step from `path`."""
        _check(load_library().dagbound_model_load(ctypes.c_void_p(self.handle), os.fsencode(path)))

    def params(self) -> np.ndarray:
        out = np.empty(MODEL_PARAMS, np.float32)
        _check(load_library().dagbound_model_params(ctypes.c_void_p(self.handle), out.ctypes.data,
                                                    None, None, None))
        return out

    def set_params(self, p) -> None:
        arr = np.ascontiguousarray(np.asarray(p, np.float32))
        assert arr.size == MODEL_PARAMS
        _check(load_library().dagbound_model_params(ctypes.c_void_p(self.handle), None, arr.ctypes.data,
                                                    None, None))

    def grad(self) -> np.ndarray:
        out = np.empty(MODEL_PARAMS, np.float32)
        _check(load_library().dagbound_model_params(ctypes.c_void_p(self.handle), None, None,
                                                    out.ctypes.data, None))
        return out

    def step(self) -> int:
        st = ctypes.c_int64(0)
        _check(load_library().dagbound_model_params(ctypes.c_void_p(self.handle), None, None, None,
                                                    ctypes.byref(st)))
        return int(st.value)


def model_forward(model: Model, batch: Batch, node_out, stream=None) -> None:
    """dagbound_model_forward: per-node head coefficients [T_N][3]."""
    (p_o,), kind, keep = _marshal([(node_out, "float32")])
    _check(load_library().dagbound_model_forward(ctypes.c_void_p(model.handle), ctypes.c_void_p(batch.handle),
                                                 p_o, kind, _stream_ptr(stream, keep)))


def model_train_step(model: Model, batch: Batch, K: int, seed: int, bounds, lr: float, stream=None) -> float:
    """dagbound_model_train_step: one Adam step; returns the loss before it."""
    (p_b,), kind, keep = _marshal([(bounds, "int64")])
    loss = ctypes.c_float(0)
    _check(load_library().dagbound_model_train_step(ctypes.c_void_p(model.handle), ctypes.c_void_p(batch.handle),
                                                    int(K), ctypes.c_uint64(seed & (2**64 - 1)), p_b,
                                                    ctypes.c_float(lr), ctypes.byref(loss), kind,
                                                    _stream_ptr(stream, keep)))
    return float(loss.value)


def model_select(model: Model, batch: Batch, K: int, seed: int, top_k: int, nodes: int, cand, scores=None,
                 stream=None) -> None:
    """dagbound_model_select: candidate lists [D][top_k+1] (device tensors)."""
    (p_c, p_s), kind, keep = _marshal([(cand, "int32"), (scores, "float32")])
    _check(load_library().dagbound_model_select(ctypes.c_void_p(model.handle), ctypes.c_void_p(batch.handle),
                                                int(K), ctypes.c_uint64(seed & (2**64 - 1)), int(top_k),
                                                int(nodes), p_c, p_s, kind, _stream_ptr(stream, keep)))


def get_division(batch: Batch, d: int):
    """dagbound_get_division: (wanc, group_of, order, num_groups) of DAG d."""
    lib = load_library()
    n = int(batch.node_off[d + 1] - batch.node_off[d])
    wanc = np.zeros(max(n, 1), np.int64)
    gof = np.zeros(max(n, 1), np.int32)
    order = np.zeros(max(n, 1), np.int32)
    ng = ctypes.c_int32(0)
    _check(lib.dagbound_get_division(ctypes.c_void_p(batch.handle), int(d), wanc.ctypes.data,
                                     gof.ctypes.data, order.ctypes.data, ctypes.byref(ng)))
    return wanc[:n], gof[:n], order[:n], int(ng.value)


def get_schedule(batch: Batch, d: int, c: int, cap: int = 4096):
    """dagbound_get_schedule: (records [n][8] int64, (bound, cp, intf)) of DAG
    d under candidate c; the buffer grows until every record fits."""
    lib = load_library()
    count = ctypes.c_int64(0)
    terms = np.zeros(3, np.int64)
    while True:
        rec = np.zeros((max(cap, 1), 8), np.int64)
        _check(lib.dagbound_get_schedule(ctypes.c_void_p(batch.handle), int(d), int(c), rec.ctypes.data,
                                         int(cap), ctypes.byref(count), terms.ctypes.data))
        if count.value <= cap:
            return rec[:count.value].copy(), tuple(int(x) for x in terms)
        cap = int(count.value)


def set_tuning(batch: Batch, key: str, value: int) -> None:
    """dagbound_set_tuning: launch-plan options (never change results)."""
    _check(load_library().dagbound_set_tuning(ctypes.c_void_p(batch.handle), key.encode(), int(value)))


def destroy_batch(batch: Batch) -> None:
    batch.close()


def shutdown() -> None:
    """dagbound_shutdown after closing every live batch and model (also run
    at interpreter exit)."""
    _close_all()
