"""Float64 reference of the learned candidate proposal -- TEST INFRASTRUCTURE ONLY.

Plain numpy: the node features, the message-passing encoder, the per-node
head coefficients, the candidate score and the training loss, with a
hand-written backward pass and a finite-difference check of it.  The GPU
kernels (BF16 on MFMA, FP32 accumulation) are compared against this file.

Model (one DAG, nodes in local-id order, N(v) = predecessors and successors):
  x_v  = 8 features (see `features`)
  H0   = relu(X W0 + b0)                               128 wide
  G_l  = mean over N(v) of H_{l-1}(u)   (zero if v has no neighbour)
  H_l  = relu(H_{l-1} Ws_l + G_l Wm_l + b_l),  l = 1, 2, 3
  A    = H3 Wa + ba;  a_v = A[v, 0:3]
Candidate score (lower = smaller predicted bound), for candidate bytes
r_v >= 1 and range_v = min(p_v, M, 255):
  t_v  = r_v / range_v,  phi(t) = (t, t^2, 1/t)
  s(r) = (1/n) sum_v a_v . phi(t_v)
Training target for candidate c >= 1: ln(bound_c) - ln(bound_0); loss =
mean squared error over the (DAG, candidate) pairs of a step.
Inference head (ranking thousands of candidates per DAG): the same score
summed over at most T nodes only (`head_select`: range > 1, largest
|a0| + |a1| + range*|a2| first, ties to the smaller id), still divided by n.

Parameters are one flat float32 vector in this order: W0 [8x128], b0 [128],
then for l = 1..3: Ws_l [128x128], Wm_l [128x128], b_l [128]; then
Wa [128x4], ba [4].  Matrices are row-major, input index first.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

F_IN, HID, LAYERS, OUT = 8, 128, 3, 4


def param_shapes() -> List[Tuple[str, Tuple[int, ...]]]:
    shapes = [("W0", (F_IN, HID)), ("b0", (HID,))]
    for l in range(1, LAYERS + 1):
        shapes += [(f"Ws{l}", (HID, HID)), (f"Wm{l}", (HID, HID)), (f"b{l}", (HID,))]
    shapes += [("Wa", (HID, OUT)), ("ba", (OUT,))]
    return shapes


def num_params() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def unflatten(flat: np.ndarray) -> Dict[str, np.ndarray]:
    out = {}
    o = 0
    for name, shp in param_shapes():
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in param_shapes()])


def features(n, src, dst, wcet, par, M, wanc, groups) -> np.ndarray:
    """Eight candidate-independent features per node (local-id order):
    log2 load / 16, log2 min(p, M) / 8, log2 W^anc / 24, log2 group size / 8,
    group position in [0, 1], log2(1 + in-degree) / 6, log2(1 + out-degree) / 6,
    and the node's share of its group's load."""
    wcet = np.asarray(wcet, np.float64)
    par = np.minimum(np.asarray(par, np.float64), M)
    X = np.zeros((n, F_IN))
    gsize = np.zeros(n)
    gpos = np.zeros(n)
    gload = np.zeros(n)
    G = len(groups)
    for j, g in enumerate(groups):
        tot = float(sum(wcet[v] for v in g))
        for v in g:
            gsize[v] = len(g)
            gpos[v] = j / max(1, G - 1)
            gload[v] = tot
    indeg = np.bincount(np.asarray(dst, np.int64), minlength=n)
    outdeg = np.bincount(np.asarray(src, np.int64), minlength=n)
    X[:, 0] = np.log2(wcet) / 16
    X[:, 1] = np.log2(par) / 8
    X[:, 2] = np.log2(np.asarray(wanc, np.float64)) / 24
    X[:, 3] = np.log2(gsize) / 8
    X[:, 4] = gpos
    X[:, 5] = np.log2(1 + indeg) / 6
    X[:, 6] = np.log2(1 + outdeg) / 6
    X[:, 7] = wcet / gload
    return X


def neighbours(n, src, dst) -> List[List[int]]:
    nb = [[] for _ in range(n)]
    for u, v in zip(src, dst):
        nb[int(u)].append(int(v))
        nb[int(v)].append(int(u))
    return nb


def _agg(H, nb):
    G = np.zeros_like(H)
    for v, lst in enumerate(nb):
        if lst:
            G[v] = H[lst].mean(0)
    return G


def _agg_t(Y, nb):
    """Transpose of the mean aggregation: out[u] = sum over v in N(u) of Y[v] / |N(v)|."""
    out = np.zeros_like(Y)
    for u, lst in enumerate(nb):
        for v in lst:
            out[u] += Y[v] / len(nb[v])
    return out


@dataclass
class Tape:
    X: np.ndarray
    H: List[np.ndarray]   # H0..H3
    G: List[np.ndarray]   # G1..G3 (index l-1)
    A: np.ndarray


def forward(p: Dict[str, np.ndarray], X: np.ndarray, nb) -> Tape:
    H = [np.maximum(X @ p["W0"] + p["b0"], 0.0)]
    Gs = []
    for l in range(1, LAYERS + 1):
        G = _agg(H[-1], nb)
        Gs.append(G)
        H.append(np.maximum(H[-1] @ p[f"Ws{l}"] + G @ p[f"Wm{l}"] + p[f"b{l}"], 0.0))
    A = H[-1] @ p["Wa"] + p["ba"]
    return Tape(X, H, Gs, A)


def phi(t: np.ndarray) -> np.ndarray:
    return np.stack([t, t * t, 1.0 / t], -1)


def scores(A: np.ndarray, rbytes: np.ndarray, rng_v: np.ndarray) -> np.ndarray:
    """rbytes [C, n] (>= 1), rng_v [n] -> scores [C]."""
    t = np.asarray(rbytes, np.float64) / np.asarray(rng_v, np.float64)[None, :]
    return (phi(t) * A[None, :, :3]).sum((1, 2)) / A.shape[0]


def head_select(A: np.ndarray, rng_v: np.ndarray, T: int) -> List[int]:
    """Nodes whose candidate bytes the per-candidate head reads: among the
    nodes of range > 1 (a node of range 1 has t = 1 in every candidate, so it
    adds the same amount to every score), the T of largest importance
    |a0| + |a1| + range * |a2|, largest first, ties to the smaller id."""
    A = np.asarray(A, np.float64)
    rng_v = np.asarray(rng_v, np.float64)
    imp = np.abs(A[:, 0]) + np.abs(A[:, 1]) + rng_v * np.abs(A[:, 2])
    eligible = [v for v in range(A.shape[0]) if rng_v[v] > 1]
    eligible.sort(key=lambda v: (-imp[v], v))
    return eligible[:T]


def head_scores(A: np.ndarray, rbytes: np.ndarray, rng_v: np.ndarray, sel: List[int]) -> np.ndarray:
    """Score of each candidate row of rbytes [C, n] over the selected nodes
    only, still divided by the DAG's node count n:
      s(r) = (1/n) sum over v in sel of a_v . phi(r_v / range_v)."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    sel = list(sel)
    if not sel:
        return np.zeros(np.asarray(rbytes).shape[0])
    t = np.asarray(rbytes, np.float64)[:, sel] / np.asarray(rng_v, np.float64)[None, sel]
    return (phi(t) * A[None, sel, :3]).sum((1, 2)) / n


def loss_and_grad(p, X, nb, rbytes, rng_v, y, scale):
    """Loss scale * sum_c (s_c - y_c)^2 of one DAG and its gradient (dict)."""
    tape = forward(p, X, nb)
    n = X.shape[0]
    t = np.asarray(rbytes, np.float64) / np.asarray(rng_v, np.float64)[None, :]
    ph = phi(t)                                  # [C, n, 3]
    s = (ph * tape.A[None, :, :3]).sum((1, 2)) / n
    diff = s - y
    loss = scale * float((diff ** 2).sum())
    ds = 2.0 * scale * diff                      # [C]
    dA = np.zeros_like(tape.A)
    dA[:, :3] = np.einsum("c,cnk->nk", ds, ph) / n
    g = {k: np.zeros_like(v) for k, v in p.items()}
    g["Wa"] = tape.H[-1].T @ dA
    g["ba"] = dA.sum(0)
    dH = dA @ p["Wa"].T
    for l in range(LAYERS, 0, -1):
        dZ = dH * (tape.H[l] > 0)
        g[f"Ws{l}"] = tape.H[l - 1].T @ dZ
        g[f"Wm{l}"] = tape.G[l - 1].T @ dZ
        g[f"b{l}"] = dZ.sum(0)
        dH = dZ @ p[f"Ws{l}"].T + _agg_t(dZ @ p[f"Wm{l}"].T, nb)
    dZ0 = dH * (tape.H[0] > 0)
    g["W0"] = X.T @ dZ0
    g["b0"] = dZ0.sum(0)
    return loss, g, s


def finite_difference_check(p, X, nb, rbytes, rng_v, y, scale, names=None, eps=1e-6, k=12, seed=0):
    """Largest relative difference between the hand-written gradient and
    central differences, over k random entries of each named parameter."""
    rng = np.random.default_rng(seed)
    _, g, _ = loss_and_grad(p, X, nb, rbytes, rng_v, y, scale)
    worst = 0.0
    for name in names or list(p):
        flat = p[name].ravel()
        for i in rng.choice(flat.size, min(k, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + eps
            lp, _, _ = loss_and_grad(p, X, nb, rbytes, rng_v, y, scale)
            flat[i] = old - eps
            lm, _, _ = loss_and_grad(p, X, nb, rbytes, rng_v, y, scale)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].ravel()[i]
            worst = max(worst, abs(fd - an) / max(1e-8, abs(fd) + abs(an)))
    return worst
