"""CPU pins of the float64 reference of the learned proposal
(oracle/surrogate_ref.py): its backward pass against central finite
differences, permutation equivariance of the message passing, the score's
closed form at t = 1, and the features of the paper's worked example."""
import json
import os

import numpy as np

import oracle
from oracle import surrogate_ref as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in S.param_shapes():
        p[name] = rng.normal(0, 0.2, shp) if name.startswith("b") else rng.uniform(-1, 1, shp) * scale * np.sqrt(3.0 / shp[0])
    return p


def example():
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    e = np.asarray(ex["edges"], np.int64)
    n, src, dst, w, p, M = ex["n"], e[:, 0], e[:, 1], ex["wcet"], ex["par"], ex["M"]
    div = oracle.division(n, src, dst, w, p, M)
    return n, src, dst, w, p, M, div


def test_parameter_count_matches_header():
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "dagbound.h")).read()
    assert f"#define DAGBOUND_MODEL_PARAMS {S.num_params()}" in hdr


def test_backward_matches_finite_differences():
    n, src, dst, w, p, M, div = example()
    X = S.features(n, src, dst, w, p, M, div.wanc, div.groups)
    nb = S.neighbours(n, src, dst)
    rng = np.random.default_rng(3)
    C = 5
    rng_v = np.minimum(np.minimum(np.asarray(p), M), 255)
    rb = np.stack([rng.integers(1, rng_v + 1) for _ in range(C)]).astype(np.float64)
    y = rng.normal(0, 0.3, C)
    params = rand_params(1)
    worst = S.finite_difference_check(params, X, nb, rb, rng_v, y, 1.0 / C, k=6)
    assert worst < 1e-6, worst


def test_message_passing_is_permutation_equivariant():
    n, src, dst, w, p, M, div = example()
    X = S.features(n, src, dst, w, p, M, div.wanc, div.groups)
    params = rand_params(2)
    A = S.forward(params, X, S.neighbours(n, src, dst)).A
    perm = np.random.default_rng(5).permutation(n)  # new id of old node v is perm[v]
    Xp = np.zeros_like(X)
    Xp[perm] = X
    Ap = S.forward(params, Xp, S.neighbours(n, perm[src], perm[dst])).A
    assert np.allclose(Ap[perm], A, rtol=1e-12, atol=1e-12)


def test_isolated_nodes_ignore_the_message_weights():
    rng = np.random.default_rng(7)
    X = rng.normal(0, 1, (6, S.F_IN))
    nb = [[] for _ in range(6)]
    p1 = rand_params(4)
    p2 = {k: v.copy() for k, v in p1.items()}
    for l in range(1, S.LAYERS + 1):
        p2[f"Wm{l}"] = rng.normal(0, 1, p2[f"Wm{l}"].shape)
    assert np.array_equal(S.forward(p1, X, nb).A, S.forward(p2, X, nb).A)


def test_score_at_full_range_is_sum_of_coefficients():
    rng = np.random.default_rng(9)
    A = rng.normal(0, 1, (7, S.OUT))
    rng_v = rng.integers(1, 40, 7)
    s = S.scores(A, rng_v[None, :].astype(np.float64), rng_v)  # t = 1 on every node
    assert np.isclose(s[0], A[:, :3].sum() / 7)
    s2 = S.scores(A, (rng_v[None, :] / 2.0), rng_v)  # t = 1/2: (t, t^2, 1/t) = (0.5, 0.25, 2)
    assert np.isclose(s2[0], (0.5 * A[:, 0] + 0.25 * A[:, 1] + 2.0 * A[:, 2]).sum() / 7)


def test_features_of_the_worked_example():
    n, src, dst, w, p, M, div = example()
    X = S.features(n, src, dst, w, p, M, div.wanc, div.groups)
    # v0 is the source (in-degree 0, out-degree 3), load 1, p 1
    assert X[0, 0] == 0.0 and X[0, 1] == 0.0
    assert X[0, 5] == 0.0 and np.isclose(X[0, 6], 2.0 / 6)
    # the sink v6 has in-degree 3 and out-degree 0
    assert np.isclose(X[6, 5], 2.0 / 6) and X[6, 6] == 0.0
    # group position runs 0 .. 1 over the groups; shares of a group sum to 1
    for g in div.groups:
        assert np.isclose(sum(X[v, 7] for v in g), 1.0)
    assert X[div.groups[0][0], 4] == 0.0 and X[div.groups[-1][0], 4] == 1.0
    # W^anc of the sink is the total load
    assert np.isclose(X[6, 2], np.log2(sum(w)) / 24)


def test_messages_do_not_depend_on_edge_direction():
    # N(v) holds predecessors and successors alike: reversing every edge
    # leaves the encoder's output unchanged for the same node features.
    n, src, dst, w, p, M, div = example()
    X = S.features(n, src, dst, w, p, M, div.wanc, div.groups)
    params = rand_params(6)
    a = S.forward(params, X, S.neighbours(n, src, dst)).A
    b = S.forward(params, X, S.neighbours(n, dst, src)).A
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    # and a node's output does depend on its neighbours
    c = S.forward(params, X, S.neighbours(n, src[:-1], dst[:-1])).A
    assert not np.allclose(a[6], c[6])
