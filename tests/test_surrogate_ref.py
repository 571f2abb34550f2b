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


def sparse_params():
    """All-zero parameters except a few entries, so that the encoder's output
    on a small graph can be worked out by hand."""
    p = {name: np.zeros(shp) for name, shp in S.param_shapes()}
    p["W0"][0, 0] = 1.0    # unit 0 <- feature 0
    p["W0"][0, 1] = -1.0   # unit 1 <- -feature 0 (cut to zero by the ReLU)
    p["Ws1"][0, 0] = 1.0   # layer 1: unit 0 keeps itself ...
    p["Wm1"][0, 0] = 1.0   # ... plus its neighbours' mean
    p["Ws1"][0, 1] = 2.0   # unit 1 <- 2 x unit 0 (input index first)
    p["Ws2"][0, 0] = 1.0
    p["Wm2"][0, 0] = 1.0
    p["Ws2"][1, 1] = 1.0
    p["b2"][1] = -3.0
    p["Ws3"][0, 0] = 1.0
    p["Wm3"][0, 0] = 1.0
    p["Wm3"][1, 1] = 1.0   # unit 1 <- its neighbours' mean of unit 1 only
    p["Wa"][0, 0] = 1.0
    p["Wa"][1, 2] = 1.0
    p["ba"][1] = 0.25
    p["ba"][3] = 7.0
    return p


def test_forward_by_hand_on_a_path():
    # Path 0 - 1 - 2 (edges 0->1, 1->2; N(1) = {0, 2}), feature 0 = (1, 2, 4).
    #   H0: unit 0 = (1, 2, 4), unit 1 = relu(-x) = 0
    #   layer 1: unit 0 = x + mean of neighbours = (1+2, 2+(1+4)/2, 4+2)
    #            = (3, 4.5, 6); unit 1 = 2 x H0 unit 0 = (2, 4, 8)
    #   layer 2: unit 0 = (3+4.5, 4.5+(3+6)/2, 6+4.5) = (7.5, 9, 10.5);
    #            unit 1 = relu((2, 4, 8) - 3) = (0, 1, 5)
    #   layer 3: unit 0 = (7.5+9, 9+(7.5+10.5)/2, 10.5+9) = (16.5, 18, 19.5);
    #            unit 1 = neighbours' mean of (0, 1, 5) = (1, (0+5)/2, 1)
    #   A = (unit 0, 0.25, unit 1, 7)
    # A sum over the neighbours instead of the mean gives 7 for node 1 in
    # layer 1 already.
    X = np.zeros((3, S.F_IN))
    X[:, 0] = (1.0, 2.0, 4.0)
    X[:, 3] = (5.0, -2.0, 0.5)  # features without a weight change nothing
    nb = S.neighbours(3, np.array([0, 1]), np.array([1, 2]))
    A = S.forward(sparse_params(), X, nb).A
    want = np.array([[16.5, 0.25, 1.0, 7.0], [18.0, 0.25, 2.5, 7.0], [19.5, 0.25, 1.0, 7.0]])
    assert np.array_equal(A, want), A


def test_score_by_hand():
    # With the A above, ranges 4 and bytes (2, 4, 1): t = (1/2, 1, 1/4),
    #   node 0: 16.5/2 + 0.25/4 + 1*2   = 10.3125
    #   node 1: 18     + 0.25   + 2.5   = 20.75
    #   node 2: 19.5/4 + 0.25/16 + 1*4  = 8.890625
    # sum 39.953125 over n = 3 nodes.
    A = np.array([[16.5, 0.25, 1.0, 7.0], [18.0, 0.25, 2.5, 7.0], [19.5, 0.25, 1.0, 7.0]])
    s = S.scores(A, np.array([[2.0, 4.0, 1.0]]), np.array([4, 4, 4]))
    assert s[0] == 39.953125 / 3


def test_head_selection_and_score_by_hand():
    # importance |a0| + |a1| + range * |a2|, nodes of range 1 never chosen:
    #   v0: 1 + 0 + 4 * 0.5 = 3;  v1: 2 + 1 + 2 * 0 = 3 (ties v0: v0 first)
    #   v2: range 1 (excluded);   v3: 0.5 + 0.5 + 8 * 0.5 = 5;  v4: 0 + 1 + 0 = 1
    A = np.array([[1.0, 0.0, 0.5, 0.0],
                  [-2.0, 1.0, 0.0, 0.0],
                  [0.0, 0.0, 1.0, 0.0],
                  [0.5, 0.5, 0.5, 0.0],
                  [0.0, -1.0, 0.0, 0.0]])
    rng_v = np.array([4, 2, 1, 8, 3])
    assert S.head_select(A, rng_v, 1) == [3]
    assert S.head_select(A, rng_v, 3) == [3, 0, 1]
    assert S.head_select(A, rng_v, 10) == [3, 0, 1, 4]
    r = np.array([[2.0, 1.0, 1.0, 4.0, 3.0],    # t = (1/2, 1/2, 1, 1/2, 1)
                  [4.0, 2.0, 1.0, 8.0, 1.0]])   # t = (1, 1, 1, 1, 1/3)
    # candidate 0 over {3, 0, 1}: v3 0.25 + 0.125 + 1 = 1.375, v0 0.5 + 1 = 1.5,
    # v1 -1 + 0.25 = -0.75: 2.125 / 5.  Candidate 1: v3 1.5, v0 1.5, v1 -1: 2 / 5.
    assert np.allclose(S.head_scores(A, r, rng_v, [3, 0, 1]), [2.125 / 5, 2.0 / 5], rtol=0, atol=1e-15)
    # one node: v3 only; all four: v4 adds -t^2 (-1 and -1/9)
    assert np.allclose(S.head_scores(A, r, rng_v, [3]), [1.375 / 5, 1.5 / 5], rtol=0, atol=1e-15)
    assert np.allclose(S.head_scores(A, r, rng_v, [3, 0, 1, 4]), [1.125 / 5, (2.0 - 1.0 / 9) / 5],
                       rtol=0, atol=1e-15)
    # with every node chosen the head score is the full score
    full = S.head_scores(A, r, rng_v, [0, 1, 2, 3, 4])
    assert np.allclose(full, S.scores(A, r, rng_v), rtol=1e-15, atol=0)
