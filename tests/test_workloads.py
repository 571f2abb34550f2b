"""The evaluation-style input generator (Section 5.1's setups) produces the
shapes its docstring states: one source as the first layer, later layers of
2..P nodes, the layer count in range, a single sink, loads of the stated mean
with p = C_hat, acyclic and seeded (the same DAGs on every call)."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("P,depth", [(4, (5, 8)), (10, (5, 8)), (32, (12, 12))])
def test_paper_style_shapes(P, depth):
    c_avg = 20
    batch = W.paper_style(200, P, c_avg, depth=depth)
    loads = []
    for d in range(batch.num_dags):
        n, src, dst, w, p = batch.dag(d)
        assert np.array_equal(w, p)                     # m^max = C_hat
        assert w.min() >= 1 and w.max() <= 2 * c_avg - 1
        loads.append(w)
        indeg = np.bincount(dst, minlength=n)
        outdeg = np.bincount(src, minlength=n)
        assert np.count_nonzero(indeg == 0) == 1 and indeg[0] == 0   # one source, node 0
        assert np.count_nonzero(outdeg == 0) == 1 and outdeg[n - 1] == 0  # one sink, the last node
        assert np.all(src < dst)                         # ids in layer order: acyclic
        # layer of each node: the source is layer 0, a node is one past its deepest predecessor
        layer = np.zeros(n, np.int64)
        for u, v in sorted(zip(src.tolist(), dst.tolist()), key=lambda e: e[1]):
            layer[v] = max(layer[v], layer[u] + 1)
        inner = layer[1:n - 1]
        widths = np.bincount(inner)[1:]
        assert depth[0] <= len(widths) + 1 <= depth[1]
        assert widths.min() >= 2 and widths.max() <= P
    mean = np.concatenate(loads).mean()
    assert abs(mean - c_avg) < 1.0
    again = W.paper_style(200, P, c_avg, depth=depth)
    assert np.array_equal(again.src, batch.src) and np.array_equal(again.wcet, batch.wcet)
