"""Pins for the oracle's product-graph planner (Sec. 3.2): least-cost paths
on the product of a transition system and a monitor whose missing moves mark
bad prefixes.

  - scipy's Dijkstra (an independent library routine) on the product graph
    written out as a sparse matrix gives the same distances;
  - a monitor that accepts everything reduces the product to the transition
    system itself: distances equal scipy's on (V, E);
  - the predecessor of every reached vertex ends a least-cost path and is the
    smallest such product edge id (checked edge by edge in numpy), and
    following predecessors leads back to the start;
  - the split_lane example of Sec. 3.2 (never two consecutive lane splits):
    the paths found never split twice in a row, cost at least the
    unconstrained optimum, and a small graph where the cheapest path splits
    twice is forced onto the detour;
  - invalid inputs are rejected.
"""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph

import oracle

REJ = 0xFF
INF = 0xFFFFFFFF


def split_lane_monitor():
    """Monitor of G(split -> X not split) over one proposition: state 1 means
    the last transition split lanes; a second split in a row has no move."""
    # delta[(q << 1) | sigma]
    return np.array([0, 1, 0, REJ], np.uint8)


def random_system(rng, n_v, n_e, n_props, max_cost=20, p_label=0.3):
    src = rng.integers(0, n_v, n_e).astype(np.uint32)
    dst = rng.integers(0, n_v, n_e).astype(np.uint32)
    cost = rng.integers(1, max_cost + 1, n_e).astype(np.uint32)
    L = (rng.uniform(size=(n_e, n_props)) < p_label).astype(np.uint8)
    return src, dst, cost, L


def random_monitor(rng, n_states, n_props, p_reject=0.2):
    d = rng.integers(0, n_states, n_states << n_props).astype(np.uint8)
    d[rng.uniform(size=len(d)) < p_reject] = REJ
    return d


def product_matrix(n_v, src, dst, cost, L, delta):
    n_props = L.shape[1]
    Q = len(delta) >> n_props
    sig = (L != 0).astype(np.int64) @ (1 << np.arange(n_props))
    best = {}
    for e in range(len(src)):
        for q in range(Q):
            q2 = delta[(q << n_props) | sig[e]]
            if q2 >= Q:
                continue
            k = (int(src[e]) * Q + q, int(dst[e]) * Q + int(q2))
            best[k] = min(best.get(k, 1 << 62), int(cost[e]))
    n = n_v * Q
    if not best:
        return scipy.sparse.csr_matrix((n, n)), Q
    r, c = zip(*best.keys())
    return scipy.sparse.csr_matrix((list(best.values()), (r, c)), shape=(n, n)), Q


def scipy_dist(M, start):
    d = scipy.sparse.csgraph.dijkstra(M, directed=True, indices=start)
    return np.where(np.isinf(d), INF, d).astype(np.uint64)


def check_pred(n_v, src, dst, cost, L, delta, v0, q0, dist, pred):
    n_props = L.shape[1]
    Q = len(delta) >> n_props
    sig = (L != 0).astype(np.int64) @ (1 << np.arange(n_props))
    start = v0 * Q + q0
    want = np.full(n_v * Q, INF, np.uint64)
    for e in range(len(src)):
        for q in range(Q):
            fr = int(src[e]) * Q + q
            q2 = delta[(q << n_props) | sig[e]]
            if dist[fr] == INF or q2 >= Q:
                continue
            to = int(dst[e]) * Q + int(q2)
            if to != start and int(dist[fr]) + int(cost[e]) == int(dist[to]):
                want[to] = min(want[to], e * Q + q)
    assert np.array_equal(pred.astype(np.uint64), want)
    # predecessors lead back to the start
    for v in np.nonzero(dist != INF)[0]:
        x, steps = int(v), 0
        while x != start:
            p = int(pred[x])
            e, q = divmod(p, Q)
            x = int(src[e]) * Q + q
            steps += 1
            assert steps <= n_v * Q


@pytest.mark.parametrize("seed,n_v,n_e,n_props,Q", [(0, 30, 90, 1, 2), (1, 50, 200, 2, 3), (2, 80, 400, 3, 4),
                                                    (3, 20, 40, 1, 1), (4, 60, 300, 2, 8)])
def test_matches_scipy_dijkstra_on_product(seed, n_v, n_e, n_props, Q):
    rng = np.random.default_rng(seed)
    src, dst, cost, L = random_system(rng, n_v, n_e, n_props)
    delta = random_monitor(rng, Q, n_props)
    q0 = int(rng.integers(0, Q))
    v0 = int(src[np.argmax(np.bincount(src))])  # a vertex with many transitions
    dist, pred = oracle.product_paths(n_v, src, dst, cost, L, delta, v0, q0)
    M, _ = product_matrix(n_v, src, dst, cost, L, delta)
    assert np.array_equal(dist.astype(np.uint64), scipy_dist(M, v0 * Q + q0))
    assert (dist != INF).sum() > 1
    check_pred(n_v, src, dst, cost, L, delta, v0, q0, dist, pred)


def test_accept_all_monitor_is_the_transition_system():
    rng = np.random.default_rng(7)
    n_v = 200
    src, dst, cost, L = random_system(rng, n_v, 1200, 2)
    delta = np.zeros(1 << 2, np.uint8)  # one state, every label moves to it
    dist, pred = oracle.product_paths(n_v, src, dst, cost, L, delta, 5, 0)
    best = {}
    for a, b, c in zip(src, dst, cost):
        best[(int(a), int(b))] = min(best.get((int(a), int(b)), 1 << 62), int(c))
    r, c = zip(*best.keys())
    M = scipy.sparse.csr_matrix((list(best.values()), (r, c)), shape=(n_v, n_v))
    assert np.array_equal(dist.astype(np.uint64), scipy_dist(M, 5))
    check_pred(n_v, src, dst, cost, L, delta, 5, 0, dist, pred)


def path_edges(src, Q, pred, start, x):
    out = []
    while x != start:
        e, q = divmod(int(pred[x]), Q)
        out.append(e)
        x = int(src[e]) * Q + q
    return out[::-1]


def test_split_lane_paths_never_split_twice():
    rng = np.random.default_rng(11)
    n_v = 300
    src, dst, cost, L = random_system(rng, n_v, 2400, 1, p_label=0.5)
    delta = split_lane_monitor()
    dist, pred = oracle.product_paths(n_v, src, dst, cost, L, delta, 0, 0)
    free, _ = oracle.product_paths(n_v, src, dst, cost, L, np.zeros(2, np.uint8), 0, 0)
    reached = 0
    for v in range(n_v):
        for q in range(2):
            x = v * 2 + q
            if dist[x] == INF:
                continue
            reached += 1
            assert dist[x] >= free[v]
            es = path_edges(src, 2, pred, 0, x)
            assert sum(int(cost[e]) for e in es) == dist[x]
            splits = [int(L[e, 0]) for e in es]
            assert not any(a and b for a, b in zip(splits, splits[1:]))
            assert (splits[-1] if splits else 0) == q
    assert reached > n_v


def test_split_lane_detour():
    # 0 -split-> 1 -split-> 3 costs 2; the detour 0 -split-> 1 -> 2 -> 3 costs 3
    src = np.array([0, 1, 1, 2], np.uint32)
    dst = np.array([1, 3, 2, 3], np.uint32)
    cost = np.array([1, 1, 1, 1], np.uint32)
    L = np.array([[1], [1], [0], [0]], np.uint8)
    dist, pred = oracle.product_paths(4, src, dst, cost, L, split_lane_monitor(), 0, 0)
    free, _ = oracle.product_paths(4, src, dst, cost, L, np.zeros(2, np.uint8), 0, 0)
    assert free[3] == 2
    assert dist[3 * 2 + 0] == 3 and dist[3 * 2 + 1] == INF
    assert path_edges(src, 2, pred, 0, 3 * 2 + 0) == [0, 2, 3]


def test_rejects_invalid_edges():
    L = np.zeros((1, 1), np.uint8)
    with pytest.raises(ValueError):
        oracle.product_paths(2, [0], [2], [1], L, np.zeros(2, np.uint8), 0, 0)
    with pytest.raises(ValueError):
        oracle.product_paths(2, [0], [1], [0], L, np.zeros(2, np.uint8), 0, 0)
