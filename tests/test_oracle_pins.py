"""Pins for the C oracle against brute force, closed forms and the paper's
invariants (CPU only).

* Decomposition: the C oracle (implicit Contract, lexicographic Dijkstra)
  must equal the brute force that builds every contracted graph G_i with
  Procedure Contract and takes each state from Floyd-Warshall distances, and
  the brute force that runs the Delta-growing steps literally (Section 3,
  Algorithm 1).
* One growth level: literal steps with the paper's tie rule give the same
  distances as the lexicographic rule and as the closed form.
* Special case: when ceil(8 tau log2 n) > n every node is a singleton, G_C = G
  and Phi_approx = Phi(G) exactly (scipy Floyd-Warshall).
* Invariants of Algorithm 1 and Section 4 on larger inputs.
* Quotient, diameter and SSSP against scipy / dict brute force.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle
from oracle import brute


def _edges(g):
    u, v, w = g.edges()
    return [(int(a), int(b), int(c)) for a, b, c in zip(u, v, w)]


def _scipy_graph(g):
    return sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))


def _families():
    """Tiny graphs large enough for several stages (n >= ~100 at tau = 1)."""
    out = []
    rng = np.random.default_rng(12345)
    for i in range(24):
        n = int(rng.integers(90, 220))
        p = float(rng.choice([0.02, 0.04, 0.08]))
        wmax = int(rng.choice([1, 2, 5, 100, 10000]))
        out.append((f"er{i}", graphgen.random_small(rng, n, p, wmax, connected=bool(i % 3))))
    for side, wmax in ((10, 3), (12, 50), (14, 1), (15, 1000)):
        g = graphgen.grid(side, side, wmax, 7 + side)
        out.append((f"grid{side}", g))
    # path, cycle, star and a two-component graph with equal weights (ties)
    n = 150
    out.append(("path", graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [1] * (n - 1))))
    out.append(("cycle", graphgen.csr_from_edges_np(n, range(n), [(i + 1) % n for i in range(n)], [2] * n)))
    out.append(("star", graphgen.csr_from_edges_np(n, [0] * (n - 1), range(1, n), list(range(1, n)))))
    a = [(i, i + 1) for i in range(69)] + [(70 + i, 70 + i + 1) for i in range(69)]
    out.append(("twocomp", graphgen.csr_from_edges_np(140, [x for x, _ in a], [y for _, y in a], [1] * len(a))))
    return out


FAMILIES = _families()


def _assert_same(dec, ref, name):
    assert dec.cluster.tolist() == [int(c) for c in ref["cluster"]], name
    assert dec.D.tolist() == [int(d) for d in ref["D"]], name
    assert dec.stages == ref["stages"], name
    assert dec.delta_end == ref["delta_end"], name
    assert dec.num_clusters == ref["num_clusters"], name
    assert dec.radius == int(ref["radius"]), name
    assert dec.levels == ref["levels"], name


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f for f, _ in FAMILIES])
@pytest.mark.parametrize("tau,seed", [(1, 1), (1, 99), (2, 5)])
def test_decompose_equals_explicit_contract_apsp(name, g, tau, seed):
    dec = oracle.decompose(g, tau, seed)
    ref = brute.cluster(g.n, _edges(g), tau, seed, mode="apsp")
    _assert_same(dec, ref, name)


@pytest.mark.parametrize("name,g", FAMILIES[::3], ids=[f for f, _ in FAMILIES[::3]])
def test_decompose_equals_literal_growing_steps(name, g):
    dec = oracle.decompose(g, 1, 3)
    ref = brute.cluster(g.n, _edges(g), 1, 3, mode="steps")
    _assert_same(dec, ref, name)


@pytest.mark.parametrize("delta0", [1, 7, 10**6])
def test_decompose_explicit_initial_delta(delta0):
    g = FAMILIES[0][1]
    dec = oracle.decompose(g, 1, 11, delta0=delta0)
    ref = brute.cluster(g.n, _edges(g), 1, 11, delta0=delta0, mode="apsp")
    _assert_same(dec, ref, "er0")
    assert dec.delta0 == delta0


def test_stages_really_happen():
    """The family above must exercise several stages and Delta doublings."""
    stages = [oracle.decompose(g, 1, 1).stages for _, g in FAMILIES]
    levels = [oracle.decompose(g, 1, 1).levels for _, g in FAMILIES]
    assert max(stages) >= 2 and sum(s >= 1 for s in stages) >= len(stages) // 2
    assert max(l - s for l, s in zip(levels, stages)) >= 2


def test_single_level_literal_ties_same_distances():
    """One PartialGrowth: the paper's literal tie rule, the lexicographic rule
    and the closed form lexmin over X of (dist(x, v), x) agree on distances;
    labels agree between the lexicographic rule and the closed form."""
    rng = np.random.default_rng(3)
    for trial in range(30):
        g = graphgen.random_small(rng, 60, 0.06, int(rng.choice([1, 3, 20])), connected=True)
        edges = _edges(g)
        adj = {v: {} for v in range(g.n)}
        for u, v, w in edges:
            brute._add_edge(adj, u, v, w)
        X = sorted(set(int(x) for x in rng.choice(g.n, size=4, replace=False)))
        delta = int(rng.integers(1, 30))
        nodes = list(range(g.n))
        init = {v: ((0, v) if v in X else (brute.INF, None)) for v in nodes}
        lit = dict(init)
        lex = dict(init)
        brute.growing_steps(nodes, adj, X, delta, lit, literal_ties=True)
        brute.growing_steps(nodes, adj, X, delta, lex, literal_ties=False)
        idx, d = brute.floyd_warshall(nodes, adj)
        for v in nodes:
            best = min(((d[idx[x], idx[v]], x) for x in X if d[idx[x], idx[v]] <= delta),
                       default=(brute.INF, None))
            assert lit[v][0] == lex[v][0] == best[0]
            assert lex[v][1] == best[1]


def test_all_singletons_gives_exact_diameter():
    """ceil(8 tau log2 n) > n: CLUSTER makes every node a singleton, so G_C is
    G itself and Phi_approx = Phi(G) (Section 4)."""
    rng = np.random.default_rng(8)
    for trial in range(10):
        g = graphgen.random_small(rng, 40, 0.1, 1000, connected=True)
        dec = oracle.decompose(g, 1, trial)
        assert dec.stages == 0 and dec.num_clusters == g.n and dec.radius == 0
        q = oracle.quotient(g, dec)
        est = oracle.estimate(q, dec)
        dist = csgraph.floyd_warshall(_scipy_graph(g), directed=False)
        assert est.phi_approx == est.phi_gc == int(dist[np.isfinite(dist)].max())


def test_stop_threshold_boundary():
    """n = 64, tau = 1: STOP = 48 <= n, so exactly one kind of stage runs;
    the oracle must agree with brute force at this boundary."""
    n = 64
    g = graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [5] * (n - 1))
    assert math.ceil(8.0 * 1 * math.log2(n)) == 48
    for seed in range(1, 6):
        dec = oracle.decompose(g, 1, seed)
        ref = brute.cluster(n, _edges(g), 1, seed, mode="apsp")
        _assert_same(dec, ref, f"path64-{seed}")


def _check_invariants(g, tau, seed):
    dec = oracle.decompose(g, tau, seed)
    n = g.n
    cl = dec.cluster.astype(np.int64)
    # a partition whose centers belong to their own clusters
    assert cl.min() >= 0 and cl.max() < n
    centers = np.unique(cl)
    assert np.all(cl[centers] == centers)
    assert dec.num_clusters == len(centers)
    assert dec.num_clusters == sum(dec.stage_centers) + dec.singletons
    # stages: at least half covered (or nothing more reachable); Delta doubles
    L = math.log2(n)
    assert dec.stop == math.ceil(8.0 * tau * L)
    for s in range(dec.stages):
        # connected input: every uncovered node is reachable once a source exists
        if s > 0 or dec.stage_centers[s] > 0:
            assert 2 * dec.stage_covered[s] >= dec.stage_uncovered[s]
        ratio = dec.stage_delta[s] // dec.delta0
        assert dec.stage_delta[s] % dec.delta0 == 0 and ratio & (ratio - 1) == 0
        if s:
            assert dec.stage_delta[s] >= dec.stage_delta[s - 1]
            assert dec.stage_uncovered[s] == dec.stage_uncovered[s - 1] - dec.stage_covered[s - 1]
    last = dec.stage_uncovered[-1] - dec.stage_covered[-1] if dec.stages else n
    assert last == dec.singletons and (last < dec.stop or last == 0)
    # radius grows by at most Delta per stage (Section 3)
    assert dec.radius <= sum(dec.stage_delta)
    # D bounds the true distance to the center
    G = _scipy_graph(g)
    sample = centers if len(centers) <= 300 else np.random.default_rng(0).choice(centers, 300, replace=False)
    dist = csgraph.dijkstra(G, directed=False, indices=sample)
    for row, c in zip(dist, sample):
        members = np.nonzero(cl == c)[0]
        assert np.all(row[members] <= dec.D[members].astype(np.float64))
    return dec


def test_invariants_grid_small():
    dec = _check_invariants(graphgen.grid_small(), 1, 1)
    assert dec.stages >= 1


@pytest.mark.parametrize("seed", [1, 2])
def test_invariants_road_256(seed):
    _check_invariants(graphgen.road_like(256, seed), 1, seed)


def test_invariants_rmat_12():
    _check_invariants(graphgen.rmat(12, seed=3), 1, 3)


def test_estimate_is_conservative():
    """Phi_approx >= Phi(G) (Section 4), with Phi(G) from scipy APSP."""
    for g, tau in ((graphgen.grid_small(), 1), (graphgen.grid(40, 40, 10000, 9), 1), (graphgen.rmat(10, seed=4), 1)):
        dec = oracle.decompose(g, tau, 1)
        est = oracle.estimate(oracle.quotient(g, dec), dec)
        dist = csgraph.dijkstra(_scipy_graph(g), directed=False)
        phi = int(dist[np.isfinite(dist)].max())
        assert est.phi_approx >= phi
        assert dec.num_clusters < g.n


@pytest.mark.parametrize("name,g", FAMILIES[::2], ids=[f for f, _ in FAMILIES[::2]])
def test_quotient_equals_dict_min(name, g):
    dec = oracle.decompose(g, 1, 1)
    q = oracle.quotient(g, dec)
    k, ref = brute.quotient(g.n, _edges(g), dec.cluster.tolist(), [int(x) for x in dec.D])
    assert q.k == k
    assert list(zip(q.ea.tolist(), q.eb.tolist())) == sorted(ref.keys())
    assert q.ew.tolist() == [ref[key] for key in sorted(ref.keys())]
    assert np.all(q.ea < q.eb)
    assert q.center.tolist() == sorted(set(dec.cluster.tolist()))


def test_quotient_larger_graph_properties():
    g = graphgen.road_like(128, 5)
    dec = oracle.decompose(g, 1, 5)
    q = oracle.quotient(g, dec)
    k, ref = brute.quotient(g.n, _edges(g), dec.cluster.tolist(), [int(x) for x in dec.D])
    assert q.k == k and len(q.ea) == len(ref)
    assert all(q.ew[i] == ref[(int(q.ea[i]), int(q.eb[i]))] for i in range(len(q.ea)))


def test_diameter_equals_scipy():
    rng = np.random.default_rng(21)
    for trial in range(10):
        k = int(rng.integers(2, 60))
        g = graphgen.random_small(rng, k, 0.15, 10**9, connected=bool(trial % 2))
        ea, eb, ew = g.edges()
        phi = oracle.diameter_edges(k, ea, eb, ew.astype(np.uint64))
        dist = csgraph.floyd_warshall(_scipy_graph(g), directed=False)
        assert phi == int(dist[np.isfinite(dist)].max())
        if len(ea):
            assert phi == brute.diameter(k, {(int(a), int(b)): int(c) for a, b, c in zip(ea, eb, ew)})


@pytest.mark.parametrize("maker", [lambda: graphgen.grid_small(), lambda: graphgen.road_like(300, 2),
                                   lambda: graphgen.rmat(13, seed=2),
                                   lambda: graphgen.random_small(np.random.default_rng(1), 80, 0.02, 9)])
def test_sssp_equals_scipy_dijkstra(maker):
    g = maker()
    src = oracle.sssp_source(g.n, 1)
    dist, mx = oracle.sssp(g, src)
    ref = csgraph.dijkstra(_scipy_graph(g), directed=False, indices=src)
    fin = np.isfinite(ref)
    assert np.all(dist[~fin] == 0xFFFFFFFF)
    assert np.array_equal(dist[fin].astype(np.float64), ref[fin])
    assert mx == int(ref[fin].max())


def test_sssp_two_approximation_bounds_diameter():
    """max finite SSSP distance <= Phi(G) <= 2 * that (Section 1)."""
    g = graphgen.grid(30, 30, 500, 4)
    _, mx = oracle.sssp(g, oracle.sssp_source(g.n, 1))
    dist = csgraph.dijkstra(_scipy_graph(g), directed=False)
    phi = int(dist.max())
    assert mx <= phi <= 2 * mx


def test_default_delta_is_floor_of_mean_arc_weight():
    g = graphgen.grid_small()
    assert oracle.default_delta(g) == int(g.w.astype(np.int64).sum() // g.m)
    assert oracle.decompose(g, 1, 1).delta0 == oracle.default_delta(g)


def test_single_node_and_pair():
    for n in (1, 2):
        g = graphgen.csr_from_edges_np(n, [0] if n == 2 else [], [1] if n == 2 else [], [4] if n == 2 else [])
        dec = oracle.decompose(g, 1, 1)
        assert dec.stages == 0 and dec.num_clusters == n and dec.cluster.tolist() == list(range(n))
        ref = brute.cluster(n, _edges(g), 1, 1)
        _assert_same(dec, ref, f"n{n}")


def test_overflow_is_reported():
    n = 128
    g = graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [2**31] * (n - 1))
    with pytest.raises(oracle.OracleError) as e:
        oracle.decompose(g, 1, 1, delta0=2**31)
    assert e.value.code == oracle.OR_EOVERFLOW
