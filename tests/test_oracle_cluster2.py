"""Pins for CLUSTER2 (Algorithm 2, Section 4) in the C oracle.

* Equality with the brute force that builds every contracted graph with
  Procedure Contract2 (rescaled edges d_u + w - 2R_CL) and takes each state
  from Floyd-Warshall distances over edges of weight <= 2R_CL.
* Properties the paper states or the construction implies: D is the length of
  a path from the center (so D >= dist(c, v)); a cluster grows by at most
  2R_CL per iteration; a node at light distance d from a center drawn in
  iteration j is assigned by iteration j + ceil(d / 2R_CL) - 1; the estimate
  is conservative; with R_CL = 0 every node is a singleton."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle
from oracle import brute

from test_oracle_pins import FAMILIES, _edges, _scipy_graph


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f for f, _ in FAMILIES])
@pytest.mark.parametrize("tau,seed", [(1, 1), (2, 5)])
def test_cluster2_equals_explicit_contract2(name, g, tau, seed):
    dec = oracle.decompose_cluster2(g, tau, seed)
    ref = brute.cluster2(g.n, _edges(g), tau, seed)
    assert dec.cluster.tolist() == [int(c) for c in ref["cluster"]], name
    assert dec.D.tolist() == [int(d) for d in ref["D"]], name
    assert dec.work["radius1"] == ref["radius1"]
    assert dec.delta_end == ref["delta2"] and dec.stages == ref["iterations"]
    assert dec.num_clusters == ref["num_clusters"] and dec.radius == ref["radius"]


def test_cluster2_radius1_is_cluster_radius():
    for name, g in FAMILIES[:8]:
        assert oracle.decompose_cluster2(g, 1, 3).work["radius1"] == oracle.decompose(g, 1, 3).radius


@pytest.mark.parametrize("name,g", FAMILIES[::3], ids=[f for f, _ in FAMILIES[::3]])
def test_cluster2_path_bounds(name, g):
    dec = oracle.decompose_cluster2(g, 1, 9)
    d2 = dec.delta_end
    dist = csgraph.dijkstra(_scipy_graph(g), directed=False)
    for v in range(g.n):
        c = int(dec.cluster[v])
        assert dec.cluster[c] == c
        assert dist[c, v] <= int(dec.D[v])                   # D is a path length from the center
    assert dec.radius <= d2 * dec.stages                      # at most 2R_CL per iteration
    assert dec.work["radius1"] * 2 == d2


@pytest.mark.parametrize("name,g", FAMILIES[:12:2], ids=[f for f, _ in FAMILIES[:12:2]])
def test_cluster2_light_distance_reach(name, g):
    """A node at light distance d > 0 from a center drawn in iteration j is
    assigned no later than iteration j + ceil(d / 2R_CL) - 1 (the property the
    diameter bound rests on)."""
    dec = oracle.decompose_cluster2(g, 1, 4)
    d2 = dec.delta_end
    if d2 == 0:
        return
    u, v, w = g.edges()
    keep = w <= d2
    light = sp.coo_matrix((w[keep].astype(np.float64), (u[keep], v[keep])), shape=(g.n, g.n)).tocsr()
    ld = csgraph.dijkstra(light, directed=False)
    # birth iteration of each center (replaying the draws) and assignment
    # iteration of each node: a node reached in iteration i by a cluster born
    # in j has D = d + 2R_CL (i - j) with 0 < d <= 2R_CL
    centers = [c for c in range(g.n) if dec.cluster[c] == c]
    assigned = {}
    birth = {}
    n = g.n
    iters = dec.stages
    U = set(range(n))
    k0 = 4
    for i in range(1, iters + 1):
        p = 2.0 ** i / n
        T = (1 << 32) if p >= 1.0 else math.floor(p * 4294967296.0)
        for x in sorted(U):
            if oracle.philox4x32_10((x, i, 0, 1), (k0, 0))[0] < T and dec.cluster[x] == x:
                birth[x] = i
        for x in list(U):
            c = int(dec.cluster[x])
            if c in birth:
                local = int(dec.D[x]) - d2 * (i - birth[c])
                if 0 <= local <= d2 and (x == c or local > 0):
                    assigned[x] = i
        U -= set(assigned)
    assert set(birth) == set(centers)
    for c in centers:
        for x in range(n):
            d = ld[c, x]
            if x == c or not np.isfinite(d):
                continue
            assert assigned[x] <= birth[c] + math.ceil(d / d2) - 1 or assigned[x] < birth[c], (c, x)


def test_cluster2_estimate_is_conservative():
    for name, g in FAMILIES[:10]:
        dec = oracle.decompose_cluster2(g, 1, 2)
        est = oracle.estimate(oracle.quotient(g, dec), dec)
        dist = csgraph.dijkstra(_scipy_graph(g), directed=False)
        phi = dist[np.isfinite(dist)].max()
        assert est.phi_approx >= phi


def test_cluster2_zero_radius_gives_singletons():
    g = graphgen.grid(5, 5, 10, 1)      # ceil(8 log2 n) > n: CLUSTER makes singletons, R_CL = 0
    dec = oracle.decompose_cluster2(g, 1, 1)
    assert dec.work["radius1"] == 0 and dec.delta_end == 0
    assert dec.cluster.tolist() == list(range(g.n)) and int(dec.D.max()) == 0


def test_cluster2_single_node():
    g = graphgen.csr_from_edges_np(1, [], [], [])
    dec = oracle.decompose_cluster2(g, 1, 1)
    assert dec.cluster.tolist() == [0] and dec.stages == 0
