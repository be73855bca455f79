"""Brute-force checkers for tiny graphs, TEST INFRASTRUCTURE ONLY.

Pure Python, written to be read against the paper (arXiv:1506.03265) rather
than to be fast.  Unlike the C oracle, CLUSTER here builds every contracted
graph G_i explicitly with Procedure Contract (Section 3) and finds each node's
state from all-pairs distances of G_i (Floyd-Warshall).  It can also run the
Delta-growing steps literally, as synchronous Bellman-Ford rounds.  These are
the pins for the C oracle's implicit contraction and its Dijkstra growth.
"""
from __future__ import annotations

import math

import numpy as np

INF = float("inf")
M32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
    multiplications, with a Weyl-sequence key schedule."""
    c0, c1, c2, c3 = (int(x) & M32 for x in ctr)
    k0, k1 = (int(x) & M32 for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c3 ^ k1) & M32, p0 & M32
    return c0, c1, c2, c3


def floyd_warshall(nodes, adj):
    """All-pairs distances over `nodes` with adjacency dict adj[u][v] = w
    (Floyd-Warshall; one vectorised relaxation through each middle node)."""
    idx = {v: i for i, v in enumerate(nodes)}
    k = len(nodes)
    d = np.full((k, k), INF)
    np.fill_diagonal(d, 0.0)
    for u, nb in adj.items():
        for v, w in nb.items():
            a, b = idx[u], idx[v]
            d[a, b] = min(d[a, b], float(w))
    for m in range(k):
        d = np.minimum(d, d[:, m:m + 1] + d[m:m + 1, :])
    return idx, d


def _add_edge(adj, u, v, w):
    """Undirected edge, keeping the lightest of parallel copies."""
    if v not in adj[u] or w < adj[u][v]:
        adj[u][v] = w
        adj[v][u] = w


def growing_steps(nodes, adj, X, delta, state, literal_ties=False):
    """Repeats the Delta-growing step of Section 3 until no state changes.

    state[v] = (d, c) with d = INF, c = None when unset.  One step, in
    parallel: every node u with d_u < Delta offers (d_u + w, c_u) to each
    light neighbour v when d_u + w <= Delta and d_v > d_u + w; v takes the
    offer with the smallest distance, then the smallest center.  With
    literal_ties=False an offer at equal distance and smaller center also
    wins (the lexicographic reading).  Returns the number of steps that
    changed some state."""
    steps = 0
    while True:
        offers = {}
        for u in nodes:
            du, cu = state[u]
            if du >= delta:
                continue
            for v, w in adj[u].items():
                if w > delta or du + w > delta:
                    continue
                cand = (du + w, cu)
                dv, cv = state[v]
                better = cand[0] < dv if literal_ties else (cv is None or cand < (dv, cv))
                if better and (v not in offers or cand < offers[v]):
                    offers[v] = cand
        if not offers:
            return steps
        for v, cand in offers.items():
            state[v] = cand
        steps += 1


def cluster(n, edges, tau, seed, delta0=0, mode="apsp"):
    """CLUSTER(G, tau) of Algorithm 1 with an explicit Contract after every
    stage.  mode="apsp": each node's state is the lexicographic minimum over
    X of (dist_Gi(x, v), x) restricted to dist <= Delta; mode="steps": literal
    Delta-growing steps (lexicographic ties); mode="steps_literal": the
    paper's literal tie rule (distances are then compared only).

    Returns dict(cluster, D, stages, delta_end, num_clusters, radius, levels)."""
    gamma = 4.0 * math.log(2.0)
    L = math.log2(n)
    stop = math.ceil(8.0 * tau * L)
    m_arcs = 2 * len(edges)
    if delta0:
        delta = delta0
    else:
        delta = max(1, (2 * sum(w for _, _, w in edges)) // m_arcs) if m_arcs else 1
    k0, k1 = seed & M32, (seed >> 32) & M32

    # G_1 = G
    Vi = set(range(n))
    adj = {v: {} for v in range(n)}
    for u, v, w in edges:
        _add_edge(adj, u, v, w)
    Ci = set()
    cluster_of = [None] * n
    D = [0] * n
    R = [0] * n
    s = 0
    levels = 0
    while True:
        U = sorted(Vi - Ci)
        if n < 2 or not U or len(U) < stop:
            break
        p = gamma * tau * L / len(U)
        T = (1 << 32) if p >= 1.0 else math.floor(p * 4294967296.0)
        new = [v for v in U if philox4x32_10((v, s, 0, 0), (k0, k1))[0] < T]
        X = Ci | set(new)
        state = {v: ((0, v) if v in X else (INF, None)) for v in Vi}
        nodes = sorted(Vi)
        if mode == "apsp":
            idx, dist = floyd_warshall(nodes, adj)
        while True:
            levels += 1
            if mode == "apsp":
                for v in U:
                    best = (INF, None)
                    for x in X:
                        dxv = dist[idx[x], idx[v]]
                        if dxv <= delta and (dxv, x) < best:
                            best = (dxv, x)
                    if v not in X:
                        state[v] = best
            else:
                growing_steps(nodes, adj, X, delta, state, literal_ties=(mode == "steps_literal"))
            covered = [v for v in U if state[v][0] <= delta]
            if 2 * len(covered) >= len(U):
                break
            # can a larger Delta reach more uncovered nodes?
            reach = set(X) | set(covered)
            frontier_edge = any(v not in reach for u in reach for v in adj[u] if v in set(U))
            if not frontier_edge:
                break
            if 2 * delta > (1 << 31):
                raise OverflowError("Delta above 2^31")
            delta *= 2
        for v in covered:
            c = state[v][1]
            cluster_of[v] = c
            D[v] = state[v][0] + R[c]
        for v in covered:
            c = cluster_of[v]
            R[c] = max(R[c], D[v])
        # Procedure Contract
        clustered = set(X) | set(covered)
        label = {v: (v if v in X else state[v][1]) for v in clustered}
        nadj = {v: {} for v in Vi if v not in clustered or v in X}
        for u in Vi:
            for v, w in adj[u].items():
                if u > v:
                    continue
                cu, cv = label.get(u), label.get(v)
                if cu is not None and cv is not None:
                    continue
                if cu is None and cv is None:
                    _add_edge(nadj, u, v, w)
                elif cu is not None:
                    _add_edge(nadj, cu, v, w)
                else:
                    _add_edge(nadj, u, cv, w)
        Vi = set(nadj.keys())
        adj = nadj
        Ci = X
        s += 1
    for v in Vi - Ci:
        cluster_of[v] = v
        D[v] = 0
    return dict(cluster=cluster_of, D=D, stages=s, delta_end=delta,
                num_clusters=sum(1 for v in range(n) if cluster_of[v] == v),
                radius=max(D) if D else 0, levels=levels)


class MessageCount:
    """Counts the messages of the literal steps over the ORIGINAL graph (the
    paper's work counter: offers sent), independently of how the growth is
    computed.  In a step the active set A sends one offer over every original
    arc (u, v, w) with d_u + w <= Delta, where d_u is 0 for a node assigned in
    an earlier stage (Procedure Contract makes it part of its center) and its
    current distance otherwise.  A is the set of nodes updated by the previous
    step; the new centers join it when a stage starts; the nodes that sent at
    some step of the current Delta and had an arc with d_u + w > Delta (set B)
    join it whenever Delta doubles and when a stage ends (they may offer at the
    next Delta or, assigned, in the next stage)."""

    def __init__(self, n, edges):
        self.adj = {v: [] for v in range(n)}
        for u, v, w in edges:
            self.adj[u].append(w)
            self.adj[v].append(w)
        self.assigned = set()
        self.A, self.B = set(), set()
        self.messages = 0

    def step(self, state, delta):
        for u in self.A:
            du = 0 if u in self.assigned else state[u][0]
            assert du != INF, "an active node has a distance"
            for w in self.adj[u]:
                if du + w <= delta:
                    self.messages += 1
                else:
                    self.B.add(u)

    def release_blocked(self):
        self.A |= self.B
        self.B = set()


def partial_growth_steps(nodes, adj, delta, state, U, covered0, step_cap=0, msg=None):
    """Procedure PartialGrowth of Algorithm 1 taken literally: synchronous
    Delta-growing steps (every node u with d_u < Delta offers d_u + w to each
    neighbour over an edge with d_u + w <= Delta; v accepts only a strictly
    smaller distance, the smallest center winning among the offers of one
    step), repeated until a step updates no state or at least half of the
    uncovered nodes U have d <= Delta, or after step_cap steps (0 = no cap).
    With a MessageCount, every step's messages are counted before its offers
    are applied, and the step's updated nodes become its active set.

    Returns (steps executed, node updates, number of U nodes with d <= Delta,
    whether the last step updated some state)."""
    Uset = set(U)
    covered = covered0
    steps = updates = 0
    if 2 * covered >= len(U):
        return steps, updates, covered, False
    while True:
        if msg is not None:
            msg.step(state, delta)
        offers = {}
        for u in nodes:
            du, cu = state[u]
            if du >= delta:
                continue
            for v, w in adj[u].items():
                if du + w > delta:
                    continue
                cand = (du + w, cu)
                if cand[0] < state[v][0] and (v not in offers or cand < offers[v]):
                    offers[v] = cand
        steps += 1
        for v, cand in offers.items():
            if state[v][0] == INF and v in Uset:
                covered += 1
            state[v] = cand
        updates += len(offers)
        if msg is not None:
            msg.A = set(offers)
        if not offers or 2 * covered >= len(U) or (step_cap and steps >= step_cap):
            return steps, updates, covered, bool(offers)


def cluster_steps(n, edges, tau, seed, delta0=0, step_cap=0):
    """CLUSTER(G, tau) of Algorithm 1 with literal PartialGrowth (synchronous
    steps, the strict-distance tie rule, the per-step half-coverage stop with
    threshold |V_i - C_i| / 2, an optional cap on the steps of one
    PartialGrowth call) and Delta doubled one step at a time; explicit
    Contract after every stage.  A stage stops doubling when no uncovered
    node is reachable from the clusters at any Delta.

    Returns dict(cluster, D, stages, delta_end, num_clusters, radius, levels,
    rounds, updates, messages)."""
    gamma = 4.0 * math.log(2.0)
    L = math.log2(n)
    stop = math.ceil(8.0 * tau * L)
    m_arcs = 2 * len(edges)
    if delta0:
        delta = delta0
    else:
        delta = max(1, (2 * sum(w for _, _, w in edges)) // m_arcs) if m_arcs else 1
    k0, k1 = seed & M32, (seed >> 32) & M32
    Vi = set(range(n))
    adj = {v: {} for v in range(n)}
    for u, v, w in edges:
        _add_edge(adj, u, v, w)
    Ci = set()
    cluster_of = [None] * n
    D = [0] * n
    R = [0] * n
    s = levels = rounds = updates = 0
    msg = MessageCount(n, edges)
    while True:
        U = sorted(Vi - Ci)
        if n < 2 or not U or len(U) < stop:
            break
        p = gamma * tau * L / len(U)
        T = (1 << 32) if p >= 1.0 else math.floor(p * 4294967296.0)
        new = [v for v in U if philox4x32_10((v, s, 0, 0), (k0, k1))[0] < T]
        X = Ci | set(new)
        state = {v: ((0, v) if v in X else (INF, None)) for v in Vi}
        nodes = sorted(Vi)
        covered = len(new)
        msg.A |= set(new)
        while 2 * covered < len(U):
            levels += 1
            k, up, covered, moved = partial_growth_steps(nodes, adj, delta, state, U, covered, step_cap, msg)
            rounds += k
            updates += up
            if 2 * covered >= len(U):
                break
            reach = {v for v in Vi if state[v][0] != INF}
            if not moved and not any(v not in reach for u in reach for v in adj[u]):
                break
            if 2 * delta > (1 << 31):
                raise OverflowError("Delta above 2^31")
            delta *= 2
            msg.release_blocked()
        got = [v for v in U if state[v][0] <= delta]
        for v in got:
            c = state[v][1]
            cluster_of[v] = c
            D[v] = state[v][0] + R[c]
        for v in got:
            R[cluster_of[v]] = max(R[cluster_of[v]], D[v])
        msg.assigned |= set(got)
        msg.release_blocked()
        clustered = set(X) | set(got)
        label = {v: (v if v in X else state[v][1]) for v in clustered}
        nadj = {v: {} for v in Vi if v not in clustered or v in X}
        for u in Vi:
            for v, w in adj[u].items():
                if u > v:
                    continue
                cu, cv = label.get(u), label.get(v)
                if cu is not None and cv is not None:
                    continue
                if cu is None and cv is None:
                    _add_edge(nadj, u, v, w)
                elif cu is not None:
                    _add_edge(nadj, cu, v, w)
                else:
                    _add_edge(nadj, u, cv, w)
        Vi = set(nadj.keys())
        adj = nadj
        Ci = X
        s += 1
    for v in Vi - Ci:
        cluster_of[v] = v
        D[v] = 0
    return dict(cluster=cluster_of, D=D, stages=s, delta_end=delta,
                num_clusters=sum(1 for v in range(n) if cluster_of[v] == v),
                radius=max(D) if D else 0, levels=levels, rounds=rounds, updates=updates,
                messages=msg.messages)


def cluster2(n, edges, tau, seed, delta0=0):
    """CLUSTER2(G, tau) of Algorithm 2 with an explicit Contract2 after every
    iteration.  R_CL is the radius of cluster(..., mode="apsp"); every growth
    runs to its fixpoint with Delta2 = 2 R_CL, each node's state being the
    lexicographic minimum over X of (dist, x) where dist uses only edges of
    weight <= Delta2 and is at most Delta2 (Floyd-Warshall on G_i).  Contract2
    removes the grown nodes, keeps their centers, and replaces every edge
    (u, v) of weight <= Delta2 with c_u defined and c_v undefined by (c_u, v)
    of weight d_u + w - Delta2.  D of a node reached in iteration i by the
    cluster of a center drawn in iteration j is its G_i distance plus
    Delta2 (i - j).

    Returns dict(cluster, D, iterations, delta2, radius1, num_clusters,
    radius)."""
    r1 = cluster(n, edges, tau, seed, delta0=delta0, mode="apsp")["radius"]
    d2 = 2 * int(r1)
    if d2 > (1 << 31):
        raise OverflowError("2 R_CL above 2^31")
    k0, k1 = seed & M32, (seed >> 32) & M32
    iters = 0
    while (1 << iters) < n:
        iters += 1
    Vi = set(range(n))
    adj = {v: {} for v in range(n)}
    for u, v, w in edges:
        if w <= d2:
            _add_edge(adj, u, v, w)
    Ci = set()
    birth = {}
    cluster_of = [None] * n
    D = [0] * n
    for i in range(1, iters + 1):
        U = sorted(Vi - Ci)
        p = 2.0 ** i / n
        T = (1 << 32) if p >= 1.0 else math.floor(p * 4294967296.0)
        new = [v for v in U if philox4x32_10((v, i, 0, 1), (k0, k1))[0] < T]
        for v in new:
            birth[v] = i
        X = Ci | set(new)
        nodes = sorted(Vi)
        idx, dist = floyd_warshall(nodes, adj)
        state = {}
        for v in U:
            best = (INF, None)
            for x in X:
                dxv = dist[idx[x], idx[v]]
                if dxv <= d2 and (dxv, x) < best:
                    best = (dxv, x)
            state[v] = (0, v) if v in new else best
        got = [v for v in U if state[v][1] is not None]
        for v in got:
            d, c = state[v]
            cluster_of[v] = c
            D[v] = int(d) + d2 * (i - birth[c])
        # Procedure Contract2
        label = {v: state[v][1] for v in got}
        for x in Ci:
            label[x] = x
        nadj = {v: {} for v in Vi if v not in label or v in X}
        for u in Vi:
            for v, w in adj[u].items():
                if u > v:
                    continue
                cu, cv = label.get(u), label.get(v)
                if cu is not None and cv is not None:
                    continue
                if cu is None and cv is None:
                    _add_edge(nadj, u, v, w)
                    continue
                # the endpoint in a cluster (a) and the one outside it (b)
                a, b, ca = (u, v, cu) if cu is not None else (v, u, cv)
                da = 0 if a in Ci else int(state[a][0])
                nw = da + w - d2
                assert 1 <= nw <= d2
                _add_edge(nadj, ca, b, nw)
        Vi = set(nadj.keys())
        adj = nadj
        Ci = X
    for v in range(n):
        if cluster_of[v] is None:
            cluster_of[v] = v
            D[v] = 0
    return dict(cluster=cluster_of, D=D, iterations=iters, delta2=d2, radius1=int(r1),
                num_clusters=sum(1 for v in range(n) if cluster_of[v] == v), radius=max(D) if D else 0)


def quotient(n, edges, cluster_of, D):
    """Weighted quotient graph of Section 4 as a dict (a, b) -> weight over
    dense cluster indices a < b (clusters numbered by ascending center)."""
    centers = sorted(v for v in range(n) if cluster_of[v] == v)
    dense = {c: i for i, c in enumerate(centers)}
    q = {}
    for u, v, w in edges:
        cu, cv = cluster_of[u], cluster_of[v]
        if cu == cv:
            continue
        a, b = sorted((dense[cu], dense[cv]))
        x = w + D[u] + D[v]
        if (a, b) not in q or x < q[(a, b)]:
            q[(a, b)] = x
    return len(centers), q


def diameter(k, edge_dict):
    """Max finite pairwise distance, Floyd-Warshall."""
    adj = {v: {} for v in range(k)}
    for (a, b), w in edge_dict.items():
        _add_edge(adj, a, b, w)
    _, d = floyd_warshall(list(range(k)), adj)
    fin = d[np.isfinite(d)]
    return int(fin.max()) if fin.size else 0
