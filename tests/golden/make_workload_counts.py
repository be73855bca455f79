"""Writes the oracle's results and work counts for the benchmark workloads.

Calls only graphgen (inputs) and oracle/ (results).  The JSON files it writes
hold expected values for the full-size workloads, compared bit for bit by the
GPU tests:

  road4096   the road-like 4096x4096 mesh: decomposition (cluster and D
             digests, per-stage counts), quotient graph (digests of its
             centers and symmetric CSR), estimate, and the work counts from
             which the algorithmic bytes of one decomposition and one quotient
             build are computed; the same for CLUSTER2 and the literal
             step-synchronous variant (with its round and work counters); the
             Delta-stepping competitor's distances from its source rule
  rmat24     R-MAT scale 24: decomposition, quotient graph, estimate, work
  rgg256     the batch of 256 random geometric graphs: every graph's
             decomposition, quotient size and estimate
  serve2000  the 2,000-request serving mix: for every resident graph, two
             sampled requests (the first and the last that use it) with their
             request seeds: decomposition and estimate
  mesh29     the 2^29-node mesh with 2.16G arcs (64-bit row offsets):
             decomposition, quotient graph, estimate (takes minutes and about
             50 GB of host memory; not in the default list)

Run:  python tests/golden/make_workload_counts.py [workload ...]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

TEXT = {
    "road4096": "road-like 4096x4096 mesh, 5% edges dropped, 1% diagonals, largest component, "
                "weights uniform in [1, 1e4], graph seed 1",
    "rmat24": "R-MAT scale 24, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, simple, "
              "largest component, weights uniform in [1, 2^20], graph seed 1",
    "mesh29": "16384x32768 mesh (2^29 nodes) with 1% diagonals, weights uniform in [1, 1e4], graph seed 1, "
              "64-bit row offsets",
}


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def quotient_digests(q) -> dict:
    """Digests of the quotient graph as the library lays it out: centers
    (int32), symmetric CSR row offsets (int64), columns (int32), weights (u64)."""
    rp, col, w = q.csr()
    return dict(center=digest(q.center.astype(np.int32)), row_ptr=digest(rp.astype(np.int64)),
                col=digest(col.astype(np.int32)), w=digest(w.astype(np.uint64)))


def decomposition_entry(dec, q, est) -> dict:
    return dict(stages=dec.stages, levels=dec.levels, delta0=dec.delta0, delta_end=dec.delta_end,
                num_clusters=dec.num_clusters, singletons=dec.singletons, radius=dec.radius,
                quotient_k=q.k, quotient_edges=int(len(q.ea)), phi_gc=est.phi_gc, phi_approx=est.phi_approx,
                cluster_sha256=digest(dec.cluster), D_sha256=digest(dec.D), quotient_sha256=quotient_digests(q))


def single(name, g, tau, seed, variants=False, sssp=False):
    t0 = time.time()
    dec = oracle.decompose(g, tau, seed)
    q = oracle.quotient(g, dec)
    est = oracle.estimate(q, dec)
    t1 = time.time()
    ab = oracle.algorithmic_bytes(g, dec, q)
    out = dict(workload=name, text=TEXT[name], tau=tau, seed=seed, n=g.n, m_arcs=g.m,
               edges=g.m // 2, stages=dec.stages, levels=dec.levels, delta0=dec.delta0,
               delta_end=dec.delta_end, num_clusters=dec.num_clusters, singletons=dec.singletons,
               radius=dec.radius, stage_uncovered=dec.stage_uncovered, stage_centers=dec.stage_centers,
               stage_covered=dec.stage_covered, stage_delta=dec.stage_delta, work=dec.work,
               quotient_k=q.k, quotient_edges=int(len(q.ea)), inter_cluster_edges=q.pairs,
               phi_gc=est.phi_gc, phi_approx=est.phi_approx,
               bytes_decompose=ab["decompose"], bytes_quotient=ab["quotient"],
               cluster_sha256=digest(dec.cluster), D_sha256=digest(dec.D),
               quotient_sha256=quotient_digests(q), oracle_seconds=round(t1 - t0, 2))
    if variants:
        t2 = time.time()
        d2 = oracle.decompose_cluster2(g, tau, seed)
        q2 = oracle.quotient(g, d2)
        e2 = oracle.estimate(q2, d2)
        out["cluster2"] = dict(stages=d2.stages, delta_end=d2.delta_end, num_clusters=d2.num_clusters,
                               radius=d2.radius, radius1=d2.work["radius1"], quotient_k=q2.k,
                               quotient_edges=int(len(q2.ea)),
                               phi_gc=e2.phi_gc, phi_approx=e2.phi_approx, cluster_sha256=digest(d2.cluster),
                               D_sha256=digest(d2.D), quotient_sha256=quotient_digests(q2),
                               oracle_seconds=round(time.time() - t2, 2))
        t3 = time.time()
        d3 = oracle.decompose_steps(g, tau, seed)
        q3 = oracle.quotient(g, d3)
        e3 = oracle.estimate(q3, d3)
        out["steps"] = dict(stages=d3.stages, levels=d3.levels, delta_end=d3.delta_end,
                            num_clusters=d3.num_clusters, radius=d3.radius, rounds=d3.work["rounds"],
                            messages=d3.work["messages"], updates=d3.work["updates"], quotient_k=q3.k,
                            quotient_edges=int(len(q3.ea)),
                            phi_gc=e3.phi_gc, phi_approx=e3.phi_approx, cluster_sha256=digest(d3.cluster),
                            D_sha256=digest(d3.D), quotient_sha256=quotient_digests(q3),
                            oracle_seconds=round(time.time() - t3, 2))
    if sssp:
        t4 = time.time()
        src = oracle.sssp_source(g.n, seed)
        dist, mx = oracle.sssp(g, src)
        out["sssp"] = dict(source=src, max_dist=mx, two_approx=2 * mx, dist_sha256=digest(dist),
                           oracle_seconds=round(time.time() - t4, 2))
    return out


def rgg256():
    graphs = graphgen.rgg_batch(256, seed=1)
    t0 = time.time()
    rows = []
    for i, g in enumerate(graphs):
        seed = (i << 32) | 1
        dec = oracle.decompose(g, 1, seed)
        q = oracle.quotient(g, dec)
        est = oracle.estimate(q, dec)
        rows.append(dict(graph=i, seed=seed, n=g.n, m_arcs=g.m, **decomposition_entry(dec, q, est)))
    return dict(workload="rgg256", text="256 random geometric graphs (graphgen.rgg_batch(256, seed=1)), sizes "
                "log-uniform in [1e3, 1e6], average degree 8, w = round(1e4*len)+1, largest components; "
                "tau=1, seed of graph g = (g << 32) | 1", tau=1, graphs=rows,
                nodes=sum(g.n for g in graphs), arcs=sum(g.m for g in graphs),
                oracle_seconds=round(time.time() - t0, 2))


def serve_key(r):
    """Resident graph of a request: meshes quantised to sides that are
    multiples of 256, R-MAT scales 12..22."""
    return f"grid{max(256, (r.size // 256) * 256)}" if r.kind == "grid" else f"rmat{r.size}"


def serve_graph(key):
    if key.startswith("grid"):
        s = int(key[4:])
        return graphgen.grid(s, s, 10000, s)
    return graphgen.rmat(int(key[4:]), seed=int(key[4:]))


def serve2000():
    reqs = graphgen.serving_mix(2000, rate=200.0, seed=1)
    by_key = {}
    for r in reqs:
        by_key.setdefault(serve_key(r), []).append(r.rid)
    t0 = time.time()
    rows = []
    for key in sorted(by_key):
        g = serve_graph(key)
        rids = sorted({by_key[key][0], by_key[key][-1]})
        for rid in rids:
            dec = oracle.decompose(g, 1, rid)
            q = oracle.quotient(g, dec)
            est = oracle.estimate(q, dec)
            e = decomposition_entry(dec, q, est)
            del e["quotient_sha256"]
            rows.append(dict(graph=key, rid=rid, seed=rid, n=g.n, m_arcs=g.m, **e))
    return dict(workload="serve2000", text="graphgen.serving_mix(2000, rate=200, seed=1); resident graphs: "
                "grid{s} = graphgen.grid(s, s, 10000, s) with the side rounded down to a multiple of 256, "
                "rmat{S} = graphgen.rmat(S, seed=S); tau=1, seed = request id; two sampled requests per graph",
                tau=1, requests=len(reqs), resident_graphs=len(by_key), samples=rows,
                oracle_seconds=round(time.time() - t0, 2))


def mesh29():
    g = graphgen.mesh29(1)
    return single("mesh29", g, 4, 1)


MAKERS = {
    "road4096": lambda: single("road4096", graphgen.road_like(4096, 1), 4, 1, variants=True, sssp=True),
    "rmat24": lambda: single("rmat24", graphgen.rmat(24, seed=1), 4, 1),
    "rgg256": rgg256,
    "serve2000": serve2000,
    "mesh29": mesh29,
}
DEFAULT = ["road4096", "rmat24", "rgg256", "serve2000"]


def main(names):
    for name in names:
        out = MAKERS[name]()
        path = os.path.join(HERE, f"{name}_counts.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, out.get("oracle_seconds"), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or DEFAULT)
