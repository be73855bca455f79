"""Writes the oracle's results and work counts for the benchmark workloads.

Calls only graphgen (inputs) and oracle/ (results).  The JSON it writes holds
expected values for the full-size workload (cluster count, stages, Delta,
estimate, per-stage counts) and the work counts from which the algorithmic
bytes of one decomposition and one quotient build are computed; for the
road-like mesh also the results of CLUSTER2 and of the literal
step-synchronous variant (with its round and work counters).

Run:  python tests/golden/make_workload_counts.py
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

WORKLOADS = {
    "road4096": dict(maker=lambda: graphgen.road_like(4096, 1), tau=4, seed=1,
                     text="road-like 4096x4096 mesh, 5% edges dropped, 1% diagonals, largest component, "
                          "weights uniform in [1, 1e4], graph seed 1", variants=True),
    "rmat24": dict(maker=lambda: graphgen.rmat(24, seed=1), tau=4, seed=1,
                   text="R-MAT scale 24, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, simple, "
                        "largest component, weights uniform in [1, 2^20], graph seed 1"),
}


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(names):
    for name in names:
        wl = WORKLOADS[name]
        g = wl["maker"]()
        t0 = time.time()
        dec = oracle.decompose(g, wl["tau"], wl["seed"])
        q = oracle.quotient(g, dec)
        est = oracle.estimate(q, dec)
        t1 = time.time()
        ab = oracle.algorithmic_bytes(g, dec, q)
        out = dict(workload=name, text=wl["text"], tau=wl["tau"], seed=wl["seed"], n=g.n, m_arcs=g.m,
                   edges=g.m // 2, stages=dec.stages, levels=dec.levels, delta0=dec.delta0,
                   delta_end=dec.delta_end, num_clusters=dec.num_clusters, singletons=dec.singletons,
                   radius=dec.radius, stage_uncovered=dec.stage_uncovered, stage_centers=dec.stage_centers,
                   stage_covered=dec.stage_covered, stage_delta=dec.stage_delta, work=dec.work,
                   quotient_k=q.k, quotient_edges=int(len(q.ea)), inter_cluster_edges=q.pairs,
                   phi_gc=est.phi_gc, phi_approx=est.phi_approx,
                   bytes_decompose=ab["decompose"], bytes_quotient=ab["quotient"],
                   cluster_sha256=digest(dec.cluster), D_sha256=digest(dec.D), oracle_seconds=round(t1 - t0, 2))
        if wl.get("variants"):
            t2 = time.time()
            d2 = oracle.decompose_cluster2(g, wl["tau"], wl["seed"])
            q2 = oracle.quotient(g, d2)
            e2 = oracle.estimate(q2, d2)
            out["cluster2"] = dict(stages=d2.stages, delta_end=d2.delta_end, num_clusters=d2.num_clusters,
                                   radius=d2.radius, radius1=d2.work["radius1"], quotient_k=q2.k,
                                   phi_gc=e2.phi_gc, phi_approx=e2.phi_approx, cluster_sha256=digest(d2.cluster),
                                   D_sha256=digest(d2.D), oracle_seconds=round(time.time() - t2, 2))
            t3 = time.time()
            d3 = oracle.decompose_steps(g, wl["tau"], wl["seed"])
            q3 = oracle.quotient(g, d3)
            e3 = oracle.estimate(q3, d3)
            out["steps"] = dict(stages=d3.stages, levels=d3.levels, delta_end=d3.delta_end,
                                num_clusters=d3.num_clusters, radius=d3.radius, rounds=d3.work["rounds"],
                                messages=d3.work["messages"], updates=d3.work["updates"], quotient_k=q3.k,
                                phi_gc=e3.phi_gc, phi_approx=e3.phi_approx, cluster_sha256=digest(d3.cluster),
                                D_sha256=digest(d3.D), oracle_seconds=round(time.time() - t3, 2))
        path = os.path.join(HERE, f"{name}_counts.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, out["num_clusters"], out["phi_approx"], out["oracle_seconds"])


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
