"""Writes the oracle's results and work counts for the benchmark workloads.

Calls only graphgen (inputs) and oracle/ (results).  The JSON it writes holds
expected values for the full-size workload (cluster count, stages, Delta,
estimate, per-stage counts) and the work counts from which the algorithmic
bytes of one decomposition and one quotient build are computed.

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
                          "weights uniform in [1, 1e4], graph seed 1"),
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
        path = os.path.join(HERE, f"{name}_counts.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, out["num_clusters"], out["phi_approx"], out["oracle_seconds"])


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
