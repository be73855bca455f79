"""Full-size oracle parity for the batched and the served workloads.

Batched: the 256 random geometric graphs of the batch benchmark (37.2M nodes,
297M arcs) decomposed in one device job, under the default schedule and under
the schedule the tuner picks for this batch; every graph's cluster ids and
distance bounds are compared with the oracle's (SHA-256 digests), together
with its stage count, Delta, cluster count, radius, quotient size and
estimate.

Served: the 2,000-request Poisson mix at 200 requests/s (half meshes of side
256-2048, half R-MAT scale 12-22) through the stream-pool request loop with
the benchmark's four workers, against the same requests served one at a time:
every result is equal (tolerance 0), and the two sampled requests of every
resident graph match the oracle bit for bit.

Expected values were written by tests/golden/make_workload_counts.py, which
calls only the oracle."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen
import paper_1506_03265_amd as cd

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cd.load_library()


@pytest.mark.timeout(900)
def test_rgg256_batched_job_equals_oracle():
    counts = json.load(open(os.path.join(HERE, "golden", "rgg256_counts.json")))
    _say("[configs] generating the 256 random geometric graphs")
    graphs = graphgen.rgg_batch(256, seed=1)
    rows = counts["graphs"]
    assert [(g.n, g.m) for g in graphs] == [(r["n"], r["m_arcs"]) for r in rows]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    del graphs
    params = [(counts["tau"], r["seed"], 0) for r in rows]
    # default schedule, then the tuner's usual pick for this batch (8 local
    # rounds, no distance bucket)
    for knobs in ({}, dict(local_rounds=8, bucket_width=-1.0)):
        _say(f"[configs] rgg256 batched job, knobs {knobs}")
        job = cd.DecomposeJob(dgs, params, **knobs)
        stats = job.run()
        for i, (r, st) in enumerate(zip(rows, stats)):
            assert (st.stages, st.levels, st.delta0, st.delta_end, st.num_clusters, st.singletons, st.radius) == \
                (r["stages"], r["levels"], r["delta0"], r["delta_end"], r["num_clusters"], r["singletons"],
                 r["radius"]), i
            assert _digest(job.cluster[i].cpu().numpy()) == r["cluster_sha256"], i
            assert _digest(cd.u64(job.D[i])) == r["D_sha256"], i
    _say("[configs] rgg256 quotients and estimates")
    est = cd.EstimateJob(1, 1, dgs[0].row_ptr.device)
    for i, (r, dg, st) in enumerate(zip(rows, dgs, stats)):
        q = cd.QuotientJob(dg).run(job.cluster[i], job.D[i])
        assert q.k == r["quotient_k"] and q.qm == 2 * r["quotient_edges"], i
        got = dict(center=_digest(q.center.cpu().numpy()), row_ptr=_digest(q.row_ptr.cpu().numpy()),
                   col=_digest(q.col.cpu().numpy()), w=_digest(cd.u64(q.w)))
        assert got == r["quotient_sha256"], i
        assert est.run(q, st.radius) == (r["phi_gc"], r["phi_approx"]), i


@pytest.mark.timeout(900)
def test_serve2000_mix_equals_plain_and_oracle():
    from paper_1506_03265_amd import serve
    counts = json.load(open(os.path.join(HERE, "golden", "serve2000_counts.json")))
    mix = graphgen.serving_mix(counts["requests"], rate=200.0, seed=1)

    def key(r):
        return f"grid{max(256, (r.size // 256) * 256)}" if r.kind == "grid" else f"rmat{r.size}"

    keys = sorted({key(r) for r in mix})
    assert len(keys) == counts["resident_graphs"]
    _say(f"[configs] generating {len(keys)} resident graphs")
    pool = {}
    for k in keys:
        _say(f"[configs] resident graph {k}")
        if k.startswith("grid"):
            s = int(k[4:])
            g = graphgen.grid(s, s, 10000, s)
        else:
            g = graphgen.rmat(int(k[4:]), seed=int(k[4:]))
        pool[k] = cd.cldiam_load_csr(g)
    samples = {s["rid"]: s for s in counts["samples"]}
    assert {s["graph"] for s in samples.values()} == set(keys)
    reqs = [serve.Request(r.rid, r.arrival_s, key(r), counts["tau"], r.rid) for r in mix]
    _say("[configs] serving 2000 requests at 200/s with 4 workers")
    served, wall = serve.serve(reqs, pool, workers=4, hbm_budget_bytes=200 << 30, keep_outputs=set(samples))
    _say(f"[configs] served in {wall:.1f} s; the same requests one at a time")
    plain, _ = serve.serve(reqs, pool, workers=1, hbm_budget_bytes=200 << 30, keep_outputs=set(samples))
    assert [r.rid for r in served] == [r.rid for r in plain] == list(range(len(reqs)))
    for a, b in zip(served, plain):
        assert (a.status, a.stages, a.num_clusters, a.radius, a.phi_gc, a.phi_approx) == \
            (b.status, b.stages, b.num_clusters, b.radius, b.phi_gc, b.phi_approx), a.rid
    for res in (served, plain):
        for rid, s in samples.items():
            r = res[rid]
            assert (r.stages, r.num_clusters, r.radius, r.phi_gc, r.phi_approx) == \
                (s["stages"], s["num_clusters"], s["radius"], s["phi_gc"], s["phi_approx"]), rid
            assert _digest(r.cluster.cpu().numpy()) == s["cluster_sha256"], rid
            assert _digest(cd.u64(r.D)) == s["D_sha256"], rid
