"""Full-size parity on the benchmark workloads (road-like 4096x4096 mesh,
16.8M nodes, 64.1M arcs; R-MAT scale 24, 8.9M nodes, 521M arcs; tau = 4,
seed 1), in the launch configuration the benchmark times.  Expected values were written by the oracle
(tests/golden/make_workload_counts.py): per-node outputs are compared through
SHA-256 digests of the oracle's arrays, plus stage counts, the quotient graph
(digests of its centers and of its symmetric CSR: row offsets, columns,
weights), the estimate, and the Delta-stepping competitor's distances."""
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


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _check_quotient(q, ref):
    """The quotient graph equals the oracle's: k, arc count and the digests of
    its centers (int32), row offsets (int64), columns (int32), weights (u64)."""
    assert q.k == ref["quotient_k"] and q.qm == 2 * ref["quotient_edges"]
    got = dict(center=_digest(q.center.cpu().numpy()), row_ptr=_digest(q.row_ptr.cpu().numpy()),
               col=_digest(q.col.cpu().numpy()), w=_digest(cd.u64(q.w)))
    assert got == ref["quotient_sha256"]


@pytest.fixture(scope="module")
def road():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    counts = json.load(open(os.path.join(HERE, "golden", "road4096_counts.json")))
    print("[fullsize] generating road4096", file=sys.stderr, flush=True)
    g = graphgen.road_like(4096, 1)
    assert (g.n, g.m) == (counts["n"], counts["m_arcs"])
    return g, counts, cd.cldiam_load_csr(g)


@pytest.mark.parametrize("driver", [cd.DRIVER_AUTO, cd.DRIVER_HOST], ids=["auto", "host"])
def test_road4096_decompose_quotient_estimate(road, driver):
    g, counts, dg = road
    print(f"[fullsize] decompose driver={driver}", file=sys.stderr, flush=True)
    cluster, D, st = cd.cldiam_decompose(dg, counts["tau"], counts["seed"], driver=driver)
    assert (st.stages, st.levels, st.delta0, st.delta_end) == \
        (counts["stages"], counts["levels"], counts["delta0"], counts["delta_end"])
    assert (st.num_clusters, st.singletons, st.radius) == \
        (counts["num_clusters"], counts["singletons"], counts["radius"])
    assert st.stage_uncovered == counts["stage_uncovered"]
    assert st.stage_centers == counts["stage_centers"]
    assert st.stage_covered == counts["stage_covered"]
    assert st.stage_delta == counts["stage_delta"]
    assert _digest(cluster.cpu().numpy()) == counts["cluster_sha256"]
    assert _digest(cd.u64(D)) == counts["D_sha256"]
    q = cd.cldiam_build_quotient(dg, cluster, D)
    _check_quotient(q, counts)
    phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
    assert (phi, approx) == (counts["phi_gc"], counts["phi_approx"])


def test_road4096_pulling_from_the_first_stage(road):
    """Every level and stage grown by pulling from the unreached side (the
    mesh never switches by itself): the same digests."""
    g, counts, dg = road
    print("[fullsize] road4096 pull mode always", file=sys.stderr, flush=True)
    cluster, D, st = cd.cldiam_decompose(dg, counts["tau"], counts["seed"], pull_mode=cd.PULL_ALWAYS)
    assert (st.stages, st.levels, st.delta_end, st.num_clusters, st.radius) == \
        (counts["stages"], counts["levels"], counts["delta_end"], counts["num_clusters"], counts["radius"])
    assert _digest(cluster.cpu().numpy()) == counts["cluster_sha256"]
    assert _digest(cd.u64(D)) == counts["D_sha256"]


def test_road4096_sssp_equals_dijkstra(road):
    """The competitor's Delta-stepping distances from the source rule, with
    the default bucket width and with the benchmark's best, against the
    oracle's Dijkstra (digest of all 16.8M distances)."""
    g, counts, dg = road
    ref = counts["sssp"]
    for bd in (0, 16 * 5000):
        print(f"[fullsize] sssp src={ref['source']} bucket={bd}", file=sys.stderr, flush=True)
        dist, mx = cd.cldiam_sssp_delta_stepping(dg, ref["source"], bd)
        assert mx == ref["max_dist"]
        assert _digest(cd.u32(dist)) == ref["dist_sha256"]


def test_road4096_invariants_on_samples(road):
    """Properties that hold at any size, on sampled clusters: a partition
    whose centers are their own cluster, and D bounded by the stage radii."""
    g, counts, dg = road
    cluster, D, st = cd.cldiam_decompose(dg, counts["tau"], counts["seed"])
    c = cluster.cpu().numpy()
    d = cd.u64(D)
    centers = np.unique(c)
    assert len(centers) == st.num_clusters
    assert np.all(c[centers] == centers)
    assert np.all(d[centers] == 0)
    assert int(d.max()) == st.radius <= sum(st.stage_delta)


@pytest.mark.parametrize("variant", ["cluster2", "steps"])
def test_road4096_variants(road, variant):
    """CLUSTER2 and the literal step-synchronous variant at full size."""
    g, counts, dg = road
    ref = counts[variant]
    var = cd.VARIANT_CLUSTER2 if variant == "cluster2" else cd.VARIANT_STEPS
    print(f"[fullsize] {variant}", file=sys.stderr, flush=True)
    cluster, D, st = cd.cldiam_decompose(dg, counts["tau"], counts["seed"], variant=var)
    assert (st.stages, st.delta_end, st.num_clusters, st.radius) == \
        (ref["stages"], ref["delta_end"], ref["num_clusters"], ref["radius"])
    if variant == "cluster2":
        assert st.radius1 == ref["radius1"]
    else:
        assert (st.levels, st.rounds, st.messages, st.updates) == \
            (ref["levels"], ref["rounds"], ref["messages"], ref["updates"])
    assert _digest(cluster.cpu().numpy()) == ref["cluster_sha256"]
    assert _digest(cd.u64(D)) == ref["D_sha256"]
    q = cd.cldiam_build_quotient(dg, cluster, D)
    _check_quotient(q, ref)
    phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
    assert (phi, approx) == (ref["phi_gc"], ref["phi_approx"])


def _check_packed_rows(dg):
    """Every row of the packed arcs is ascending by (w, col) and holds the
    same arcs as the input row (per-row sums of col, w and col ^ w), checked
    on the device for all 521M arcs."""
    import torch
    n, m = dg.n, dg.m
    arcs = dg.arcs[:m]
    rp = dg.row_ptr
    deg = rp[1:] - rp[:-1]
    start = torch.zeros(m, dtype=torch.bool, device=arcs.device)
    start[rp[:-1][deg > 0]] = True
    assert bool(((arcs[1:] >= arcs[:-1]) | start[1:]).all()), "a packed row is out of order"
    row = torch.repeat_interleave(torch.arange(n, device=arcs.device), deg)
    col, w = arcs & 0xFFFFFFFF, arcs >> 32
    col0, w0 = dg.col.long(), dg.w.long() & 0xFFFFFFFF
    for a, b in ((col, col0), (w, w0), (col ^ w, col0 ^ w0)):
        sa = torch.zeros(n, dtype=torch.int64, device=arcs.device).index_add_(0, row, a)
        sb = torch.zeros(n, dtype=torch.int64, device=arcs.device).index_add_(0, row, b)
        assert bool((sa == sb).all()), "a packed row lost or gained arcs"


@pytest.mark.timeout(900)
def test_rmat24_decompose_quotient_estimate():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    counts = json.load(open(os.path.join(HERE, "golden", "rmat24_counts.json")))
    print("[fullsize] generating rmat24", file=sys.stderr, flush=True)
    g = graphgen.rmat(24, seed=1)
    assert (g.n, g.m) == (counts["n"], counts["m_arcs"])
    dg = cd.cldiam_load_csr(g)
    del g
    print("[fullsize] rmat24 ingest order", file=sys.stderr, flush=True)
    _check_packed_rows(dg)
    print("[fullsize] rmat24 decompose", file=sys.stderr, flush=True)
    cluster, D, st = cd.cldiam_decompose(dg, counts["tau"], counts["seed"])
    assert (st.stages, st.levels, st.delta0, st.delta_end) == \
        (counts["stages"], counts["levels"], counts["delta0"], counts["delta_end"])
    assert (st.num_clusters, st.singletons, st.radius) == \
        (counts["num_clusters"], counts["singletons"], counts["radius"])
    assert st.stage_covered == counts["stage_covered"]
    assert _digest(cluster.cpu().numpy()) == counts["cluster_sha256"]
    assert _digest(cd.u64(D)) == counts["D_sha256"]
    print("[fullsize] rmat24 quotient", file=sys.stderr, flush=True)
    q = cd.cldiam_build_quotient(dg, cluster, D)
    _check_quotient(q, counts)
    phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
    assert (phi, approx) == (counts["phi_gc"], counts["phi_approx"])
