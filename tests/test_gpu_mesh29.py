"""One GPU's part of the billion-edge row (Section 5, R-MAT(29) of Table 3):
the 16384 x 32768 mesh with 1% diagonals (2^29 nodes, 2,158M arcs, past the
reach of 32-bit row offsets) through the whole path - ingest, decomposition,
quotient graph, estimate - against the oracle, which takes 64-bit row offsets
too: digests of all 2^29 cluster ids and distance bounds, of the quotient
graph's centers and symmetric CSR, the per-stage counts and the estimate.
Expected values were written by tests/golden/make_workload_counts.py
(workload mesh29), which calls only the oracle."""
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


@pytest.mark.timeout(900)
def test_mesh29_past_2_31_arcs_equals_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    counts = json.load(open(os.path.join(HERE, "golden", "mesh29_counts.json")))
    torch.cuda.empty_cache()   # device memory cached by earlier tests
    _say("[mesh29] generating 16384 x 32768 mesh")
    g = graphgen.mesh29(1)
    assert (g.n, g.m) == (counts["n"], counts["m_arcs"]) and g.m > 2**31
    _say("[mesh29] ingest")
    dg = cd.cldiam_load_csr(g)
    del g
    torch.cuda.empty_cache()
    _say("[mesh29] decompose")
    cluster, D, st = cd.cldiam_decompose(dg, counts["tau"], counts["seed"])
    assert (st.stages, st.levels, st.delta0, st.delta_end, st.num_clusters, st.singletons, st.radius) == \
        (counts["stages"], counts["levels"], counts["delta0"], counts["delta_end"], counts["num_clusters"],
         counts["singletons"], counts["radius"])
    assert st.stage_uncovered == counts["stage_uncovered"][:len(st.stage_uncovered)]
    assert st.stage_covered == counts["stage_covered"][:len(st.stage_covered)]
    _say("[mesh29] digests of cluster ids and distance bounds")
    assert _digest(cluster.cpu().numpy()) == counts["cluster_sha256"]
    assert _digest(cd.u64(D)) == counts["D_sha256"]
    _say("[mesh29] quotient")
    q = cd.cldiam_build_quotient(dg, cluster, D)
    assert q.k == counts["quotient_k"] and q.qm == 2 * counts["quotient_edges"]
    got = dict(center=_digest(q.center.cpu().numpy()), row_ptr=_digest(q.row_ptr.cpu().numpy()),
               col=_digest(q.col.cpu().numpy()), w=_digest(cd.u64(q.w)))
    assert got == counts["quotient_sha256"]
    phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
    assert (phi, approx) == (counts["phi_gc"], counts["phi_approx"])
