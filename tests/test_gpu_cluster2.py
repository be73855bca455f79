"""GPU parity of CLUSTER2 (Algorithm 2, CLDIAM_VARIANT_CLUSTER2) against the
oracle's decompose_cluster2: cluster ids, D, iterations, 2 R_CL, R_CL, the
per-iteration log, and the quotient graph and estimate built on top, all
exactly equal."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1506_03265_amd as cd

from test_gpu_parity import TINY

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cd.load_library()


def _check(name, g, tau, seed, driver=cd.DRIVER_HOST, estimate=False):
    _say(f"[cluster2] {name} n={g.n} m={g.m} tau={tau} seed={seed} driver={driver}")
    ref = oracle.decompose_cluster2(g, tau, seed)
    dg = cd.cldiam_load_csr(g)
    c, D, st = cd.cldiam_decompose(dg, tau, seed, driver=driver, variant=cd.VARIANT_CLUSTER2)
    got_c, got_D = c.cpu().numpy(), cd.u64(D)
    assert np.array_equal(got_c, ref.cluster), f"{name}: cluster differs at {np.nonzero(got_c != ref.cluster)[0][:10]}"
    assert np.array_equal(got_D, ref.D), f"{name}: D differs"
    assert (st.stages, st.levels, st.delta_end, st.num_clusters, st.singletons, st.radius, st.radius1) == \
        (ref.stages, ref.levels, ref.delta_end, ref.num_clusters, ref.singletons, ref.radius, ref.work["radius1"])
    k = len(st.stage_covered)
    assert (st.stage_uncovered, st.stage_centers, st.stage_covered) == \
        (ref.stage_uncovered[:k], ref.stage_centers[:k], ref.stage_covered[:k])
    if estimate:
        q = cd.cldiam_build_quotient(dg, c, D)
        phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
        qr = oracle.quotient(g, ref)
        er = oracle.estimate(qr, ref)
        assert q.k == qr.k and (phi, approx) == (er.phi_gc, er.phi_approx)
    return st


@pytest.mark.parametrize("name,g", TINY, ids=[n for n, _ in TINY])
@pytest.mark.parametrize("driver", [cd.DRIVER_HOST, cd.DRIVER_PERSISTENT], ids=["host", "persistent"])
def test_cluster2_tiny(name, g, driver):
    _check(name, g, 1, 23, driver=driver)


MEDIUM = [("road384", lambda: graphgen.road_like(384, 2), 2), ("rmat14", lambda: graphgen.rmat(14, seed=4), 1),
          ("grid200", lambda: graphgen.grid(200, 150, 10000, 9), 1), ("rmat17", lambda: graphgen.rmat(17, seed=6), 1)]


@pytest.mark.parametrize("name,make,tau", MEDIUM, ids=[m[0] for m in MEDIUM])
def test_cluster2_medium(name, make, tau):
    st = _check(name, make(), tau, 3, estimate=True)
    assert st.stages >= 10 and st.num_clusters > 1


def test_cluster2_in_a_batch_beside_other_variants():
    graphs = [graphgen.road_like(200, 5), graphgen.rmat(13, seed=3), graphgen.grid(90, 70, 100, 2)]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    params = [(1, 11, 0, cd.VARIANT_CLUSTER2, 0), (1, 12, 0, cd.VARIANT_FIXPOINT, 0), (2, 13, 0, cd.VARIANT_STEPS, 0)]
    clusters, Ds, stats = cd.cldiam_decompose_batch(dgs, params)
    refs = [oracle.decompose_cluster2(graphs[0], 1, 11), oracle.decompose(graphs[1], 1, 12),
            oracle.decompose_steps(graphs[2], 2, 13)]
    for c, D, ref in zip(clusters, Ds, refs):
        assert np.array_equal(c.cpu().numpy(), ref.cluster)
        assert np.array_equal(cd.u64(D), ref.D)
