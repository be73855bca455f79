"""GPU parity of the literal step-synchronous variant (CLDIAM_VARIANT_STEPS):
synchronous Delta-growing steps with the strict distance tie rule, the
per-step half-coverage stop, Delta doubled one step at a time and the
optional step cap.  Exact equality with the oracle's decompose_steps:
clusters, distance bounds, stages, PartialGrowth calls, Delta, and the round
and work counters (steps, messages, node updates)."""
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


def _check(name, g, tau, seed, delta0=0, step_cap=0, driver=cd.DRIVER_HOST):
    _say(f"[steps] {name} n={g.n} m={g.m} tau={tau} seed={seed} delta0={delta0} cap={step_cap} driver={driver}")
    ref = oracle.decompose_steps(g, tau, seed, delta0=delta0, step_cap=step_cap)
    dg = cd.cldiam_load_csr(g)
    c, D, st = cd.cldiam_decompose(dg, tau, seed, delta0=delta0, driver=driver, variant=cd.VARIANT_STEPS,
                                   step_cap=step_cap)
    got_c, got_D = c.cpu().numpy(), cd.u64(D)
    assert np.array_equal(got_c, ref.cluster), f"{name}: cluster differs at {np.nonzero(got_c != ref.cluster)[0][:10]}"
    assert np.array_equal(got_D, ref.D), f"{name}: D differs"
    assert (st.stages, st.levels, st.delta_end, st.num_clusters, st.singletons, st.radius) == \
        (ref.stages, ref.levels, ref.delta_end, ref.num_clusters, ref.singletons, ref.radius)
    assert st.stage_covered == ref.stage_covered[:len(st.stage_covered)]
    assert (st.rounds, st.messages, st.updates) == \
        (ref.work["rounds"], ref.work["messages"], ref.work["updates"]), name
    return st


@pytest.mark.parametrize("name,g", TINY, ids=[n for n, _ in TINY])
@pytest.mark.parametrize("driver", [cd.DRIVER_HOST, cd.DRIVER_PERSISTENT], ids=["host", "persistent"])
def test_steps_tiny(name, g, driver):
    _check(name, g, 1, 17, driver=driver)


@pytest.mark.parametrize("cap", [1, 3, 8])
def test_steps_with_cap(cap):
    for name, g in TINY[:8]:
        _check(name, g, 1, 5, step_cap=cap)


MEDIUM = [("road384", lambda: graphgen.road_like(384, 2), 2), ("rmat14", lambda: graphgen.rmat(14, seed=4), 1),
          ("grid200", lambda: graphgen.grid(200, 150, 10000, 9), 1), ("rmat16", lambda: graphgen.rmat(16, seed=6), 1)]


@pytest.mark.parametrize("name,make,tau", MEDIUM, ids=[m[0] for m in MEDIUM])
def test_steps_medium(name, make, tau):
    st = _check(name, make(), tau, 3)
    assert st.rounds > st.levels >= 1


def test_steps_medium_with_cap_and_small_delta():
    g = graphgen.road_like(256, 4)
    _check("road256-cap", g, 1, 8, delta0=1, step_cap=4)


def test_steps_in_a_batch_beside_fixpoint_graphs():
    """Both variants in one device job: each graph equals its own oracle."""
    graphs = [graphgen.road_like(200, 5), graphgen.rmat(13, seed=3), graphgen.grid(90, 70, 100, 2)]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    params = [(1, 11, 0, cd.VARIANT_STEPS, 0), (1, 12, 0, cd.VARIANT_FIXPOINT, 0), (2, 13, 0, cd.VARIANT_STEPS, 3)]
    clusters, Ds, stats = cd.cldiam_decompose_batch(dgs, params)
    for g, c, D, st, (tau, seed, d0, var, cap) in zip(graphs, clusters, Ds, stats, params):
        ref = oracle.decompose_steps(g, tau, seed, step_cap=cap) if var else oracle.decompose(g, tau, seed)
        assert np.array_equal(c.cpu().numpy(), ref.cluster)
        assert np.array_equal(cd.u64(D), ref.D)
        if var:
            assert (st.rounds, st.messages, st.updates) == \
                (ref.work["rounds"], ref.work["messages"], ref.work["updates"])
