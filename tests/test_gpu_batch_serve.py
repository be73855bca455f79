"""GPU tests of the systems layers: batched jobs, schedule knobs, the tuner
and the serving loop.  Every result is compared exactly: with the oracle, and
between runs that differ only in scheduling (alone vs in a mix, one job vs one
job per graph, different knob settings)."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1506_03265_amd as cd

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cd.load_library()


@pytest.mark.parametrize("local_rounds,grid_blocks,driver", [(0, 0, 1), (1, 7, 1), (7, 64, 1), (16, 300, 1),
                                                             (3, 33, 2), (0, 256, 2)])
def test_schedule_knobs_do_not_change_results(local_rounds, grid_blocks, driver):
    g = graphgen.road_like(400, 6)
    _say(f"[systems] knobs rounds={local_rounds} blocks={grid_blocks} driver={driver}")
    ref = oracle.decompose(g, 2, 9)
    dg = cd.cldiam_load_csr(g)
    c, D, st = cd.cldiam_decompose(dg, 2, 9, driver=driver, local_rounds=local_rounds, grid_blocks=grid_blocks)
    assert np.array_equal(c.cpu().numpy(), ref.cluster)
    assert np.array_equal(cd.u64(D), ref.D)
    assert (st.stages, st.levels, st.delta_end) == (ref.stages, ref.levels, ref.delta_end)


@pytest.mark.parametrize("bucket_width,row_shift,variant", [(0.0, 0, 0), (0.0, 1, 0), (0.0, 31, 0), (0.0, -1, 0),
                                                            (-1.0, 0, 0), (4.0, 3, 0), (1.0, 12, 0), (0.0, 1, 2),
                                                            (-1.0, 2, 2)])
def test_bucket_knobs_on_long_rows(bucket_width, row_shift, variant):
    """Distance buckets (all nodes, and the narrower one of long rows) only
    reorder relaxations: an R-MAT graph with hub rows of thousands of arcs
    gives the oracle's outputs at every width, for CLUSTER and CLUSTER2."""
    g = graphgen.rmat(14, seed=3)
    _say(f"[systems] buckets width={bucket_width} row_shift={row_shift} variant={variant}")
    ref = oracle.decompose_cluster2(g, 1, 4) if variant == cd.VARIANT_CLUSTER2 else oracle.decompose(g, 1, 4)
    dg = cd.cldiam_load_csr(g)
    c, D, st = cd.cldiam_decompose(dg, 1, 4, variant=variant, bucket_width=bucket_width, row_bucket_shift=row_shift)
    assert np.array_equal(c.cpu().numpy(), ref.cluster)
    assert np.array_equal(cd.u64(D), ref.D)
    assert (st.stages, st.levels, st.delta_end) == (ref.stages, ref.levels, ref.delta_end)


@pytest.mark.parametrize("chunk_factor,grid_blocks,driver", [(1, 0, 1), (2, 7, 1), (7, 64, 1), (64, 300, 1),
                                                             (5, 33, 2)])
def test_chunk_factor_on_long_rows(chunk_factor, grid_blocks, driver):
    """Growth chunks handed out on demand (any number per workgroup, either
    driver) leave the R-MAT outputs equal to the oracle's."""
    g = graphgen.rmat(14, seed=5)
    _say(f"[systems] chunks factor={chunk_factor} blocks={grid_blocks} driver={driver}")
    ref = oracle.decompose(g, 2, 6)
    dg = cd.cldiam_load_csr(g)
    c, D, st = cd.cldiam_decompose(dg, 2, 6, driver=driver, grid_blocks=grid_blocks, chunk_factor=chunk_factor)
    assert np.array_equal(c.cpu().numpy(), ref.cluster)
    assert np.array_equal(cd.u64(D), ref.D)
    assert (st.stages, st.levels, st.delta_end) == (ref.stages, ref.levels, ref.delta_end)


@pytest.mark.parametrize("wave_row_min,group_row_min,local_queue", [(0, 0, 0), (1, 1, 0), (4, 64, 0), (8, 1024, 64),
                                                                    (128, 65536, 512), (2000, 2000, 4096),
                                                                    (1 << 20, 1 << 30, 0)])
def test_row_tiers_and_queue_tile(wave_row_min, group_row_min, local_queue):
    """Threads per row (one thread, a wave or the whole workgroup, by degree)
    and the local queue tile only change which threads relax an arc and when:
    an R-MAT graph with hub rows, a road-like mesh and a batch of both give the
    oracle's outputs for every setting, for CLUSTER and CLUSTER2, and the
    literal steps (which use the same tiers) give the oracle's counters."""
    knobs = dict(wave_row_min=wave_row_min, group_row_min=group_row_min, local_queue=local_queue)
    _say(f"[systems] row tiers {knobs}")
    graphs = [graphgen.rmat(13, seed=8), graphgen.road_like(160, 2)]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    for g, dg in zip(graphs, dgs):
        for variant in (cd.VARIANT_FIXPOINT, cd.VARIANT_CLUSTER2):
            ref = oracle.decompose_cluster2(g, 1, 5) if variant else oracle.decompose(g, 1, 5)
            c, D, st = cd.cldiam_decompose(dg, 1, 5, variant=variant, **knobs)
            assert np.array_equal(c.cpu().numpy(), ref.cluster), variant
            assert np.array_equal(cd.u64(D), ref.D), variant
        ref = oracle.decompose_steps(g, 1, 5)
        c, D, st = cd.cldiam_decompose(dg, 1, 5, variant=cd.VARIANT_STEPS, **knobs)
        assert np.array_equal(c.cpu().numpy(), ref.cluster)
        assert (st.rounds, st.messages, st.updates) == \
            (ref.work["rounds"], ref.work["messages"], ref.work["updates"])
    clusters, Ds, stats = cd.cldiam_decompose_batch(dgs, [(2, 11, 0), (2, 12, 0)], **knobs)
    for g, c, D, (tau, seed) in zip(graphs, clusters, Ds, [(2, 11), (2, 12)]):
        ref = oracle.decompose(g, tau, seed)
        assert np.array_equal(c.cpu().numpy(), ref.cluster) and np.array_equal(cd.u64(D), ref.D)


@pytest.mark.parametrize("scale,gseed", [(10, 1), (12, 2), (14, 3), (16, 1)])
def test_rmat_family_under_two_schedules(scale, gseed):
    """R-MAT graphs of several sizes and seeds, CLUSTER and CLUSTER2, under the
    default schedule and under on-demand chunks on an odd grid: the oracle's
    outputs every time."""
    g = graphgen.rmat(scale, seed=gseed)
    dg = cd.cldiam_load_csr(g)
    _say(f"[systems] rmat{scale} seed {gseed} schedules")
    for tau, seed in ((1, 7), (4, 3)):
        for variant in (cd.VARIANT_FIXPOINT, cd.VARIANT_CLUSTER2):
            ref = oracle.decompose_cluster2(g, tau, seed) if variant else oracle.decompose(g, tau, seed)
            for cf, blocks in ((0, 0), (3, 97)):
                c, D, st = cd.cldiam_decompose(dg, tau, seed, variant=variant, chunk_factor=cf, grid_blocks=blocks)
                assert np.array_equal(c.cpu().numpy(), ref.cluster), (tau, seed, variant, cf)
                assert np.array_equal(cd.u64(D), ref.D), (tau, seed, variant, cf)


def test_batch_of_geometric_graphs_matches_oracle():
    sizes = [1000, 1500, 2500, 4000, 7000, 12000, 20000, 30000] * 3
    graphs = [graphgen.rgg(n, i, 5) for i, n in enumerate(sizes)]
    params = [(1, (i << 32) | 5, 0) for i in range(len(graphs))]
    _say(f"[systems] batch of {len(graphs)} geometric graphs")
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    clusters, Ds, stats = cd.cldiam_decompose_batch(dgs, params)
    for g, c, D, st, (tau, seed, d0) in zip(graphs, clusters, Ds, stats, params):
        ref = oracle.decompose(g, tau, seed, delta0=d0)
        assert np.array_equal(c.cpu().numpy(), ref.cluster)
        assert np.array_equal(cd.u64(D), ref.D)
        assert st.num_clusters == ref.num_clusters and st.radius == ref.radius


def test_tuner_returns_a_candidate_and_checks_equality(tmp_path, monkeypatch):
    from paper_1506_03265_amd import tune
    monkeypatch.setenv("CLDIAM_TUNE_CACHE", str(tmp_path / "tune.json"))
    graphs = [graphgen.rgg(n, i, 2) for i, n in enumerate([3000, 9000, 500])]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    params = [(1, i + 1, 0) for i in range(3)]
    best = tune.tune_batch(dgs, params, reps=1)
    assert best in tune.CANDIDATES
    assert tune.tune_batch(dgs, params, reps=1) == best   # cached
    assert (tmp_path / "tune.json").exists()


def test_served_results_equal_alone_results():
    """Continuous batching: each request's cluster ids and distance bounds are
    the same when it runs in the mix and when it runs alone (tolerance 0)."""
    from paper_1506_03265_amd import serve
    pool_graphs = {"grid96": graphgen.grid(96, 96, 10000, 96), "grid200": graphgen.grid(200, 200, 10000, 200),
                   "rmat12": graphgen.rmat(12, seed=12), "rmat14": graphgen.rmat(14, seed=14),
                   "road256": graphgen.road_like(256, 3)}
    pool = {k: cd.cldiam_load_csr(g) for k, g in pool_graphs.items()}
    keys = sorted(pool)
    rng = np.random.default_rng(11)
    reqs = [serve.Request(i, float(t), keys[int(rng.integers(0, len(keys)))], 1, 1000 + i)
            for i, t in enumerate(np.cumsum(rng.exponential(0.002, size=40)))]
    _say("[systems] serving 40 requests with 4 workers")
    mixed, _ = serve.serve(reqs, pool, workers=4, keep_outputs=True)
    _say("[systems] the same requests one at a time")
    alone, _ = serve.serve(reqs, pool, workers=1, keep_outputs=True)
    assert [r.rid for r in mixed] == [r.rid for r in alone] == list(range(40))
    for a, b, req in zip(mixed, alone, reqs):
        assert bool((a.cluster == b.cluster).all()) and bool((a.D == b.D).all())
        assert (a.num_clusters, a.radius, a.phi_approx) == (b.num_clusters, b.radius, b.phi_approx)
    # and against the oracle for a sample of requests
    for req, res in list(zip(reqs, mixed))[:6]:
        g = pool_graphs[req.graph]
        ref = oracle.decompose(g, req.tau, req.seed)
        est = oracle.estimate(oracle.quotient(g, ref), ref)
        assert np.array_equal(res.cluster.cpu().numpy(), ref.cluster)
        assert res.phi_approx == est.phi_approx
    assert all(r.latency_s >= 0 for r in mixed)


def test_pinned_readback_buffers_stay_bounded():
    """Every request of the stream pool runs on a fresh host thread; the
    pinned readback buffers are pooled, so 64 served requests with at most 4
    in flight leave at most 4 more buffers behind (none are leaked per thread)."""
    from paper_1506_03265_amd import serve
    lib = cd.load_library()
    g = graphgen.grid(64, 64, 1000, 5)
    pool = {"g": cd.cldiam_load_csr(g)}
    cd.cldiam_decompose(pool["g"], 1, 1)   # the pool holds at least one buffer from here on
    before = lib.cldiam_pinned_host_bytes()
    reqs = [serve.Request(i, 0.0, "g", 1, i) for i in range(64)]
    _say("[systems] 64 requests on fresh threads, pinned pool size")
    res, _ = serve.serve(reqs, pool, workers=4)
    assert len(res) == 64
    after = lib.cldiam_pinned_host_bytes()
    assert after - before <= 4 * 4096, (before, after)


def test_serving_respects_a_tiny_budget():
    """With a budget below two footprints, requests run one at a time and
    still all complete with the same results."""
    from paper_1506_03265_amd import serve
    g = graphgen.grid(128, 128, 1000, 3)
    pool = {"g": cd.cldiam_load_csr(g)}
    fp = serve.footprint_bytes(pool["g"])
    reqs = [serve.Request(i, 0.0, "g", 1, i) for i in range(6)]
    res, _ = serve.serve(reqs, pool, workers=4, hbm_budget_bytes=fp + fp // 2)
    starts = sorted((r.start_s, r.done_s) for r in res)
    assert all(s1 >= d0 - 1e-6 for (_, d0), (s1, _) in zip(starts, starts[1:]))
    for r in res:
        ref = oracle.decompose(g, 1, r.rid)
        assert r.num_clusters == ref.num_clusters and r.radius == ref.radius


def test_server_matches_oracle_with_slot_and_range_reuse():
    """In-engine continuous batching: requests submitted while others run,
    more requests than slots and node ranges, finished slots and ranges handed
    to queued ones; each result equals the oracle's exactly."""
    sizes = [800, 5000, 1200, 9000, 300, 2500, 7000, 4000, 600, 9000, 1, 2]
    graphs = [graphgen.rgg(n, i, 3) if n > 2 else graphgen.csr_from_edges_np(n, [0] * (n - 1), [1] * (n - 1), [5] * (n - 1))
              for i, n in enumerate(sizes)]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    srv = cd.Server(12000, max_graphs=3, local_rounds=2)
    _say(f"[systems] server: {len(graphs)} requests, 3 slots, 12000 nodes")
    for i in range(5):
        srv.submit(dgs[i], 1 + i % 2, 100 + i, i)
    got, steps = {}, 0
    while len(got) < len(graphs):
        srv.step(3)
        for tag, st, g, c, D in srv.poll():
            got[tag] = (st, c.cpu().numpy(), cd.u64(D))
        steps += 1
        if steps == 4:
            for i in range(5, len(graphs)):
                srv.submit(dgs[i], 1 + i % 2, 100 + i, i)
        assert steps < 200000
    srv.close()
    for i, g in enumerate(graphs):
        st, c, D = got[i]
        ref = oracle.decompose(g, 1 + i % 2, 100 + i)
        assert st.status == cd.CLDIAM_OK
        assert np.array_equal(c, ref.cluster), i
        assert np.array_equal(D, ref.D), i
        assert (st.stages, st.levels, st.num_clusters, st.radius) == (ref.stages, ref.levels, ref.num_clusters,
                                                                       ref.radius)


def test_server_isolates_a_failing_request():
    """A request whose Delta overflows finishes alone with EOVERFLOW in its
    statistics; the requests beside it are unaffected."""
    n = 128
    bad = graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [2**31] * (n - 1))
    good = [graphgen.grid(40, 40, 1000, 4), graphgen.rmat(11, seed=2)]
    srv = cd.Server(8000, max_graphs=4)
    srv.submit(cd.cldiam_load_csr(good[0]), 1, 7, 0)
    srv.submit(cd.cldiam_load_csr(bad), 1, 1, 1, delta0=2**31)
    srv.submit(cd.cldiam_load_csr(good[1]), 2, 9, 2)
    with pytest.raises(cd.CldiamError):
        srv.submit(cd.cldiam_load_csr(graphgen.grid(100, 100, 10, 1)), 1, 1, 3)   # above the node capacity
    got, steps = {}, 0
    while len(got) < 3:
        srv.step(4)
        for tag, st, g, c, D in srv.poll():
            got[tag] = (st, c.cpu().numpy())
        steps += 1
        assert steps < 100000
    srv.close()
    assert got[1][0].status == cd.CLDIAM_EOVERFLOW
    for tag, g, tau, seed in ((0, good[0], 1, 7), (2, good[1], 2, 9)):
        ref = oracle.decompose(g, tau, seed)
        assert got[tag][0].status == cd.CLDIAM_OK and np.array_equal(got[tag][1], ref.cluster)


def test_engine_serving_equals_alone_results():
    """serve_engine: each request's outputs equal those of the same request run
    alone through the plain sequential loop."""
    from paper_1506_03265_amd import serve
    pool_graphs = {"grid96": graphgen.grid(96, 96, 10000, 96), "rmat12": graphgen.rmat(12, seed=12),
                   "rmat14": graphgen.rmat(14, seed=14), "road256": graphgen.road_like(256, 3)}
    pool = {k: cd.cldiam_load_csr(g) for k, g in pool_graphs.items()}
    keys = sorted(pool)
    rng = np.random.default_rng(5)
    reqs = [serve.Request(i, float(t), keys[int(rng.integers(0, len(keys)))], 1 + i % 2, 2000 + i)
            for i, t in enumerate(np.cumsum(rng.exponential(0.001, size=30)))]
    _say("[systems] engine serving of 30 requests")
    eng, _ = serve.serve_engine(reqs, pool, max_graphs=8, keep_outputs=True)
    split, _ = serve.serve_engine(reqs, pool, max_graphs=4, keep_outputs=True, split_nodes=20000)
    alone, _ = serve.serve(reqs, pool, workers=1, keep_outputs=True)
    assert [r.rid for r in eng] == [r.rid for r in split] == list(range(30))
    for a, b, c in zip(eng, alone, split):
        assert bool((c.cluster == b.cluster).all()) and bool((c.D == b.D).all()) and c.phi_approx == b.phi_approx
        assert a.status == 0
        assert bool((a.cluster == b.cluster).all()) and bool((a.D == b.D).all())
        assert (a.num_clusters, a.radius, a.phi_gc, a.phi_approx) == (b.num_clusters, b.radius, b.phi_gc, b.phi_approx)
        assert a.latency_s >= 0


def _pull_families():
    rng = np.random.default_rng(31)
    fams = [("grid_small", graphgen.grid_small()), ("road200", graphgen.road_like(200, 7)),
            ("rmat12", graphgen.rmat(12, seed=4)), ("rmat15", graphgen.rmat(15, seed=6)),
            ("bimodal128", graphgen.bimodal_mesh(128, 3))]
    for i in range(3):
        n = int(rng.integers(150, 400))
        fams.append((f"er{i}", graphgen.random_small(rng, n, 0.03, int(rng.choice([2, 100, 10000])),
                                                    connected=bool(i % 2))))
    n = 300
    fams.append(("star", graphgen.csr_from_edges_np(n, [0] * (n - 1), range(1, n), list(range(1, n)))))
    fams.append(("twocomp", graphgen.csr_from_edges_np(200, list(range(99)) + list(range(100, 199)),
                                                       list(range(1, 100)) + list(range(101, 200)), [3] * 198)))
    return fams


PULL_FAMILIES = _pull_families()


@pytest.mark.parametrize("pull_mode", [cd.PULL_NEVER, cd.PULL_ALWAYS, cd.PULL_AUTO], ids=["never", "always", "auto"])
@pytest.mark.parametrize("name,g", PULL_FAMILIES, ids=[f for f, _ in PULL_FAMILIES])
def test_pull_mode_equals_oracle(name, g, pull_mode):
    """New levels and stages grown by pulling from the unreached side (the
    unreached nodes take their best offer from their neighbours, and NEXT is
    computed from their side) give the oracle's outputs on every family, for
    several tau, seeds and initial Delta (small ones force many levels), and
    CLUSTER2 (which never pulls) is unaffected by the knob."""
    dg = cd.cldiam_load_csr(g)
    _say(f"[systems] pull mode {pull_mode} on {name} n={g.n}")
    for tau, seed, d0 in ((1, 3, 0), (2, 8, 1), (4, 5, 0)):
        ref = oracle.decompose(g, tau, seed, delta0=d0)
        c, D, st = cd.cldiam_decompose(dg, tau, seed, delta0=d0, pull_mode=pull_mode)
        assert np.array_equal(c.cpu().numpy(), ref.cluster), (tau, seed, d0)
        assert np.array_equal(cd.u64(D), ref.D), (tau, seed, d0)
        assert (st.stages, st.levels, st.delta_end, st.num_clusters, st.radius) == \
            (ref.stages, ref.levels, ref.delta_end, ref.num_clusters, ref.radius), (tau, seed, d0)
    ref = oracle.decompose_cluster2(g, 1, 2)
    c, D, st = cd.cldiam_decompose(dg, 1, 2, variant=cd.VARIANT_CLUSTER2, pull_mode=pull_mode)
    assert np.array_equal(c.cpu().numpy(), ref.cluster) and np.array_equal(cd.u64(D), ref.D)


def test_pull_mode_in_a_batch_and_a_server():
    """A batch mixing graphs that pull and graphs that push, and the same
    graphs served through the continuous-batching server: the oracle's
    outputs for each."""
    graphs = [graphgen.rmat(13, seed=9), graphgen.road_like(150, 4), graphgen.rmat(11, seed=3)]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    params = [(1, 21, 0), (2, 22, 1), (1, 23, 0)]
    for pm in (cd.PULL_ALWAYS, cd.PULL_AUTO):
        _say(f"[systems] pull mode {pm} in a batch")
        clusters, Ds, stats = cd.cldiam_decompose_batch(dgs, params, pull_mode=pm)
        for g, c, D, (tau, seed, d0) in zip(graphs, clusters, Ds, params):
            ref = oracle.decompose(g, tau, seed, delta0=d0)
            assert np.array_equal(c.cpu().numpy(), ref.cluster) and np.array_equal(cd.u64(D), ref.D)
    srv = cd.Server(sum(g.n for g in graphs), max_graphs=2, pull_mode=cd.PULL_ALWAYS)
    for i, (dg, (tau, seed, d0)) in enumerate(zip(dgs, params)):
        srv.submit(dg, tau, seed, i, delta0=d0)
    done = {}
    for _ in range(10000):
        act, queued = srv.step(8)
        for tag, st, _g, cl, D in srv.poll():
            done[tag] = (cl, D)
        if len(done) == len(graphs):
            break
    assert len(done) == len(graphs)
    for i, (g, (tau, seed, d0)) in enumerate(zip(graphs, params)):
        ref = oracle.decompose(g, tau, seed, delta0=d0)
        assert np.array_equal(done[i][0].cpu().numpy(), ref.cluster) and np.array_equal(cd.u64(done[i][1]), ref.D)
